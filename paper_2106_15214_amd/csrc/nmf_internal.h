// Internal declarations shared by the host library and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nmf {

// Classes of beta with specialised element-wise terms (the general class uses
// exp2/log2 for Lambda^(beta-2)).
// BC_B2G: beta = 2 with the Gram-form denominators of Table 2 (Q H~^T = W~ (H~ H~^T)
// and chi_2^T Q = (chi_2^T W~) H~): the passes contract P = V only.
enum BetaClass { BC_GEN = 0, BC_B2 = 1, BC_B1 = 2, BC_B0 = 3, BC_B05 = 4, BC_B15 = 5, BC_B2G = 6 };

// What a pass over V accumulates.
enum Kind {
  KIND_UPDATE = 0,  // numerator (P) and denominator (Q) contractions
  KIND_GRAD = 1,    // gradient term E = Lambda^(beta-2) (Lambda - V) only
  KIND_OBJ = 2      // objective terms only (no contraction)
};

constexpr int kBlock = 256;      // threads per workgroup (4 wave64)
constexpr int kWaves = 4;
constexpr int kTile = 32;        // tile edge handled by one wave per step
constexpr int kBlockRows = kWaves * kTile;  // rows (or columns) owned by one workgroup

// Workgroups per compute unit the sweeps are compiled for (register budget):
// the column pass with separate chi_1 / chi_2 tiles and all K > 64 variants
// need the whole register file of a SIMD.
constexpr int sweep_rows_occupancy(int KB) { return KB >= 4 ? 1 : 2; }
// Rows of W per W-update unit (four thread slices per row of KP threads).
constexpr int update_w_unit_rows(int KB) { return kBlock / (32 * KB * 4) > 0 ? kBlock / (32 * KB * 4) : 1; }
constexpr int sweep_cols_occupancy(int bc, int KB, int kind, bool dual) {
  return (KB >= 4 || (dual && kind == KIND_UPDATE && bc != BC_B1)) ? 1 : 2;
}

__host__ __device__ inline int beta_class(double beta) {
  if (beta == 2.0) return BC_B2;
  if (beta == 1.0) return BC_B1;
  if (beta == 0.0) return BC_B0;
  if (beta == 0.5) return BC_B05;
  if (beta == 1.5) return BC_B15;
  return BC_GEN;
}

// gamma(beta), paper eq. (def_gamma)
__host__ __device__ inline double gamma_of(double beta) {
  if (beta < 1.0) return 1.0 / (2.0 - beta);
  if (beta <= 2.0) return 1.0;
  return 1.0 / (beta - 1.0);
}

struct SweepRowsArgs {
  const float* V; int64_t ldv;
  const float* W; int64_t ldw;     // tilde W (rows owned by each wave)
  const float* H; int64_t ldh;     // tilde H
  int F, N, K;
  float bm2, kappa;                // beta - 2, smoothing constant
  double beta;
  int n_groups, tiles_per_group;   // grid = row_blocks (128 rows) * n_groups
  float* pnum; float* pden;        // [n_groups][F][KP] partial W contractions
  float* prs;                      // [n_groups][KP] partial row sums of H (beta = 1)
  double* pobj;                    // [grid] objective partials (nullable)
  int vec4;                        // V rows 16-byte aligned
  int hvec;                        // H rows 16-byte aligned
  int vstream;                     // V loads with the nontemporal hint (load policy; 0 by default)
  unsigned* flags;                 // status word (float16 range check)
  float* Pst; float* Qst; int NT;  // P, Q tiles [row tile * NT + column tile][32 n][32 f] (fused joint pass)
  const unsigned* halt;            // nullable: the launch does nothing when *halt != 0 (stopped run)
};

struct SweepColsArgs {
  const float* V; int64_t ldv;
  const float* WT; int64_t ldwt;   // transposed factor forming Lambda (K x F): W~ joint, W_new alternating
  const float* H; int64_t ldh;     // tilde H (columns owned by each wave)
  const float* C1; const float* C2;  // contraction operands (chi_1, chi_2): F x KP, ld KP, zero-padded
  const float* C0;                   // row-major factor forming Lambda (low-precision joint pass): F x KP
  int F, N, K;
  float bm2, kappa;
  int f_groups, tiles_per_group;   // grid = col_blocks (128 columns) * f_groups
  float* pnum; float* pden;        // [f_groups][N][KP] partial H contractions
  const float* Pst; const float* Qst; int NT;  // stored P, Q tiles (fused joint pass)
  unsigned* flags;                 // status word (float16 range check)
  // column sums of W_new^2 and W_new (normalization), nullable: workgroups of
  // the first `col_parts` column blocks each cover `col_chunk` rows of their
  // row group and write pcol[g * col_parts + cb][2][KP]
  const float* Wn; double* pcol; int col_parts, col_chunk;
  const unsigned* halt;            // nullable: the launch does nothing when *halt != 0
};

struct UpdateWArgs {
  const float* W; int64_t ldw;     // tilde W
  const float* pnum; const float* pden; const float* prs;
  int F, K, n_groups;
  double beta, gamma;
  int joint, beta_one;
  float* Wn; float* C1; float* C2; // [F][KP]
  float* WT; int64_t ldt;          // [KP][ldt]: W~^T (joint) or W_new^T (alternating)
  float* C0;                       // nullable: W~ row-major, ld KP (joint, low-precision products)
  double* pcol;                    // [grid][2][KP] column norm^2 and sum partials
  unsigned* flags;
  const unsigned* halt;            // nullable: the launch does nothing when *halt != 0
  const double* gram;              // nullable: [KP][KP] H~ H~^T; the denominator is W~ (H~ H~^T) (beta = 2)
};

struct UpdateHArgs {
  float* H; int64_t ldh;
  const float* pnum; const float* pden;
  int F, N, K, f_groups;
  double gamma;
  int beta_one, normalize;
  const double* pcol; int pcol_blocks;   // column partials of W_new (pcol_blocks rows)
  const double* pobj; int nobj; double* d_obj;  // objective partials of the W pass
  const float* Wn; float* W; int64_t ldw;  // W: nullable (no write-back)
  unsigned* flags;
  // joint MM, a sub-iteration before the last: instead of H, write
  // chi_1(H_new, H~) and chi_2(H_new, H~) ([K][ldc]) for the next W step
  float* C1h; float* C2h; int64_t ldc; double beta;
  const unsigned* halt;            // nullable: the launch does nothing when *halt != 0
  const double* gram;              // nullable: [KP][KP] G2 = chi_2^T W~ (joint) or W_new^T W_new
                                   // (alternating); the denominator is G2 H~ (beta = 2)
};

// launchers (nmf_kernels.hip)
// pq: the joint W pass keeps P, Q (Pst, Qst) and the joint H pass contracts them
hipError_t launch_sweep_rows(int bc, int kb, int kind, bool obj, bool pq, int grid, hipStream_t s,
                             const SweepRowsArgs& a);
// W pass of a later joint sub-iteration: a.H = chi_1(H_l, H~), a.W = chi_2(H_l, H~)
hipError_t launch_sweep_rows_pq(int bc, int kb, int grid, hipStream_t s, const SweepRowsArgs& a);
hipError_t launch_sweep_cols(int bc, int kb, int kind, bool dual, bool pq, int grid, hipStream_t s,
                             const SweepColsArgs& a);
// low-precision products (prec 1 = bfloat16, 2 = float16; update kind, K <= 64)
hipError_t launch_sweep_rows_lp(int prec, int bc, int kb, bool obj, bool pq, int grid, hipStream_t s,
                                const SweepRowsArgs& a);
hipError_t launch_sweep_cols_lp(int prec, int bc, int kb, bool dual, bool pq, int grid, hipStream_t s,
                                const SweepColsArgs& a);
hipError_t launch_update_w(int kb, int grid, hipStream_t s, const UpdateWArgs& a);
hipError_t launch_update_h(int kb, int grid, hipStream_t s, const UpdateHArgs& a);
hipError_t launch_finalize_objective(hipStream_t s, const double* pobj, int n, double* out, unsigned* flags);
// dscale (nullable, device): the gradient is multiplied by scale * *dscale
hipError_t launch_grad_w(int kb, int grid, hipStream_t s, const float* pnum, int F, int K, int n_groups,
                         double scale, const double* dscale, float* dW, int64_t lddw);
hipError_t launch_grad_h(int kb, int grid, hipStream_t s, const float* pnum, int N, int K, int f_groups,
                         double scale, const double* dscale, float* dH, int64_t lddh);
hipError_t launch_transpose(hipStream_t s, const float* W, int64_t ldw, int F, int K, int KP, float* WT,
                            int64_t ldt, float* Wp);
// Fused single-launch outer iteration (cooperative; grid barriers between the
// W pass, W update, H pass and H update).  Returns hipErrorNotSupported when
// the instantiation does not exist.
struct FusedArgs {
  SweepRowsArgs r;
  UpdateWArgs uw;
  SweepColsArgs c;
  UpdateHArgs uh;
  int n_items_w, n_items_h, slabs, ntiles;
  unsigned* bar;        // [2]: arrival count, generation
  float* colsum;        // [2][KP]: column norms and sums of W_new
  unsigned spin_limit;  // barrier polls before giving up (sets NMF_FLAG_BARRIER)
  unsigned long long* stamps;  // nullable: [8] wall-clock stamps of workgroup 0 at phase boundaries
};
int fused_max_blocks(int bc, int kb, bool joint, bool obj, int num_cus);
hipError_t launch_fused(int bc, int kb, bool joint, bool obj, int grid, hipStream_t s, const FusedArgs& a);

// Many problems in one persistent launch.  Each problem's outer iteration is
// split into four phases of independent work items (W-pass items, W-update
// units, H-pass items, H-update units); phase q of a problem may start once
// every item of its phase q - 1 has finished.  The items of all problems are
// listed phase-major, so an item only ever waits for items listed before it:
// those were taken by running workgroups, which makes the wait finite without
// co-residency or a cooperative launch.
enum { PH_WPASS = 0, PH_WUPDATE = 1, PH_HPASS = 2, PH_HUPDATE = 3 };
struct BatchProblem {
  SweepRowsArgs ra;
  UpdateWArgs ua;
  SweepColsArgs ca;
  UpdateHArgs ha;
  int bc, kb;
  int wfused;    // the W-pass items apply the W update (no W-update items)
  int hfused;    // ... and the H-pass items the H update (no H-update items)
  int items[4];  // work items per phase
  int units[4];  // update units per phase (W rows / H columns groups); an item covers `per_item` of them
  int per_item[4];
};
struct BatchArgs {
  const BatchProblem* probs;
  const int2* list;     // [total]: (problem, phase << 24 | item), phase-major
  int total;
  const int* counts;    // nullable: total and the problem count read from [0], [1] instead
  unsigned* next;       // queue position (zero at launch; reset by the last workgroup)
  unsigned* exited;     // workgroups that left the queue loop
  unsigned* done;       // [problems][4] finished items per phase (reset at exit)
  int nprob;
  double* d_obj;        // nullable: [problems] objective of the entry iterate
  unsigned* flags;      // sticky status word
  unsigned spin_limit;  // dependency polls before giving up (sets NMF_FLAG_BARRIER)
};
// prec 0 = float32, 1 = bfloat16 products
hipError_t launch_batched(int prec, bool joint, int grid, hipStream_t s, const BatchArgs& a);
int batched_max_blocks(int prec, bool joint, int num_cus);

// beta = 1 step for a V stored by its nonzeros in both compressed orders
// (nmf_sparse.hip).  Workspace arrays are K4-padded (K4 = K rounded up to 4).
struct SparseArgs {
  int F, N, K, normalize;
  int64_t nnz;
  const int64_t* row_ptr; const int32_t* col_idx; const float* row_val;  // CSR
  const int64_t* col_ptr; const int32_t* row_idx; const float* col_val;  // CSC (same entries)
  float* Wio; int64_t ldw;   // caller's W (read as W~, written as the result)
  float* Hio; int64_t ldh;   // caller's H
  float* HT;                 // [N][K4] H~ transposed
  float* Wc;                 // [F][K4] W~
  float* Wn;                 // [F][K4] W_new
  const float* Wg;           // gather table of the column pass (Wc or Wn)
  float* numW;               // [F][K4]
  float* numH;               // [N][K4]
  double* prow;              // [ceil(N / 64)][K4] partial row sums of H~
  double* pcw;               // [ceil(F / 64)][K4] partial column sums of W~
  double* pobj;              // [row-pass blocks] objective partials (nullable: no objective)
  double* pcol;              // [ceil(F / 64)][2][K4] column sums and squares of W_new
  double* d_obj;             // objective of the entry iterate (nullable)
  unsigned* flags;
};
// grid sizes: transpose / copy blocks of H and W (64 each), row- and column-pass
// blocks (four lines each)
int sparse_blocks(int F, int N, int* hb, int* wcb, int* rb, int* cb);
// one step: prep; joint: pass(rows + cols), update_w; alternating: pass(rows),
// update_w, pass(cols) with a.Wg = a.Wn; then update_h
hipError_t launch_sparse_prep(hipStream_t s, const SparseArgs& a);
hipError_t launch_sparse_pass(hipStream_t s, const SparseArgs& a, bool rows, bool cols);
hipError_t launch_sparse_update_w(hipStream_t s, const SparseArgs& a);
hipError_t launch_sparse_update_h(hipStream_t s, const SparseArgs& a);
hipError_t launch_sparse_objective(hipStream_t s, const SparseArgs& a, double* d_out);
hipError_t launch_sparse_validate(hipStream_t s, const SparseArgs& a);

// Device-side outer loop (Sec. 4.1.2): the objective trace and the stopping
// rule.  run_init sets *halt = 0 and *stop = -1.  run_decide sums the n objective
// partials of iterate t (fixed order), writes trace[t], and for t >= 1 sets
// *halt = 1 and *stop = t when (trace[t-1] - trace[t]) / trace[t] <= eps; it does
// nothing once *halt is set.
hipError_t launch_run_init(hipStream_t s, unsigned* halt, int32_t* stop);
hipError_t launch_run_decide(hipStream_t s, const double* pobj, int n, double* trace, int t, double eps,
                             unsigned* halt, int32_t* stop, unsigned* flags);
// KKT residuals of Sec. 4.1.5 from the gradient partials of the grad passes:
// res[0] = sum |min(W, grad_W)| / (F K), res[1] = sum |min(H, grad_H)| / (K N).
// `part` holds kkt_parts() float64 block partials.
int kkt_parts();
hipError_t launch_kkt(int kb, hipStream_t s, const float* pnumw, int n_groups, const float* pnumh, int f_groups,
                      const float* W, int64_t ldw, const float* H, int64_t ldh, int F, int N, int K, double* part,
                      double* res);

// Gram matrix G[k][l] = sum_i x_i[k] y_i[l] (float64), k, l < K <= 64, stored
// [KP][KP]: COLS, the i-th columns of K x N matrices (H~ H~^T); otherwise the
// i-th rows of F x K row-major matrices (chi_2^T W~, W_new^T W_new).  Two
// launches: block partials in `part` ([gram_parts()][KP][KP]), then their sum
// in a fixed order.
int gram_parts();
hipError_t launch_gram(bool cols, hipStream_t s, const float* X, int64_t ldx, const float* Y, int64_t ldy, int K,
                       int KP, int64_t len, double* part, double* G);

hipError_t launch_validate(hipStream_t s, const float* V, int64_t ldv, const float* W, int64_t ldw,
                           const float* H, int64_t ldh, int F, int N, int K, int zero_bad, unsigned* flags);

}  // namespace nmf
