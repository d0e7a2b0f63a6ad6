// Launch planning shared by the host library and the device-side planner of
// the batched step: the splits of a problem's passes, its workspace layout and
// the kernel arguments of one outer iteration (host and device code).
#pragma once

#include "nmf_beta.h"
#include "nmf_internal.h"

#define NMF_PLAN_HD __host__ __device__

namespace nmf {

NMF_PLAN_HD inline int64_t min64(int64_t a, int64_t b) { return a < b ? a : b; }
NMF_PLAN_HD inline int64_t max64(int64_t a, int64_t b) { return a > b ? a : b; }

// Workspace header (zeroed at allocation): the sticky flags word at byte 0,
// the fused kernel's grid-barrier words (arrivals, generation) at bytes 8, 12,
// its eight phase stamps (uint64) at bytes 64..127, and the halt word of the
// device-side outer loop at byte 128.
constexpr size_t kHeaderBytes = 256;
constexpr int kColChunkRows = 512;  // rows of W_new per column-partial workgroup of the H pass

// batched update items: rows of W per W-update item (all of them loaded at
// once), columns of H per H-update item (units of kBlock / KP columns)
constexpr int kBatchWRows = 64;
constexpr int kBatchUpdateCols = 256;
NMF_PLAN_HD inline int batch_h_units(int KB) { return (int)max64(1, kBatchUpdateCols / (kBlock / (32 * KB))); }

constexpr size_t kAlign = 256;
NMF_PLAN_HD inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }
NMF_PLAN_HD inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

struct Plan {
  int KB, KP;
  int row_blocks, n_groups, tiles_n;  // sweep_rows grid = row_blocks * n_groups
  int col_blocks, f_groups, tiles_f;  // sweep_cols grid = col_blocks * f_groups
  int uw_blocks, uh_blocks;
  int col_parts, col_chunk;           // column partials of W_new formed in the H pass
  int64_t ldt;                        // leading dimension of the transposed factor (K x F)
  bool fused;                         // one cooperative launch (grid = fused_grid)
  bool pq;                            // joint streaming path keeps P, Q between the passes
  bool row_pcol;                      // batch: room for one column partial per row block
  int fused_grid;
  // byte offsets inside the workspace
  size_t o_pobj, o_pnum, o_pden, o_prs, o_wn, o_c1, o_c2, o_c0, o_wt, o_pcol, o_pnumh, o_pdenh, o_colsum, o_pst,
      o_qst, o_c1h, o_c2h, total;
  int64_t ldc;                        // leading dimension of the chi(H) terms of joint sub-iterations
};

NMF_PLAN_HD inline int kblocks_for(int64_t K) {
  if (K <= 32) return 1;
  if (K <= 64) return 2;
  return 4;
}

// Region sizes (bytes) of the workspace; offsets are assigned in this order.
struct Sizes {
  size_t pobj, pnum, prs, fk, wt, pcol, pnumh, pq, kn;
};

NMF_PLAN_HD inline Plan layout(const Sizes& z, Plan p) {
  size_t o = kHeaderBytes;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
  p.o_pobj = take(z.pobj);
  p.o_pnum = take(z.pnum);
  p.o_pden = take(z.pnum);
  p.o_prs = take(z.prs);
  p.o_wn = take(z.fk);
  p.o_c1 = take(z.fk);
  p.o_c2 = take(z.fk);
  p.o_c0 = take(z.fk);
  p.o_wt = take(z.wt);
  p.o_pcol = take(z.pcol);
  p.o_pnumh = take(z.pnumh);
  p.o_pdenh = take(z.pnumh);
  p.o_colsum = take(sizeof(float) * 2 * 128);
  p.o_pst = take(z.pq);
  p.o_qst = take(z.pq);
  p.o_c1h = take(z.kn);
  p.o_c2h = take(z.kn);
  p.total = o;
  return p;
}

// `cols_occ`: workgroups per CU of the streaming column pass.  `fused_grid` > 0
// plans the single-launch path with that many workgroups.
// Column-partial split, transposed leading dimension and workspace offsets of
// a plan whose splits are set.
NMF_PLAN_HD inline Plan finish_plan(Plan p, int64_t F, int64_t N, bool inner = false) {
  {
    const int64_t rows = (int64_t)p.tiles_f * kTile;
    p.col_parts = (int)min64(p.col_blocks, cdiv(rows, kColChunkRows));
    p.col_chunk = (int)cdiv(rows, p.col_parts);
  }
  p.ldt = cdiv(F, 4) * 4;
  Sizes z;
  z.pobj = sizeof(double) * (size_t)max64((int64_t)p.row_blocks * p.n_groups, p.fused_grid);
  z.pnum = sizeof(float) * (size_t)p.n_groups * F * p.KP;
  z.prs = sizeof(float) * (size_t)p.n_groups * p.KP;
  z.fk = sizeof(float) * (size_t)F * p.KP;
  z.wt = sizeof(float) * (size_t)p.KP * p.ldt;
  z.pcol = sizeof(double) *
           (size_t)(p.fused ? p.uw_blocks
                            : max64((int64_t)p.f_groups * p.col_parts, p.row_pcol ? p.row_blocks : 0)) *
           2 * p.KP;
  z.pnumh = sizeof(float) * (size_t)p.f_groups * N * p.KP;
  z.pq = (p.fused || p.pq) ? sizeof(float) * (size_t)cdiv(F, kTile) * cdiv(N, kTile) * kTile * kTile : 0;
  p.ldc = cdiv(N, 4) * 4;
  z.kn = inner ? sizeof(float) * (size_t)p.KP * p.ldc : 0;
  return layout(z, p);
}

// Splits of a problem inside a batch: every row (column) group covers about
// `tiles` column (row) tiles; one W-update unit of rows and one H-update unit
// of columns per work item.
// Joint MM in a batch keeps the W pass's element terms P, Q for its H pass
// only at K > 32 and beta != 1: elsewhere the H pass forms Lambda~ again from a
// copy of W~ and H~ (2FNK flops against P, Q written and read back: 8FN bytes
// in float32, 4FN in bfloat16 or at beta = 1, where only P is kept).
NMF_PLAN_HD inline bool batch_keeps_pq(bool joint, int prec, int64_t K, double beta) {
  (void)prec;
  return joint && kblocks_for(K) > 1 && beta_class(beta) != BC_B1;
}

NMF_PLAN_HD inline Plan make_batch_plan(int64_t F, int64_t N, int64_t K, double beta, int tiles, bool joint,
                                        int prec) {
  Plan p{};
  p.pq = batch_keeps_pq(joint, prec, K, beta);
  p.KB = kblocks_for(K);
  p.KP = 32 * p.KB;
  const int64_t tn = cdiv(N, kTile), tf = cdiv(F, kTile);
  p.row_blocks = (int)cdiv(F, kBlockRows);
  p.n_groups = (int)cdiv(tn, tiles);
  p.tiles_n = (int)cdiv(tn, p.n_groups);
  p.n_groups = (int)cdiv(tn, p.tiles_n);
  p.col_blocks = (int)cdiv(N, kBlockRows);
  p.f_groups = (int)cdiv(tf, tiles);
  p.tiles_f = (int)cdiv(tf, p.f_groups);
  p.f_groups = (int)cdiv(tf, p.tiles_f);
  p.uw_blocks = (int)cdiv(F, update_w_unit_rows(p.KB));
  p.uh_blocks = (int)cdiv(N, kBlock / p.KP);
  p.row_pcol = true;
  return finish_plan(p, F, N);
}

// Kernel arguments of one outer iteration of a problem whose workspace regions
// (offsets of `p`) start at `ws`.
struct StepArgs {
  SweepRowsArgs ra;
  UpdateWArgs ua;
  SweepColsArgs ca;
  UpdateHArgs ha;
  int sw_grid, sh_grid;
};

NMF_PLAN_HD inline StepArgs make_step_args(const Plan& p, char* ws, unsigned* flags, int64_t F, int64_t N, int64_t K, const float* V,
                        int64_t ldv, float* W, int64_t ldw, float* H, int64_t ldh, double beta, bool joint, int prec,
                        const nmf_step_opts& o, double* d_objective) {
  const int bc = beta_class(beta);
  const bool beta_one = (bc == BC_B1);
  float* Wn = (float*)(ws + p.o_wn);
  float* C1 = (float*)(ws + p.o_c1);
  float* C2 = (float*)(ws + p.o_c2);
  StepArgs sa{};
  SweepRowsArgs& ra = sa.ra;
  ra.V = V; ra.ldv = ldv; ra.W = W; ra.ldw = ldw; ra.H = H; ra.ldh = ldh;
  ra.F = (int)F; ra.N = (int)N; ra.K = (int)K;
  ra.bm2 = (float)(beta - 2.0); ra.kappa = o.kappa; ra.beta = beta;
  ra.n_groups = p.n_groups; ra.tiles_per_group = p.tiles_n;
  ra.pnum = (float*)(ws + p.o_pnum); ra.pden = (float*)(ws + p.o_pden); ra.prs = (float*)(ws + p.o_prs);
  ra.pobj = (double*)(ws + p.o_pobj);
  ra.vec4 = ((uintptr_t)V % 16 == 0) && (ldv % 4 == 0);
  ra.hvec = ((uintptr_t)H % 16 == 0) && (ldh % 4 == 0);
  ra.vstream = 0;  // ordinary V loads (see ldc_nt)
  ra.flags = flags;
  sa.sw_grid = p.row_blocks * p.n_groups;

  UpdateWArgs& ua = sa.ua;
  ua.W = W; ua.ldw = ldw; ua.pnum = ra.pnum; ua.pden = ra.pden; ua.prs = ra.prs;
  ua.F = (int)F; ua.K = (int)K; ua.n_groups = p.n_groups;
  const double gamma = o.exponent == NMF_EXPONENT_ONE ? 1.0 : gamma_of(beta);
  ua.beta = beta; ua.gamma = gamma; ua.joint = joint; ua.beta_one = beta_one;
  ua.Wn = Wn; ua.C1 = C1; ua.C2 = C2; ua.pcol = (double*)(ws + p.o_pcol);
  ua.WT = (float*)(ws + p.o_wt); ua.ldt = p.ldt;
  ua.C0 = (prec != NMF_FP32 && joint && !p.pq) ? (float*)(ws + p.o_c0) : nullptr;
  ua.flags = flags;

  SweepColsArgs& ca = sa.ca;
  ca.V = V; ca.ldv = ldv;
  ca.WT = ua.WT; ca.ldwt = p.ldt;
  ca.C0 = ua.C0;
  ca.flags = flags;
  if (joint) { ca.C1 = C1; ca.C2 = C2; }
  else { ca.C1 = Wn; ca.C2 = Wn; }
  ca.H = H; ca.ldh = ldh;
  ca.F = (int)F; ca.N = (int)N; ca.K = (int)K;
  ca.bm2 = (float)(beta - 2.0); ca.kappa = o.kappa;
  ca.f_groups = p.f_groups; ca.tiles_per_group = p.tiles_f;
  ca.pnum = (float*)(ws + p.o_pnumh); ca.pden = (float*)(ws + p.o_pdenh);
  sa.sh_grid = p.col_blocks * p.f_groups;

  UpdateHArgs& ha = sa.ha;
  ha.H = H; ha.ldh = ldh; ha.pnum = ca.pnum; ha.pden = ca.pden;
  ha.F = (int)F; ha.N = (int)N; ha.K = (int)K; ha.f_groups = p.f_groups;
  ha.gamma = gamma; ha.beta_one = beta_one; ha.normalize = o.normalize;
  ha.pcol = ua.pcol; ha.pcol_blocks = p.fused ? p.uw_blocks : p.f_groups * p.col_parts;
  if (!p.fused) { ca.Wn = Wn; ca.pcol = ua.pcol; ca.col_parts = p.col_parts; ca.col_chunk = p.col_chunk; }
  ha.pobj = ra.pobj; ha.nobj = sa.sw_grid; ha.d_obj = d_objective;
  ha.Wn = Wn; ha.W = W; ha.ldw = ldw; ha.flags = flags;
  ha.beta = beta;
  return sa;
}

// Per-bucket tile counts of batched problems: bucket (K block, size class, beta
// class), the size class by the larger of the problem's row and column tile
// counts (<= 32, <= 64, <= 128, more).  The tile count changes how a pass
// splits its contraction into items, not the arithmetic; the beta class sets
// the cost of an item's element-wise work and so the best split.
constexpr int kBatchBetaClasses = 6;  // BC_GEN .. BC_B15
constexpr int kBatchBuckets = NMF_BATCH_BUCKETS;
static_assert(kBatchBuckets == 2 * 4 * kBatchBetaClasses, "K blocks x size classes x beta classes");
NMF_PLAN_HD inline int bucket_of(int64_t F, int64_t N, int64_t K, double beta) {
  const int64_t t = max64(cdiv(F, kTile), cdiv(N, kTile));
  const int cls = t <= 32 ? 0 : t <= 64 ? 1 : t <= 128 ? 2 : 3;
  return ((kblocks_for(K) - 1) * 4 + cls) * kBatchBetaClasses + beta_class(beta);
}

// A problem whose rows take one column group has the whole W-step
// contractions of a row block in one W-pass item, which then applies the W
// update itself: the problem has no W-update items (batches run float32 or
// bfloat16 products).
NMF_PLAN_HD inline bool batch_w_fused(const Plan& p, int prec) {
  return p.n_groups == 1 && (prec == NMF_FP32 || prec == NMF_BF16);
}
// If its columns also take one row group, the W-pass items write the column
// partials of W_new (one per row block) and the H-pass items apply the H
// update and write W back: the problem has no H-update items either.
NMF_PLAN_HD inline bool batch_h_fused(const Plan& p, int prec) { return batch_w_fused(p, prec) && p.f_groups == 1; }

// Update units and work items per phase of a problem in a batch of precision
// `prec`: W-pass items (row block x column group), W-update items of
// kBatchWRows rows (none if batch_w_fused), H-pass items (column block x row
// group), H-update items of batch_h_units column units (none if batch_h_fused).
NMF_PLAN_HD inline void batch_phases(const Plan& p, int64_t F, int prec, int units[4], int per_item[4],
                                     int items[4]) {
  units[PH_WPASS] = p.row_blocks * p.n_groups;
  units[PH_WUPDATE] = batch_w_fused(p, prec) ? 0 : (int)cdiv(F, kBatchWRows);
  units[PH_HPASS] = p.col_blocks * p.f_groups;
  units[PH_HUPDATE] = batch_h_fused(p, prec) ? 0 : p.uh_blocks;
  per_item[PH_WPASS] = 1;
  per_item[PH_WUPDATE] = 1;
  per_item[PH_HPASS] = 1;
  per_item[PH_HUPDATE] = batch_h_units(p.KB);
  for (int ph = 0; ph < 4; ++ph) items[ph] = (int)cdiv(units[ph], per_item[ph]);
}

// Kernel descriptor of one problem of a batch (workspace at `ws`): the four
// phases' arguments, and for each phase its update units and work items.
NMF_PLAN_HD inline BatchProblem make_batch_problem(const Plan& p, char* ws, unsigned* flags, const nmf_problem& q,
                                                   bool joint, const nmf_step_opts& o) {
  StepArgs sa = make_step_args(p, ws, flags, q.F, q.N, q.K, q.V, q.ldv, q.W, q.ldw, q.H, q.ldh, q.beta, joint,
                               o.precision, o, nullptr);
  if (p.pq) {  // joint: the H pass contracts the kept P, Q tiles
    sa.ra.NT = (int)cdiv(q.N, kTile);
    sa.ra.Pst = (float*)(ws + p.o_pst);
    sa.ra.Qst = (float*)(ws + p.o_qst);
    sa.ca.NT = sa.ra.NT;
    sa.ca.Pst = sa.ra.Pst;
    sa.ca.Qst = sa.ra.Qst;
  }
  BatchProblem d;
  d.ra = sa.ra;
  d.ua = sa.ua;
  d.ca = sa.ca;
  d.ha = sa.ha;
  d.bc = beta_class(q.beta);
  d.kb = p.KB;
  d.wfused = batch_w_fused(p, o.precision);
  d.hfused = batch_h_fused(p, o.precision);
  if (d.hfused) {  // column partials from the W pass, one per row block
    d.ca.pcol = nullptr;
    d.ha.pcol_blocks = p.row_blocks;
  } else {
    d.ua.pcol = nullptr;
  }
  batch_phases(p, q.F, o.precision, d.units, d.per_item, d.items);
  return d;
}

// Work items of one problem's outer iteration in a batch (all four phases).
NMF_PLAN_HD inline int64_t batch_items(const Plan& p, int64_t F, int prec) {
  int units[4], per_item[4], items[4];
  batch_phases(p, F, prec, units, per_item, items);
  return (int64_t)items[0] + items[1] + items[2] + items[3];
}

}  // namespace nmf
