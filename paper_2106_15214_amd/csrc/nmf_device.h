// Device-side building blocks of the beta-NMF kernels (gfx950, wave64).
//
// Data layout: V (F x N), W (F x K), H (K x N), float32 row-major.  Lambda = W H
// is formed tile by tile on the matrix cores (v_mfma_f32_32x32x2_f32) and is
// never written to memory.
//
// v_mfma_f32_32x32x2_f32 operand layout (lane l, li = l % 32, hi = l / 32):
//   A[i][kk] : lane holds A[li][hi];  B[kk][j] : lane holds B[hi][li];
//   C[i][j]  : lane holds C[acc_row(r, hi)][li] in accumulator register r.
// An accumulator is therefore directly the A operand of a product whose
// contraction runs over the accumulator's row index, 2 rows per instruction.
//
// Two orientations of a pass over V, each a "work item" processed by one
// workgroup of four waves:
//  * rows item: the waves own four 32-row slabs and walk 32-column tiles in
//    lockstep; Lambda^T is formed (lane -> f, register -> n), so P H^T and Q H^T
//    (the W-step contractions, reduced over n) accumulate in registers.
//  * cols item: the waves own four 32-column slabs and walk 32-row tiles;
//    Lambda is formed (lane -> n, register -> f), so chi_1^T P and chi_2^T Q (the
//    H-step contractions, reduced over f) accumulate in registers.
// Operand tiles are staged in LDS by the whole workgroup, double-buffered; each
// wave prefetches its next V tile into registers while the matrix cores work.
// An item writes one partial per output entry; update code sums the partials
// in a fixed order, so every result is deterministic.
#pragma once

#include "nmf_internal.h"
#include "nmf_math.h"

namespace nmf {

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Row offset held in accumulator register r by lane half `hi`: 8(r/4) + 4hi + r%4.
__device__ __forceinline__ int acc_row(int r, int hi) { return 8 * (r >> 2) + 4 * hi + (r & 3); }

// Lambda^(beta-2) for a smoothed Lambda (> 0).
template <int BC>
__device__ __forceinline__ float pow_bm2(float lam, float bm2) {
  if (BC == BC_B2 || BC == BC_B2G) return 1.f;
  if (BC == BC_B1) return __builtin_amdgcn_rcpf(lam);
  if (BC == BC_B0) { float r = __builtin_amdgcn_rcpf(lam); return r * r; }
  if (BC == BC_B05) { float s = __builtin_amdgcn_rsqf(lam); return s * s * s; }
  if (BC == BC_B15) return __builtin_amdgcn_rsqf(lam);
  return __builtin_amdgcn_exp2f(bm2 * __builtin_amdgcn_logf(lam));
}

// P = v lam^(beta-2), Q = lam^(beta-1) (v and lam include kappa), the two
// element-wise terms of eqs. (alt_update) / (jnt_update).  P is exactly 0 where
// v = 0: for beta < 2 the power of a small positive lam overflows float32
// (lam^(-3/2) beyond the range below lam = 2e-26, lam^(-2) below 5e-20), and
// 0 * inf would turn an entry whose value is 0 into a NaN.
template <int BC>
__device__ __forceinline__ void beta_terms(float v, float lam, float bm2, float& P, float& Q) {
  if (BC == BC_B2) { P = v; Q = lam; return; }
  if (BC == BC_B2G) { P = v; Q = 0.f; return; }  // Q H~^T comes from the Gram form
  float e;
  if (BC == BC_B1) { e = __builtin_amdgcn_rcpf(lam); Q = 1.f; }
  else if (BC == BC_B0) { const float r = __builtin_amdgcn_rcpf(lam); Q = r; e = r * r; }
  else if (BC == BC_B05) { const float s = __builtin_amdgcn_rsqf(lam); Q = s; e = s * s * s; }
  else if (BC == BC_B15) { const float s = __builtin_amdgcn_rsqf(lam); e = s; Q = lam * s; }
  else { e = __builtin_amdgcn_exp2f(bm2 * __builtin_amdgcn_logf(lam)); Q = lam * e; }
  P = v != 0.f ? v * e : 0.f;
}

// General-beta term of eq. (beta-div) (out of line: three float64 pows).
__device__ __noinline__ inline double d_beta_general(double v, double l, double beta) {
  if (v > 0.0)
    return pow(v, beta) / (beta * (beta - 1.0)) + pow(l, beta) / beta - v * pow(l, beta - 1.0) / (beta - 1.0);
  return beta > 0.0 ? pow(l, beta) / beta : __builtin_inf();
}

// d_beta(v | l) in float64 (v, l include kappa), eq. (beta-div); v = 0 takes
// the limit of the expression.
template <int BC>
__device__ __forceinline__ double d_beta(double v, double l, double beta) {
  if (BC == BC_B2 || BC == BC_B2G) { double t = v - l; return 0.5 * t * t; }
  if (BC == BC_B1) {  // v log(v / l) - v + l, and the limit l at v = 0
    const double t = v * log64(div64(v, l)) - v + l;
    return v > 0.0 ? t : l;
  }
  if (BC == BC_B0) {  // r - log r - 1 with r = v / l, and +inf at v = 0
    const double r = div64(v, l);
    const double t = r - log64(r) - 1.0;
    return v > 0.0 ? t : __builtin_inf();
  }
  // beta = 1/2 and 3/2 in the factored forms (s = sqrt v, t = sqrt l):
  //   d_{1/2} = 2 (s - t)^2 / t,   d_{3/2} = (2/3) (s - t)^2 (2 s + t),
  // algebraically equal to eq. (beta-div) and free of its cancellation at v ~ l
  if (BC == BC_B05 || BC == BC_B15) {
    const double rl = rsqrt64(l), t = l > 0.0 ? sqrt64(l, rl) : 0.0;
    const double s = v > 0.0 ? sqrt64(v, rsqrt64(v)) : 0.0;
    const double dst = (s - t) * (s - t);
    if (BC == BC_B05) return 2.0 * dst * rl;
    return (2.0 / 3.0) * dst * (2.0 * s + t);
  }
  return d_beta_general(v, l, beta);
}

// p[idx] when ok, else 0.  The load is issued unconditionally (from p[0] when
// !ok, so p must be the start of a non-empty array): a conditional load would
// be compiled as a branch that waits for it, serializing consecutive loads.
__device__ __forceinline__ float ldz(const float* __restrict__ p, int64_t idx, bool ok) {
  const float x = p[ok ? idx : 0];
  return ok ? x : 0.f;
}
// p[idx] when ok, else p[0] (a finite in-bounds value the caller masks or
// multiplies by zero later).  Only the address is selected: a select on the
// loaded value would make the compiler wait for the load right there.
__device__ __forceinline__ float ldc(const float* __restrict__ p, int64_t idx, bool ok) { return p[ok ? idx : 0]; }
__device__ __forceinline__ float4 ldc4(const float* __restrict__ p, int64_t idx, bool ok) {
  return *reinterpret_cast<const float4*>(p + (ok ? idx : 0));
}

// V loads of the W pass with the nontemporal hint, selected per launch by
// SweepRowsArgs::vstream (same selection of the address as ldc / ldc4).  The
// launch plans leave it off: on the 20000 x 10000 count workload the hinted
// 32-byte pieces of a row's 128-byte segment re-fetch lines (1.4 GB for 0.8 GB
// of V) and the W pass took 760 us (FP32) and 525 us (BF16) against 737 and
// 481 us with ordinary loads.  The per-launch choice itself stays: the tile
// loop compiled without it (ordinary loads only) measured slower still, 804
// and 551 us, from a different placement of the next tile's loads.
typedef float f32x4v __attribute__((ext_vector_type(4)));
__device__ __forceinline__ float ldc_nt(const float* __restrict__ p, int64_t idx, bool ok) {
  return __builtin_nontemporal_load(p + (ok ? idx : 0));
}
__device__ __forceinline__ float4 ldc4_nt(const float* __restrict__ p, int64_t idx, bool ok) {
  const f32x4v y = __builtin_nontemporal_load(reinterpret_cast<const f32x4v*>(p + (ok ? idx : 0)));
  return make_float4(y[0], y[1], y[2], y[3]);
}

__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, 64);
  return x;
}

// Block-wide deterministic sum of one double per thread; result valid in thread 0.
__device__ __forceinline__ double block_sum(double x, double* red) {
  x = wave_sum(x);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = x;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kWaves; ++w) s += red[w];
  __syncthreads();
  return s;
}

__device__ __forceinline__ void set_flag(unsigned* flags, unsigned bit) {
  __hip_atomic_fetch_or(flags, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __noinline__ inline double pow_out_of_line(double x, double y) { return pow(x, y); }

__device__ __forceinline__ double pow_gamma(double x, double g) {
  if (g == 1.0) return x;
  if (g == 0.5) return sqrt(x);
  return pow_out_of_line(x, g);
}

// chi_1(W, W~) = W~^(2-b) / W^(1-b) = W~ r^(b-1) for b <= 2, else W;
// chi_2(W, W~) = W for b < 1, else W^b / W~^(b-1) = W~ r^b   (r = W / W~).
__device__ __forceinline__ void chi_terms(double beta, double wt, double r, double wnew, float& c1, float& c2) {
  double x1, x2;
  if (beta >= 2.0) x1 = wnew;
  else if (beta == 1.0) x1 = wt;
  else if (beta == 0.0) x1 = wt / r;
  else if (beta == 0.5) x1 = wt / sqrt(r);
  else if (beta == 1.5) x1 = wt * sqrt(r);
  else x1 = wt * pow_out_of_line(r, beta - 1.0);
  if (beta <= 1.0) x2 = wnew;
  else if (beta == 2.0) x2 = wnew * r;
  else if (beta == 1.5) x2 = wnew * sqrt(r);
  else x2 = wt * pow_out_of_line(r, beta);
  c1 = (float)x1;
  c2 = (float)x2;
}

// Sums `groups` partial arrays (stride `gstride` floats) at offsets base + tid +
// i*kBlock (i < PER), several groups per round so that many loads are in
// flight; fixed order, float64 accumulation.  Entries at or beyond `limit`
// hold meaningless sums the caller does not use.
template <int PER>
__device__ __forceinline__ void sum_partials(const float* __restrict__ pn, const float* __restrict__ pd, int groups,
                                             int64_t gstride, int64_t base, int64_t limit, double (&num)[PER],
                                             double (&den)[PER]) {
  constexpr int U = PER >= 4 ? 4 : 16 / PER;  // groups per round
#pragma unroll
  for (int i = 0; i < PER; ++i) { num[i] = 0.0; den[i] = 0.0; }
  const int tid = threadIdx.x;
  bool ok[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) ok[i] = tid + i * kBlock < limit;
  int g = 0;
  for (; g + U <= groups; g += U) {
    float xn[U][PER], xd[U][PER];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int64_t o = (int64_t)(g + u) * gstride + base + tid + i * kBlock;
        xn[u][i] = ldc(pn, o, ok[i]);
        xd[u][i] = pd ? ldc(pd, o, ok[i]) : 0.f;
      }
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
      for (int i = 0; i < PER; ++i) { num[i] += (double)xn[u][i]; den[i] += (double)xd[u][i]; }
  }
  for (; g < groups; ++g) {
    float xn[PER], xd[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int64_t o = (int64_t)g * gstride + base + tid + i * kBlock;
      xn[i] = ldc(pn, o, ok[i]);
      xd[i] = pd ? ldc(pd, o, ok[i]) : 0.f;
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) { num[i] += (double)xn[i]; den[i] += (double)xd[i]; }
  }
}

constexpr int kHS = 36;  // LDS row stride of [k][32] tiles: float4 and dword reads conflict-free

// LDS bytes a rows item needs (two H~ tiles).
// ---------------------------------------------------------------------------
// KL objective of a 32 x 32 tile in the accumulator layout.  With z the sum of
// Lambda over the tile, d_1 summed over the tile is
//   z + sum over the entries with v > 0 of (v log(v / Lambda) - v),
// so entries with v = 0 need no float64 work.  z is summed per lane in float32
// as a pairwise tree of its 16 terms (error at most 4 ulp) and added to the
// float64 total once per tile.  The entries with v > 0 are appended to the
// wave's LDS queue (ballot + prefix count; lanes without an entry write a spare
// slot of their own, so no lane is masked off), and their float64 terms are
// evaluated 64 at a time once a round is full: the logarithms cost one round
// per 64 nonzero entries.  After a tile with at least half of its entries
// nonzero the next tile evaluates its terms in place instead (dense data).
// ---------------------------------------------------------------------------
constexpr int kKlQueue = 64 + 8 * 64;    // carried entries + eight accumulator registers
constexpr int kKlSlots = kKlQueue + 64;  // + one spare slot per lane

__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// v log(v / l) - v for v > 0 (the Lambda term is summed separately)
__device__ __forceinline__ double kl_nz(double v, double l) { return v * log64(div64(v, l)) - v; }

struct KlQueue {
  float* qv;          // [kKlSlots] data values
  float* ql;          // [kKlSlots] Lambda values
  int qn;             // queued entries (uniform over the wavefront), < 64 between tiles
  bool dense;         // evaluate the next tile's terms in place

  // full rounds of 64 queued terms; the remainder moves to the front
  __device__ __forceinline__ void rounds(double& sum) {
    const int lane = threadIdx.x & 63;
    wave_lds_sync();
    const int full = qn >> 6, rest = qn & 63;
    for (int j = 0; j < full; ++j) sum += kl_nz((double)qv[64 * j + lane], (double)ql[64 * j + lane]);
    float rv = 0.f, rl = 0.f;
    if (lane < rest) {
      rv = qv[64 * full + lane];
      rl = ql[64 * full + lane];
    }
    wave_lds_sync();
    if (lane < rest) {
      qv[lane] = rv;
      ql[lane] = rl;
    }
    qn = rest;
  }

  // v, l: data and Lambda (kappa included) at the 16 accumulator positions;
  // ok: the entry lies inside F x N
  __device__ __forceinline__ void tile(const bool (&ok)[16], const float (&v)[16], const float (&l)[16],
                                       double& sum) {
    const int lane = threadIdx.x & 63;
    float z[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) z[r] = ok[r] ? l[r] : 0.f;
#pragma unroll
    for (int w = 8; w >= 1; w >>= 1)
#pragma unroll
      for (int r = 0; r < w; ++r) z[r] += z[r + w];
    sum += (double)z[0];
    int nnz = 0;
    if (dense) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const bool nz = ok[r] && v[r] > 0.f;
        nnz += __popcll(__ballot(nz));
        const double t = kl_nz((double)v[r], (double)l[r]);
        sum += nz ? t : 0.0;
      }
    } else {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
#pragma unroll
        for (int r = 8 * h; r < 8 * h + 8; ++r) {
          const bool nz = ok[r] && v[r] > 0.f;
          const unsigned long long m = __ballot(nz);
          const int below = __builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
          const int pos = nz ? qn + below : kKlQueue + lane;
          qv[pos] = v[r];
          ql[pos] = l[r];
          const int c = __popcll(m);
          qn += c;
          nnz += c;
        }
        if (qn >= 64) rounds(sum);
      }
    }
    dense = nnz >= kTile * kTile / 2;
  }

  __device__ __forceinline__ void drain(double& sum) {
    const int lane = threadIdx.x & 63;
    wave_lds_sync();
    if (lane < qn) sum += kl_nz((double)qv[lane], (double)ql[lane]);
    qn = 0;
    wave_lds_sync();
  }
};

// LDS of a rows item: two staged H~ tiles, then each wave's KL queue
template <int KB>
constexpr int rows_item_lds() { return 2 * 32 * KB * kHS * 4 + kWaves * 2 * kKlSlots * 4; }
template <int KB>
__device__ __forceinline__ KlQueue kl_queue_of(float* lds, int wave) {
  float* const q = lds + 2 * 32 * KB * kHS + wave * 2 * kKlSlots;
  return KlQueue{q, q + kKlSlots, 0, true};
}

// ---------------------------------------------------------------------------
// W update applied by a rows item of a problem whose rows take one column group
// (its accumulators hold the whole W-step contractions of rows f0 .. f0 + 31 of
// its wave): W_new, and chi_1, chi_2 in joint mode or the transposed W_new in
// alternating mode, as update_w_rows writes them, with the same float64
// arithmetic.  ROWSUM: the beta = 1 denominator is the row sums of H~ (rsum, as
// the rows item accumulates them), gathered per k through LDS.  With u->pcol set
// it also writes the column sums of W_new^2 and W_new over the item's 128 rows
// to u->pcol[rb][2][KP].  Every thread of the workgroup calls it, after the
// item's last barrier.
// ---------------------------------------------------------------------------
template <int KB, bool ROWSUM, bool WT_TILDE, bool C0_TILDE, class UPtr>
__device__ __forceinline__ void finish_w_rows(const SweepRowsArgs& a, UPtr u, const f32x16 (&accN)[KB],
                                              const f32x16 (&accD)[KB], const float (&rsum)[KB], float* lds,
                                              int rb, int f0, bool wave_on) {
  constexpr int KP = 32 * KB;
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, hi = lane >> 5;
  const int K = a.K;
  // the beta = 1 denominator: row sums of H~ over all N (this item's single
  // group), gathered per k through LDS
  float* const rs_s = lds;  // [KP]
  if (ROWSUM) {
    __syncthreads();  // the staged tiles are no longer read
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      float x = rsum[j];
      x += __shfl_xor(x, 1, 64);
      x += __shfl_xor(x, 2, 64);
      x += __shfl_xor(x, 4, 64);
      const int e4 = tid + kBlock * j;
      if ((e4 & 7) == 0) rs_s[e4 >> 3] = x;
    }
    __syncthreads();
  }
  double csq[KB], csm[KB];  // this lane's column sums of W_new^2 and W_new
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) { csq[kb] = 0.0; csm[kb] = 0.0; }
  if (wave_on) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int k = kb * 32 + li;
      const bool kok = k < K;
      const double den1 = ROWSUM ? (double)rs_s[k] : 0.0;
      float wt[16], wn[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int f = f0 + acc_row(r, hi);
        wt[r] = ldz(u->W, (int64_t)f * u->ldw + k, f < a.F && kok);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int f = f0 + acc_row(r, hi);
        float w1 = 0.f, c1 = 0.f, c2 = 0.f;
        if (f < a.F && kok) {
          const double num = (double)accN[kb][r];
          const double den = ROWSUM ? den1 : (double)accD[kb][r];
          const double ratio = num / den;
          if (!(den > 0.0) || !isfinite(ratio)) set_flag(u->flags, 1u);
          const double rr = pow_gamma(ratio, u->gamma);
          const double w0 = (double)wt[r];
          const double wnew = w0 * rr;
          w1 = (float)wnew;
          if (u->joint) chi_terms(u->beta, w0, rr, wnew, c1, c2);
        }
        wn[r] = w1;
        if (f < a.F) {
          const int64_t o = (int64_t)f * KP + k;
          u->Wn[o] = w1;
          if (u->joint) { u->C1[o] = c1; u->C2[o] = c2; }
          if (C0_TILDE) u->C0[o] = wt[r];
        }
        csq[kb] += (double)w1 * (double)w1;
        csm[kb] += (double)w1;
      }
      if (WT_TILDE || !u->joint) {
        // the transposed factor that forms Lambda in the H pass: W~^T
        // (WT_TILDE: joint MM re-forming Lambda~) or W_new^T; registers
        // 4q..4q+3 are four consecutive rows of one column
        const float* const tr = WT_TILDE ? wt : wn;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int fb = f0 + 8 * q + 4 * hi;
          float* const dst = u->WT + (int64_t)k * u->ldt + fb;
          if (fb + 3 < a.F) {
            *reinterpret_cast<float4*>(dst) = make_float4(tr[4 * q], tr[4 * q + 1], tr[4 * q + 2], tr[4 * q + 3]);
          } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              if (fb + i < a.F) dst[i] = tr[4 * q + i];
          }
        }
      }
    }
  }
  if (u->pcol) {
    // lanes hi = 0, 1 hold the same column; the four waves' sums are added
    // in wave order through LDS (rows past F hold W_new = 0)
    double* const cs = reinterpret_cast<double*>(lds + 2 * KP);  // [kWaves][2][KP]
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const double q2 = csq[kb] + __shfl_xor(csq[kb], 32, 64);
      const double q1 = csm[kb] + __shfl_xor(csm[kb], 32, 64);
      if (hi == 0) {
        cs[(wave * 2 + 0) * KP + kb * 32 + li] = q2;
        cs[(wave * 2 + 1) * KP + kb * 32 + li] = q1;
      }
    }
    __syncthreads();
    if (tid < 2 * KP) {
      const int part = tid / KP, k = tid % KP;
      double t = 0.0;
#pragma unroll
      for (int w = 0; w < kWaves; ++w) t += cs[(w * 2 + part) * KP + k];
      u->pcol[(int64_t)rb * 2 * KP + tid] = t;
    }
  }
}

// ---------------------------------------------------------------------------
// H update applied by one wave of a cols item of a problem whose columns take
// one row group (its accumulators hold the whole H-step contractions of columns
// n0w .. n0w + 31), in place, as update_h_cols_multi computes it: H_new = H~
// (num/den)^gamma, times the column norm of W_new when normalizing, with den =
// the column sums of W_new at beta = 1; norm_s / csum_s hold those norms and
// sums.  No other item reads these columns of H~.
// ---------------------------------------------------------------------------
template <int KB, class UHPtr>
__device__ __forceinline__ void finish_h_cols(const SweepColsArgs& a, UHPtr uh, const f32x16 (&accN)[KB],
                                              const f32x16 (&accD)[KB], const float* norm_s, const float* csum_s,
                                              int n0w) {
  const int lane = threadIdx.x & 63;
  const int li = lane & 31, hi = lane >> 5;
  const int K = a.K;
  float* const Hw = uh->H;
  const int64_t ldh = uh->ldh;
  const bool h4 = ((uintptr_t)Hw % 16 == 0) && (ldh % 4 == 0);
  const int N = a.N;
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
    const int k = kb * 32 + li;
    const bool kok = k < K;
    double nk = 1.0;
    if (uh->normalize && kok) {
      const float x = norm_s[k];
      if (x > 0.f) nk = (double)x;
    }
    const double den1 = uh->beta_one && kok ? (double)csum_s[k] : 0.0;
    // H~ at the accumulator positions: registers 4q..4q+3 are columns
    // n0w + 8q + 4hi + 0..3 of row k
    float hv[16];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int nb = n0w + 8 * q + 4 * hi;
      const int64_t o = (int64_t)k * ldh + nb;
      if (h4 && nb + 3 < N) {
        const float4 x = ldc4(Hw, o, kok);
        hv[4 * q + 0] = x.x; hv[4 * q + 1] = x.y; hv[4 * q + 2] = x.z; hv[4 * q + 3] = x.w;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) hv[4 * q + j] = ldc(Hw, o + j, kok && nb + j < N);
      }
    }
    float hn[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int n = n0w + acc_row(r, hi);
      hn[r] = 0.f;
      if (kok && n < N) {
        const double num = (double)accN[kb][r];
        const double dd = uh->beta_one ? den1 : (double)accD[kb][r];
        const double ratio = num / dd;
        if (!(dd > 0.0) || !isfinite(ratio)) set_flag(uh->flags, 1u);
        hn[r] = (float)((double)hv[r] * (pow_gamma(ratio, uh->gamma) * nk));
      }
    }
    if (kok) {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int nb = n0w + 8 * q + 4 * hi;
        float* const dst = Hw + (int64_t)k * ldh + nb;
        if (h4 && nb + 3 < N) {
          *reinterpret_cast<float4*>(dst) = make_float4(hn[4 * q], hn[4 * q + 1], hn[4 * q + 2], hn[4 * q + 3]);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j)
            if (nb + j < N) dst[j] = hn[4 * q + j];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// rows item: W-step contractions (reduction over n) for 128 rows of V over the
// column tiles of one group.  Optional objective terms (added to objsum), and
// optionally P and Q stored tile by tile ([tile][n][f], tile = ti * NT + tj) for
// a later H pass that reuses them (joint MM: V~ and its element-wise terms are
// formed once per outer iteration).
// ---------------------------------------------------------------------------
// FINISH (one column group: the item's accumulators hold the whole W-step
// contractions of its rows): the item applies the W update itself
// (finish_w_rows) instead of writing partials; `u` points to the update's
// arguments (read where they are used).  WT_TILDE: the transposed factor it
// writes is W~ (joint MM whose H pass forms Lambda~ again).
template <int BC, int KB, int KIND, bool OBJ, bool STORE_PQ, bool FINISH = false, bool WT_TILDE = false,
          class UPtr = const UpdateWArgs*>
__device__ __forceinline__ void rows_item(const SweepRowsArgs& a, int item, float* lds, double& objsum,
                                          UPtr u = nullptr) {
  constexpr int KP = 32 * KB;
  constexpr int K2MAX = KP / 2;
  constexpr bool CONTRACT = (KIND != KIND_OBJ);
  constexpr bool NEED_DEN = (KIND == KIND_UPDATE) && (BC != BC_B1) && (BC != BC_B2G);
  constexpr bool ROWSUM = (KIND == KIND_UPDATE) && (BC == BC_B1);
  // Gram form at beta = 2: P = V needs no Lambda; it is formed for the objective only
  constexpr bool NEED_LAM = !(BC == BC_B2G && KIND == KIND_UPDATE && !OBJ);
  float* const Hs0 = lds;
  float* const Hs1 = lds + KP * kHS;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, hi = lane >> 5;
  const int rb = item / a.n_groups, g = item % a.n_groups;
  const int f0 = rb * kBlockRows + wave * kTile;
  const int frow = f0 + li;
  const bool frow_ok = frow < a.F;
  const bool wave_on = f0 < a.F;
  const int K = a.K, N = a.N;
  const int K2 = (K + 1) >> 1;
  KlQueue klq = kl_queue_of<KB>(lds, wave);

  // B operand of Lambda^T = H~^T W~^T: lane holds W~[frow][2s + hi]
  // (all loads issued before any is masked, so they are in flight together)
  float wB[K2MAX];
#pragma unroll
  for (int s = 0; s < K2MAX; ++s) wB[s] = ldc(a.W, (int64_t)frow * a.ldw + 2 * s + hi, frow_ok && 2 * s + hi < K);
#pragma unroll
  for (int s = 0; s < K2MAX; ++s) wB[s] = (frow_ok && 2 * s + hi < K) ? wB[s] : 0.f;
  f32x16 accN[KB], accD[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) { accN[kb][r] = 0.f; accD[kb][r] = 0.f; }
  }
  float rsum[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) rsum[j] = 0.f;

  // staging of the H~ tile: thread float4 j covers row (tid + 256 j) / 8,
  // columns 4 ((tid + 256 j) % 8) .. + 3
  // Out-of-range entries (k >= K or n >= N) hold finite values from inside H~:
  // they meet zero weights (wB, or P = Q = 0) and only feed unused outputs.
  auto load_h = [&](int n0, float4 (&r)[KB]) {
    const bool full = a.hvec && n0 + kTile <= N;  // whole tile in range: 16-byte loads
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e4 = tid + kBlock * j;
      const int k = e4 >> 3, n = n0 + 4 * (e4 & 7);
      const int64_t o = (int64_t)k * a.ldh + n;
      if (full) {
        r[j] = ldc4(a.H, o, k < K);
      } else {
        r[j].x = ldc(a.H, o + 0, k < K && n + 0 < N);
        r[j].y = ldc(a.H, o + 1, k < K && n + 1 < N);
        r[j].z = ldc(a.H, o + 2, k < K && n + 2 < N);
        r[j].w = ldc(a.H, o + 3, k < K && n + 3 < N);
      }
    }
  };
  // exact zeros outside K x N for the beta = 1 row sums
  auto masked_sum = [&](int n0, const float4& x, int j) {
    const int e4 = tid + kBlock * j;
    const int k = e4 >> 3, n = n0 + 4 * (e4 & 7);
    if (k >= K) return 0.f;
    return (n + 0 < N ? x.x : 0.f) + (n + 1 < N ? x.y : 0.f) + (n + 2 < N ? x.z : 0.f) + (n + 3 < N ? x.w : 0.f);
  };
  auto store_h = [&](float* buf, const float4 (&r)[KB]) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e4 = tid + kBlock * j;
      *reinterpret_cast<float4*>(&buf[(e4 >> 3) * kHS + 4 * (e4 & 7)]) = r[j];
    }
  };
  const int64_t vrow = (int64_t)frow * a.ldv;
  // V at the accumulator positions: registers 4q..4q+3 are columns n0 + 8q + 4hi + 0..3
  // (out-of-range entries are finite stand-ins; P and Q are zeroed there)
  auto load_v = [&](int n0, float (&v)[16]) {
    const bool full = a.vec4 && n0 + kTile <= N;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int nb = n0 + 8 * q + 4 * hi;
      if (full) {
        const float4 x = a.vstream ? ldc4_nt(a.V, vrow + nb, frow_ok) : ldc4(a.V, vrow + nb, frow_ok);
        v[4 * q + 0] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool ok = frow_ok && nb + j < N;
          v[4 * q + j] = a.vstream ? ldc_nt(a.V, vrow + nb + j, ok) : ldc(a.V, vrow + nb + j, ok);
        }
      }
    }
  };

  const int nt_total = (N + kTile - 1) / kTile;
  const int t0 = g * a.tiles_per_group;
  const int t1 = min(nt_total, t0 + a.tiles_per_group);
  float4 hreg[KB];
  float vcur[16], vnext[16];
  __syncthreads();  // LDS may still be read by the previous item
  if (t0 < t1) {
    load_h(t0 * kTile, hreg);
    if (ROWSUM)
#pragma unroll
      for (int j = 0; j < KB; ++j) rsum[j] += masked_sum(t0 * kTile, hreg[j], j);
    if (wave_on) load_v(t0 * kTile, vcur);
    store_h(Hs0, hreg);
  }
  __syncthreads();

  for (int t = t0; t < t1; ++t) {
    const float* hs = ((t - t0) & 1) ? Hs1 : Hs0;
    const bool more = t + 1 < t1;
    if (more) {
      load_h((t + 1) * kTile, hreg);
      if (wave_on) load_v((t + 1) * kTile, vnext);
    }
    if (wave_on) {
      const int n0 = t * kTile;
      // Lambda^T tile: lam[r] = Lambda[frow][n0 + acc_row(r, hi)]; A operand H~[2s+hi][n0+li]
      f32x16 lam;
#pragma unroll
      for (int r = 0; r < 16; ++r) lam[r] = 0.f;
      if (NEED_LAM) {
        // operands read one block of 4 steps ahead; blocks past K2 skipped
        float av[4], an[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) av[j] = hs[(2 * j + hi) * kHS + li];
#pragma unroll
        for (int b = 0; b < K2MAX / 4; ++b) {
          if (b + 1 < K2MAX / 4)
#pragma unroll
            for (int j = 0; j < 4; ++j) an[j] = hs[(2 * (4 * b + 4 + j) + hi) * kHS + li];
          if (4 * b < K2)
#pragma unroll
            for (int j = 0; j < 4; ++j) lam = mfma32(av[j], wB[4 * b + j], lam);
#pragma unroll
          for (int j = 0; j < 4; ++j) av[j] = an[j];
        }
      }

      float P[16], Q[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int n = n0 + acc_row(r, hi);
        const bool ok = frow_ok && n < N;
        const float lk = lam[r] + a.kappa;
        const float vk = vcur[r] + a.kappa;
        if (KIND == KIND_UPDATE) {
          beta_terms<BC>(vk, lk, a.bm2, P[r], Q[r]);
          if (!ok) { P[r] = 0.f; Q[r] = 0.f; }
        } else if (KIND == KIND_GRAD) {
          P[r] = ok ? pow_bm2<BC>(lk, a.bm2) * (lam[r] - vcur[r]) : 0.f;
        }
        if (OBJ && BC != BC_B1) {
          const double d = d_beta<BC>((double)vk, (double)lk, a.beta);
          objsum += ok ? d : 0.0;
        }
      }
      if (OBJ && BC == BC_B1) {
        bool okr[16];
        float vk[16], lk[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          okr[r] = frow_ok && n0 + acc_row(r, hi) < N;
          vk[r] = vcur[r] + a.kappa;
          lk[r] = lam[r] + a.kappa;
        }
        klq.tile(okr, vk, lk, objsum);
      }
      if (STORE_PQ) {
        // tile (slab of this wave, column tile t) as [n][f]: coalesced 32-float rows
        const int64_t tb = ((int64_t)(f0 >> 5) * a.NT + t) * (kTile * kTile);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t o = tb + acc_row(r, hi) * kTile + li;
          if (BC != BC_B2) a.Pst[o] = P[r];  // beta = 2: P is V itself, read again from V
          if (BC != BC_B1) a.Qst[o] = Q[r];
        }
      }
      if (CONTRACT) {
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            // B operand: H~[kb*32 + li][n0 + 8q + 4hi + j]
            const float4 b = *reinterpret_cast<const float4*>(&hs[(kb * 32 + li) * kHS + 8 * q + 4 * hi]);
            accN[kb] = mfma32(P[4 * q + 0], b.x, accN[kb]);
            accN[kb] = mfma32(P[4 * q + 1], b.y, accN[kb]);
            accN[kb] = mfma32(P[4 * q + 2], b.z, accN[kb]);
            accN[kb] = mfma32(P[4 * q + 3], b.w, accN[kb]);
            if (NEED_DEN) {
              accD[kb] = mfma32(Q[4 * q + 0], b.x, accD[kb]);
              accD[kb] = mfma32(Q[4 * q + 1], b.y, accD[kb]);
              accD[kb] = mfma32(Q[4 * q + 2], b.z, accD[kb]);
              accD[kb] = mfma32(Q[4 * q + 3], b.w, accD[kb]);
            }
          }
        }
      }
    }
    if (more) {
      store_h(((t - t0 + 1) & 1) ? Hs1 : Hs0, hreg);
      if (ROWSUM)
#pragma unroll
        for (int j = 0; j < KB; ++j) rsum[j] += masked_sum((t + 1) * kTile, hreg[j], j);
#pragma unroll
      for (int i = 0; i < 16; ++i) vcur[i] = vnext[i];
    }
    __syncthreads();
  }

  if (OBJ && BC == BC_B1 && wave_on) klq.drain(objsum);
  if constexpr (FINISH) {
    finish_w_rows<KB, ROWSUM, WT_TILDE, false>(a, u, accN, accD, rsum, lds, rb, f0, wave_on);
    return;
  }
  if (CONTRACT && wave_on) {
    // accumulator (i = row offset f, j = li = column k); each wave owns its rows
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int f = f0 + acc_row(r, hi);
        if (f < a.F) {
          const int64_t o = ((int64_t)g * a.F + f) * KP + kb * 32 + li;
          a.pnum[o] = accN[kb][r];
          if (NEED_DEN) a.pden[o] = accD[kb][r];
        }
      }
    }
  }
  if (ROWSUM) {
    // the eight threads sharing a row of the staged tile hold its column sums
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      float x = rsum[j];
      x += __shfl_xor(x, 1, 64);
      x += __shfl_xor(x, 2, 64);
      x += __shfl_xor(x, 4, 64);
      const int e4 = tid + kBlock * j;
      if (rb == 0 && (e4 & 7) == 0) a.prs[g * KP + (e4 >> 3)] = x;
    }
  }
}

// ---------------------------------------------------------------------------
// rows item of a later joint sub-iteration (Algorithm 2, l > 1): the W-step
// contractions P chi_1(H_l, H~)^T and Q chi_2(H_l, H~)^T over the P, Q tiles kept
// by the first W pass (P = V + kappa re-read at beta = 2; Q = 1 at beta = 1,
// where the denominator is the row sums of chi_2).  No V~ is formed.  a.H holds
// chi_1 (K x N, ld a.ldh) and a.Pst / a.Qst the kept tiles; a.W (ld a.ldw)
// holds chi_2.  Partials as rows_item writes them.
// ---------------------------------------------------------------------------
template <int KB>
constexpr int rows_pq_item_lds() { return 4 * 32 * KB * kHS * 4; }

template <int BC, int KB>
__device__ __forceinline__ void rows_pq_item(const SweepRowsArgs& a, int item, float* lds) {
  constexpr int KP = 32 * KB;
  constexpr bool NEED_DEN = (BC != BC_B1);
  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, hi = lane >> 5;
  const int rb = item / a.n_groups, g = item % a.n_groups;
  const int f0 = rb * kBlockRows + wave * kTile;
  const int frow = f0 + li;
  const bool frow_ok = frow < a.F;
  const bool wave_on = f0 < a.F;
  const int K = a.K, N = a.N;
  const float* const X1 = a.H;  // chi_1, ld a.ldh
  const float* const X2 = a.W;  // chi_2, ld a.ldw
  // staged tiles: [buffer][chi_1, chi_2][KP][kHS]
  auto stage = [&](int b, int m) { return lds + (2 * b + m) * KP * kHS; };

  f32x16 accN[KB], accD[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) { accN[kb][r] = 0.f; accD[kb][r] = 0.f; }
  }
  float rsum[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) rsum[j] = 0.f;

  // thread float4 j of a [KP][32] tile covers row (tid + 256 j) / 8, columns
  // 4 ((tid + 256 j) % 8) .. + 3; entries outside K x N are finite stand-ins
  // (they meet P = Q = 0) or exact zeros in the row sums
  auto load_x = [&](const float* X, int64_t ldx, int n0, float4 (&r)[KB]) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e4 = tid + kBlock * j;
      const int k = e4 >> 3, n = n0 + 4 * (e4 & 7);
      const int64_t o = (int64_t)k * ldx + n;
      r[j].x = ldc(X, o + 0, k < K && n + 0 < N);
      r[j].y = ldc(X, o + 1, k < K && n + 1 < N);
      r[j].z = ldc(X, o + 2, k < K && n + 2 < N);
      r[j].w = ldc(X, o + 3, k < K && n + 3 < N);
    }
  };
  auto masked_sum = [&](int n0, const float4& x, int j) {
    const int e4 = tid + kBlock * j;
    const int k = e4 >> 3, n = n0 + 4 * (e4 & 7);
    if (k >= K) return 0.f;
    return (n + 0 < N ? x.x : 0.f) + (n + 1 < N ? x.y : 0.f) + (n + 2 < N ? x.z : 0.f) + (n + 3 < N ? x.w : 0.f);
  };
  auto store_x = [&](float* buf, const float4 (&r)[KB]) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e4 = tid + kBlock * j;
      *reinterpret_cast<float4*>(&buf[(e4 >> 3) * kHS + 4 * (e4 & 7)]) = r[j];
    }
  };
  // P, Q of tile (slab of this wave, column tile t) at the accumulator positions
  auto load_pq = [&](int t, float (&P)[16], float (&Q)[16]) {
    const int64_t tb = ((int64_t)(f0 >> 5) * a.NT + t) * (kTile * kTile);
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int64_t o = tb + acc_row(r, hi) * kTile + li;
      if (BC == BC_B2) {
        const int n = t * kTile + acc_row(r, hi);
        const bool ok = frow_ok && n < N;
        P[r] = ok ? ldc(a.V, (int64_t)frow * a.ldv + n, ok) + a.kappa : 0.f;
      } else {
        P[r] = a.Pst[o];
      }
      Q[r] = NEED_DEN ? a.Qst[o] : 0.f;
    }
  };

  const int nt_total = (N + kTile - 1) / kTile;
  const int t0 = g * a.tiles_per_group;
  const int t1 = min(nt_total, t0 + a.tiles_per_group);
  float4 x1[KB], x2[KB];
  float P[16], Q[16], Pn[16], Qn[16];
  __syncthreads();  // LDS may still be read by the previous item
  if (t0 < t1) {
    load_x(X1, a.ldh, t0 * kTile, x1);
    load_x(X2, a.ldw, t0 * kTile, x2);
    if (wave_on) load_pq(t0, P, Q);
    if (!NEED_DEN)
#pragma unroll
      for (int j = 0; j < KB; ++j) rsum[j] += masked_sum(t0 * kTile, x2[j], j);
    store_x(stage(0, 0), x1);
    store_x(stage(0, 1), x2);
  }
  __syncthreads();
  for (int t = t0; t < t1; ++t) {
    const int b = (t - t0) & 1;
    const bool more = t + 1 < t1;
    if (more) {
      load_x(X1, a.ldh, (t + 1) * kTile, x1);
      load_x(X2, a.ldw, (t + 1) * kTile, x2);
      if (wave_on) load_pq(t + 1, Pn, Qn);
    }
    if (wave_on) {
      const float* s1 = stage(b, 0);
      const float* s2 = stage(b, 1);
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float4 c = *reinterpret_cast<const float4*>(&s1[(kb * 32 + li) * kHS + 8 * q + 4 * hi]);
          accN[kb] = mfma32(P[4 * q + 0], c.x, accN[kb]);
          accN[kb] = mfma32(P[4 * q + 1], c.y, accN[kb]);
          accN[kb] = mfma32(P[4 * q + 2], c.z, accN[kb]);
          accN[kb] = mfma32(P[4 * q + 3], c.w, accN[kb]);
          if (NEED_DEN) {
            const float4 d = *reinterpret_cast<const float4*>(&s2[(kb * 32 + li) * kHS + 8 * q + 4 * hi]);
            accD[kb] = mfma32(Q[4 * q + 0], d.x, accD[kb]);
            accD[kb] = mfma32(Q[4 * q + 1], d.y, accD[kb]);
            accD[kb] = mfma32(Q[4 * q + 2], d.z, accD[kb]);
            accD[kb] = mfma32(Q[4 * q + 3], d.w, accD[kb]);
          }
        }
      }
    }
    if (more) {
      store_x(stage(b ^ 1, 0), x1);
      store_x(stage(b ^ 1, 1), x2);
      if (!NEED_DEN)
#pragma unroll
        for (int j = 0; j < KB; ++j) rsum[j] += masked_sum((t + 1) * kTile, x2[j], j);
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        P[r] = Pn[r];
        Q[r] = Qn[r];
      }
    }
    __syncthreads();
  }

  if (wave_on) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int f = f0 + acc_row(r, hi);
        if (f < a.F) {
          const int64_t o = ((int64_t)g * a.F + f) * KP + kb * 32 + li;
          a.pnum[o] = accN[kb][r];
          if (NEED_DEN) a.pden[o] = accD[kb][r];
        }
      }
    }
  }
  if (!NEED_DEN) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      float x = rsum[j];
      x += __shfl_xor(x, 1, 64);
      x += __shfl_xor(x, 2, 64);
      x += __shfl_xor(x, 4, 64);
      const int e4 = tid + kBlock * j;
      if (rb == 0 && (e4 & 7) == 0) a.prs[g * KP + (e4 >> 3)] = x;
    }
  }
}

// ---------------------------------------------------------------------------
// Low-precision products (bfloat16 or float16 operands, float32 accumulation)
// with v_mfma_f32_32x32x16_{bf16,f16}: lane (li, hi) supplies A[li][8hi..8hi+7]
// and B[8hi..8hi+7][li]; the accumulator layout is the float32 one, so eight
// consecutive accumulator registers (rows acc_row(8s + e, hi)) form the A
// operand of a product contracting over those rows.
// Lambda is formed as hi*hi + lo*hi + hi*lo of split operands (x = hi + lo,
// both rounded to nearest even), accurate to about 2^-16 relative, so P, Q and
// the objective are computed from an almost float32 Lambda; the W- and H-step
// contractions take single low-precision operands.
// ---------------------------------------------------------------------------
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <class T> struct LowP;
template <> struct LowP<__bf16> {
  typedef bf16x8 v8;
  static __device__ __forceinline__ f32x16 mfma(v8 a, v8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
};
template <> struct LowP<_Float16> {
  typedef f16x8 v8;
  static __device__ __forceinline__ f32x16 mfma(v8 a, v8 b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
};

// float16 operands must stay within the float16 range: ok is cleared when a
// value about to be converted is larger than the largest finite float16 (or not
// finite).  bfloat16 has the float32 range and needs no check.
template <class T>
__device__ __forceinline__ void range_check(const float (&x)[8], bool& ok) {
  if constexpr (__is_same(T, _Float16)) {
#pragma unroll
    for (int e = 0; e < 8; ++e) ok = ok && (__builtin_fabsf(x[e]) <= 65504.f);
  }
}

template <class T>
__device__ __forceinline__ typename LowP<T>::v8 to_low(const float (&x)[8]) {
  typename LowP<T>::v8 r;
#pragma unroll
  for (int e = 0; e < 8; ++e) r[e] = (T)x[e];
  return r;
}
template <class T>
__device__ __forceinline__ void split_low(const float (&x)[8], typename LowP<T>::v8& h, typename LowP<T>::v8& l) {
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const T t = (T)x[e];
    h[e] = t;
    l[e] = (T)(x[e] - (float)t);
  }
}

// rows item with low-precision products (update kind).  The H~ tile is staged
// in LDS in float32 as in rows_item; operands are converted when read.  FINISH
// and `u` as in rows_item; C0_TILDE: the W update also writes the row-major
// copy of W~ (u->C0) that forms Lambda~ again in a low-precision joint H pass.
template <int BC, int KB, bool OBJ, class T, bool STORE_PQ = false, bool FINISH = false, bool C0_TILDE = false,
          class UPtr = const UpdateWArgs*>
__device__ __forceinline__ void rows_item_lp(const SweepRowsArgs& a, int item, float* lds, double& objsum,
                                             UPtr u = nullptr) {
  typedef typename LowP<T>::v8 v8;
  constexpr int KP = 32 * KB;
  constexpr int KS = KP / 16;  // 16-deep steps of Lambda
  constexpr bool NEED_DEN = (BC != BC_B1);
  constexpr bool ROWSUM = (BC == BC_B1);
  float* const Hs0 = lds;
  float* const Hs1 = lds + KP * kHS;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, hi = lane >> 5;
  const int rb = item / a.n_groups, g = item % a.n_groups;
  const int f0 = rb * kBlockRows + wave * kTile;
  const int frow = f0 + li;
  const bool frow_ok = frow < a.F;
  const bool wave_on = f0 < a.F;
  const int K = a.K, N = a.N;
  KlQueue klq = kl_queue_of<KB>(lds, wave);

  bool rok = true;
  // B operand of Lambda^T: lane holds W~[frow][16s + 8hi + e], split in two
  v8 wBh[KS], wBl[KS];
  {
    float w[KS][8];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 16 * s + 8 * hi + e;
        w[s][e] = ldc(a.W, (int64_t)frow * a.ldw + k, frow_ok && k < K);
      }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
      for (int e = 0; e < 8; ++e) w[s][e] = (frow_ok && 16 * s + 8 * hi + e < K) ? w[s][e] : 0.f;
      range_check<T>(w[s], rok);
      split_low<T>(w[s], wBh[s], wBl[s]);
    }
  }
  f32x16 accN[KB], accD[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) { accN[kb][r] = 0.f; accD[kb][r] = 0.f; }
  }
  float rsum[KB];
#pragma unroll
  for (int j = 0; j < KB; ++j) rsum[j] = 0.f;

  auto load_h = [&](int n0, float4 (&r)[KB]) {
    const bool full = a.hvec && n0 + kTile <= N;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e4 = tid + kBlock * j;
      const int k = e4 >> 3, n = n0 + 4 * (e4 & 7);
      const int64_t o = (int64_t)k * a.ldh + n;
      if (full) {
        r[j] = ldc4(a.H, o, k < K);
      } else {
        r[j].x = ldc(a.H, o + 0, k < K && n + 0 < N);
        r[j].y = ldc(a.H, o + 1, k < K && n + 1 < N);
        r[j].z = ldc(a.H, o + 2, k < K && n + 2 < N);
        r[j].w = ldc(a.H, o + 3, k < K && n + 3 < N);
      }
    }
  };
  // rows k >= K must be exact zeros here: Lambda's split products do not
  // multiply them by a zero weight in every term
  auto store_h = [&](float* buf, int n0, const float4 (&r)[KB]) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e4 = tid + kBlock * j;
      const int k = e4 >> 3, n = n0 + 4 * (e4 & 7);
      float4 x = r[j];
      if (k >= K) x = make_float4(0.f, 0.f, 0.f, 0.f);
      x.x = n + 0 < N ? x.x : 0.f;
      x.y = n + 1 < N ? x.y : 0.f;
      x.z = n + 2 < N ? x.z : 0.f;
      x.w = n + 3 < N ? x.w : 0.f;
      if (ROWSUM) rsum[j] += (x.x + x.y) + (x.z + x.w);
      *reinterpret_cast<float4*>(&buf[k * kHS + 4 * (e4 & 7)]) = x;
    }
  };
  const int64_t vrow = (int64_t)frow * a.ldv;
  auto load_v = [&](int n0, float (&v)[16]) {
    const bool full = a.vec4 && n0 + kTile <= N;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int nb = n0 + 8 * q + 4 * hi;
      if (full) {
        const float4 x = a.vstream ? ldc4_nt(a.V, vrow + nb, frow_ok) : ldc4(a.V, vrow + nb, frow_ok);
        v[4 * q + 0] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const bool ok = frow_ok && nb + j < N;
          v[4 * q + j] = a.vstream ? ldc_nt(a.V, vrow + nb + j, ok) : ldc(a.V, vrow + nb + j, ok);
        }
      }
    }
  };

  const int nt_total = (N + kTile - 1) / kTile;
  const int t0 = g * a.tiles_per_group;
  const int t1 = min(nt_total, t0 + a.tiles_per_group);
  float4 hreg[KB];
  float vcur[16], vnext[16];
  __syncthreads();
  if (t0 < t1) {
    load_h(t0 * kTile, hreg);
    if (wave_on) load_v(t0 * kTile, vcur);
    store_h(Hs0, t0 * kTile, hreg);
  }
  __syncthreads();

  for (int t = t0; t < t1; ++t) {
    const float* hs = ((t - t0) & 1) ? Hs1 : Hs0;
    const bool more = t + 1 < t1;
    if (more) {
      load_h((t + 1) * kTile, hreg);
      if (wave_on) load_v((t + 1) * kTile, vnext);
    }
    if (wave_on) {
      const int n0 = t * kTile;
      f32x16 lam;
#pragma unroll
      for (int r = 0; r < 16; ++r) lam[r] = 0.f;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        // A operand H~^T[n0+li][16s + 8hi + e] = H~[16s + 8hi + e][n0 + li]
        float x[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) x[e] = hs[(16 * s + 8 * hi + e) * kHS + li];
        v8 ah, al;
        split_low<T>(x, ah, al);
        lam = LowP<T>::mfma(ah, wBh[s], lam);
        lam = LowP<T>::mfma(al, wBh[s], lam);
        lam = LowP<T>::mfma(ah, wBl[s], lam);
      }
      float P[16], Q[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int n = n0 + acc_row(r, hi);
        const bool ok = frow_ok && n < N;
        const float lk = lam[r] + a.kappa;
        const float vk = vcur[r] + a.kappa;
        beta_terms<BC>(vk, lk, a.bm2, P[r], Q[r]);
        if (!ok) { P[r] = 0.f; Q[r] = 0.f; }
        if (OBJ && BC != BC_B1) {
          const double d = d_beta<BC>((double)vk, (double)lk, a.beta);
          objsum += ok ? d : 0.0;
        }
      }
      if (OBJ && BC == BC_B1) {
        bool okr[16];
        float vk[16], lk[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          okr[r] = frow_ok && n0 + acc_row(r, hi) < N;
          vk[r] = vcur[r] + a.kappa;
          lk[r] = lam[r] + a.kappa;
        }
        klq.tile(okr, vk, lk, objsum);
      }
      if (STORE_PQ) {
        // P, Q in the product type, tile-major [n][f] as the float32 path keeps them
        T* const Pl = reinterpret_cast<T*>(a.Pst);
        T* const Ql = reinterpret_cast<T*>(a.Qst);
        const int64_t tb = ((int64_t)(f0 >> 5) * a.NT + t) * (kTile * kTile);
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int64_t o = tb + acc_row(r, hi) * kTile + li;
          if (BC != BC_B2) Pl[o] = (T)P[r];
          if (NEED_DEN) Ql[o] = (T)Q[r];
        }
      }
#pragma unroll
      for (int st = 0; st < 2; ++st) {
        float pa[8], qa[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) { pa[e] = P[8 * st + e]; qa[e] = Q[8 * st + e]; }
        range_check<T>(pa, rok);
        if (NEED_DEN) range_check<T>(qa, rok);
        const v8 pv = to_low<T>(pa);
        const v8 qv = to_low<T>(qa);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          // B operand H~[kb*32 + li][n0 + acc_row(8 st + e, hi)]: columns 16 st + 4hi + {0..3, 8..11}
          const float* row = &hs[(kb * 32 + li) * kHS + 16 * st + 4 * hi];
          const float4 b0 = *reinterpret_cast<const float4*>(row);
          const float4 b1 = *reinterpret_cast<const float4*>(row + 8);
          const float bx[8] = {b0.x, b0.y, b0.z, b0.w, b1.x, b1.y, b1.z, b1.w};
          range_check<T>(bx, rok);
          const v8 bv = to_low<T>(bx);
          accN[kb] = LowP<T>::mfma(pv, bv, accN[kb]);
          if (NEED_DEN) accD[kb] = LowP<T>::mfma(qv, bv, accD[kb]);
        }
      }
    }
    if (more) {
      store_h(((t - t0 + 1) & 1) ? Hs1 : Hs0, (t + 1) * kTile, hreg);
#pragma unroll
      for (int i = 0; i < 16; ++i) vcur[i] = vnext[i];
    }
    __syncthreads();
  }

  if (OBJ && BC == BC_B1 && wave_on) klq.drain(objsum);
  if (!rok) set_flag(a.flags, 8u);  // operand outside the float16 range
  if constexpr (FINISH) {
    finish_w_rows<KB, ROWSUM, false, C0_TILDE>(a, u, accN, accD, rsum, lds, rb, f0, wave_on);
    return;
  }
  if (wave_on) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int f = f0 + acc_row(r, hi);
        if (f < a.F) {
          const int64_t o = ((int64_t)g * a.F + f) * KP + kb * 32 + li;
          a.pnum[o] = accN[kb][r];
          if (NEED_DEN) a.pden[o] = accD[kb][r];
        }
      }
    }
  }
  if (ROWSUM) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      float x = rsum[j];
      x += __shfl_xor(x, 1, 64);
      x += __shfl_xor(x, 2, 64);
      x += __shfl_xor(x, 4, 64);
      const int e4 = tid + kBlock * j;
      if (rb == 0 && (e4 & 7) == 0) a.prs[g * KP + (e4 >> 3)] = x;
    }
  }
}

// LDS bytes of a low-precision cols item: the Lambda-forming factor tile and
// chi_1 (and chi_2), row-major [32][KP + 4], double-buffered.
template <int KB, bool C2_TILE>
constexpr int cols_item_lp_lds() {
  return 2 * kTile * (32 * KB + 4) * (C2_TILE ? 3 : 2) * 4;
}

// cols item with low-precision products (update kind).  The factor forming
// Lambda is read row-major (C0, ld KP): W~ (joint) or W_new (alternating, then
// C0 == C1 and its tile is staged once).  FINISH, uh, norm_s and csum_s as in
// cols_item.
template <int BC, int KB, bool DUAL, class T, bool FINISH = false, class UHPtr = const UpdateHArgs*>
__device__ __forceinline__ void cols_item_lp(const SweepColsArgs& a, int item, float* lds, UHPtr uh = nullptr,
                                             const float* norm_s = nullptr, const float* csum_s = nullptr) {
  typedef typename LowP<T>::v8 v8;
  constexpr int KP = 32 * KB;
  constexpr int KS = KP / 16;
  constexpr int CS = KP + 4;
  constexpr bool NEED_DEN = (BC != BC_B1);
  constexpr bool C2_TILE = DUAL && NEED_DEN;
  constexpr int NT_ = C2_TILE ? 3 : 2;  // staged tiles per buffer (C0, C1[, C2]); C0 unused when !DUAL
  float* const base0 = lds;
  float* const base1 = lds + NT_ * kTile * CS;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, hi = lane >> 5;
  const int cb = item / a.f_groups, g = item % a.f_groups;
  const int n0w = cb * kBlockRows + wave * kTile;
  const int ncol = n0w + li;
  const bool ncol_ok = ncol < a.N;
  const bool wave_on = n0w < a.N;
  const int K = a.K, F = a.F;

  bool rok = true;
  // B operand of Lambda = W H~: lane holds H~[16s + 8hi + e][ncol], split
  v8 hBh[KS], hBl[KS];
  {
    float h[KS][8];
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int k = 16 * s + 8 * hi + e;
        h[s][e] = ldc(a.H, (int64_t)k * a.ldh + ncol, ncol_ok && k < K);
      }
#pragma unroll
    for (int s = 0; s < KS; ++s) {
#pragma unroll
      for (int e = 0; e < 8; ++e) h[s][e] = (ncol_ok && 16 * s + 8 * hi + e < K) ? h[s][e] : 0.f;
      range_check<T>(h[s], rok);
      split_low<T>(h[s], hBh[s], hBl[s]);
    }
  }
  f32x16 accN[KB], accD[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) { accN[kb][r] = 0.f; accD[kb][r] = 0.f; }
  }

  // staged tiles: [0] factor forming Lambda (C0; == C1 when !DUAL), [1] chi_1, [2] chi_2
  float4 treg[NT_][KB];
  const float* src[3] = {DUAL ? a.C0 : a.C1, a.C1, a.C2};
  auto load_tiles = [&](int f0) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e4 = tid + kBlock * j;
      const int i = e4 / (KP / 4), c = 4 * (e4 % (KP / 4));
      const bool ok = f0 + i < F;
      const int64_t o = (int64_t)(f0 + i) * KP + c;
#pragma unroll
      for (int m = (DUAL ? 0 : 1); m < NT_; ++m) treg[m][j] = ldc4(src[m], o, ok);
    }
  };
  // rows f >= F staged as zeros (the Lambda split products need exact zeros)
  auto store_tiles = [&](float* base, int f0) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e4 = tid + kBlock * j;
      const int i = e4 / (KP / 4), c = 4 * (e4 % (KP / 4));
      const bool ok = f0 + i < F;
#pragma unroll
      for (int m = (DUAL ? 0 : 1); m < NT_; ++m)
        *reinterpret_cast<float4*>(&base[m * kTile * CS + i * CS + c]) = ok ? treg[m][j] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto load_v = [&](int f0, float (&v)[16]) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int f = f0 + acc_row(r, hi);
      v[r] = ldc(a.V, (int64_t)f * a.ldv + ncol, ncol_ok && f < F);
    }
  };

  const int ft_total = (F + kTile - 1) / kTile;
  const int t0 = g * a.tiles_per_group;
  const int t1 = min(ft_total, t0 + a.tiles_per_group);
  float vcur[16], vnext[16];
  __syncthreads();
  if (t0 < t1) {
    load_tiles(t0 * kTile);
    if (wave_on) load_v(t0 * kTile, vcur);
    store_tiles(base0, t0 * kTile);
  }
  __syncthreads();

  for (int t = t0; t < t1; ++t) {
    const float* base = ((t - t0) & 1) ? base1 : base0;
    const bool more = t + 1 < t1;
    if (more) {
      load_tiles((t + 1) * kTile);
      if (wave_on) load_v((t + 1) * kTile, vnext);
    }
    if (wave_on) {
      const int f0 = t * kTile;
      const float* w0 = base + (DUAL ? 0 : 1) * kTile * CS;
      const float* c1s = base + kTile * CS;
      const float* c2s = C2_TILE ? base + 2 * kTile * CS : c1s;
      f32x16 lam;
#pragma unroll
      for (int r = 0; r < 16; ++r) lam[r] = 0.f;
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        // A operand W[f0 + li][16s + 8hi + e]
        const float* row = &w0[li * CS + 16 * s + 8 * hi];
        const float4 x0 = *reinterpret_cast<const float4*>(row);
        const float4 x1 = *reinterpret_cast<const float4*>(row + 4);
        const float x[8] = {x0.x, x0.y, x0.z, x0.w, x1.x, x1.y, x1.z, x1.w};
        if (DUAL) range_check<T>(x, rok);
        v8 ah, al;
        split_low<T>(x, ah, al);
        lam = LowP<T>::mfma(ah, hBh[s], lam);
        lam = LowP<T>::mfma(al, hBh[s], lam);
        lam = LowP<T>::mfma(ah, hBl[s], lam);
      }
      float P[16], Q[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int f = f0 + acc_row(r, hi);
        const bool ok = ncol_ok && f < F;
        beta_terms<BC>(vcur[r] + a.kappa, lam[r] + a.kappa, a.bm2, P[r], Q[r]);
        if (!ok) { P[r] = 0.f; Q[r] = 0.f; }
      }
#pragma unroll
      for (int st = 0; st < 2; ++st) {
        float pa[8], qa[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) { pa[e] = P[8 * st + e]; qa[e] = Q[8 * st + e]; }
        range_check<T>(pa, rok);
        if (NEED_DEN) range_check<T>(qa, rok);
        const v8 pv = to_low<T>(pa);
        const v8 qv = to_low<T>(qa);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          float b1[8], b2[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int row = acc_row(8 * st + e, hi) * CS + kb * 32 + li;
            b1[e] = c1s[row];
            b2[e] = c2s[row];
          }
          range_check<T>(b1, rok);
          if (NEED_DEN) range_check<T>(b2, rok);
          accN[kb] = LowP<T>::mfma(pv, to_low<T>(b1), accN[kb]);
          if (NEED_DEN) accD[kb] = LowP<T>::mfma(qv, to_low<T>(b2), accD[kb]);
        }
      }
    }
    if (more) {
      store_tiles(((t - t0 + 1) & 1) ? base1 : base0, (t + 1) * kTile);
#pragma unroll
      for (int i = 0; i < 16; ++i) vcur[i] = vnext[i];
    }
    __syncthreads();
  }

  if (!rok) set_flag(a.flags, 8u);  // operand outside the float16 range
  if constexpr (FINISH) {
    if (wave_on) finish_h_cols<KB>(a, uh, accN, accD, norm_s, csum_s, n0w);
    return;
  }
  if (wave_on) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int n = n0w + acc_row(r, hi);
        if (n < a.N) {
          const int64_t o = ((int64_t)g * a.N + n) * KP + kb * 32 + li;
          a.pnum[o] = accN[kb][r];
          if (NEED_DEN) a.pden[o] = accD[kb][r];
        }
      }
    }
  }
}

// Column sums of W_new^2 and W_new over rows [f0, f1) of the row-major W_new
// (ld KP), in float64 and a fixed order -> out[0..KP) and out[KP..2KP).  Done
// by a few workgroups of the H pass, so the H update reads a handful of partial
// rows instead of one per W-update workgroup.
template <int KB>
__device__ __forceinline__ void column_partials(const float* Wn, int f0, int f1, double* out, double* scratch) {
  constexpr int KP = 32 * KB;
  constexpr int R = kBlock / KP;
  constexpr int U = 4;
  const int tid = threadIdx.x;
  const int k = tid % KP, part = tid / KP;
  double x = 0.0, y = 0.0;
  int f = f0 + part;
  for (; f + (U - 1) * R < f1; f += U * R) {
    float w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) w[u] = Wn[(int64_t)(f + u * R) * KP + k];
#pragma unroll
    for (int u = 0; u < U; ++u) { x += (double)w[u] * (double)w[u]; y += (double)w[u]; }
  }
  for (; f < f1; f += R) {
    const double w = (double)Wn[(int64_t)f * KP + k];
    x += w * w;
    y += w;
  }
  __syncthreads();
  scratch[tid] = x;
  scratch[kBlock + tid] = y;
  __syncthreads();
  if (tid < KP) {
    double xs = 0.0, ys = 0.0;
    for (int j = 0; j < R; ++j) { xs += scratch[j * KP + tid]; ys += scratch[kBlock + j * KP + tid]; }
    out[tid] = xs;
    out[KP + tid] = ys;
  }
  __syncthreads();
}

// H-pass prologue: the workgroups of the first col_parts column blocks write
// the column partials of their share of the rows (see SweepColsArgs).
template <int KB>
__device__ __forceinline__ void cols_prologue(const SweepColsArgs& a, int item, float* lds) {
  if (!a.pcol) return;
  const int cb = item / a.f_groups, g = item % a.f_groups;
  if (cb >= a.col_parts) return;
  const int gf0 = g * a.tiles_per_group * kTile;
  const int gf1 = min(a.F, gf0 + a.tiles_per_group * kTile);
  const int f0 = min(gf1, gf0 + cb * a.col_chunk);
  const int f1 = min(gf1, f0 + a.col_chunk);
  column_partials<KB>(a.Wn, f0, f1, a.pcol + (int64_t)(g * a.col_parts + cb) * 2 * 32 * KB,
                      reinterpret_cast<double*>(lds));
}

// cols item of the joint H pass with low-precision products contracting the
// P, Q tiles the W pass kept in the product type (no Lambda~, no powers): lane
// (li, hi) reads, for column n0w + li, the eight rows acc_row(8 st + e, hi) of
// step st as two 4-entry runs.  At beta = 2, P = V + kappa is read from V.
// FINISH, uh, norm_s and csum_s as in cols_item.
template <int BC, int KB, class T, bool FINISH = false, class UHPtr = const UpdateHArgs*>
__device__ __forceinline__ void cols_item_lp_pq(const SweepColsArgs& a, int item, float* lds, UHPtr uh = nullptr,
                                                const float* norm_s = nullptr, const float* csum_s = nullptr) {
  typedef typename LowP<T>::v8 v8;
  constexpr int KP = 32 * KB;
  constexpr int CS = KP + 4;
  constexpr bool NEED_DEN = (BC != BC_B1);
  constexpr int NT_ = NEED_DEN ? 2 : 1;  // staged tiles per buffer: chi_1[, chi_2]
  float* const base0 = lds;
  float* const base1 = lds + NT_ * kTile * CS;
  typedef T t4 __attribute__((ext_vector_type(4)));

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, hi = lane >> 5;
  const int cb = item / a.f_groups, g = item % a.f_groups;
  const int n0w = cb * kBlockRows + wave * kTile;
  const int ncol = n0w + li;
  const bool ncol_ok = ncol < a.N;
  const bool wave_on = n0w < a.N;
  const int F = a.F;
  bool rok = true;

  f32x16 accN[KB], accD[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) { accN[kb][r] = 0.f; accD[kb][r] = 0.f; }
  }
  float4 treg[NT_][KB];
  const float* src[2] = {a.C1, a.C2};
  auto load_tiles = [&](int f0) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e4 = tid + kBlock * j;
      const int i = e4 / (KP / 4), c = 4 * (e4 % (KP / 4));
      const bool ok = f0 + i < F;
      const int64_t o = (int64_t)(f0 + i) * KP + c;
#pragma unroll
      for (int m = 0; m < NT_; ++m) treg[m][j] = ldc4(src[m], o, ok);
    }
  };
  auto store_tiles = [&](float* base) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e4 = tid + kBlock * j;
      const int i = e4 / (KP / 4), c = 4 * (e4 % (KP / 4));
#pragma unroll
      for (int m = 0; m < NT_; ++m) *reinterpret_cast<float4*>(&base[m * kTile * CS + i * CS + c]) = treg[m][j];
    }
  };
  // kept tiles: 4-entry runs of P, Q in the product type, or V at beta = 2 for P
  struct Kept {
    t4 p[4], q[4];
    float v[16];
  };
  auto load_kept = [&](int f0, Kept& x) {
    const int64_t tb = ((int64_t)(f0 >> 5) * a.NT + (n0w >> 5)) * (kTile * kTile) + li * kTile;
    const T* Pl = reinterpret_cast<const T*>(a.Pst);
    const T* Ql = reinterpret_cast<const T*>(a.Qst);
#pragma unroll
    for (int st = 0; st < 2; ++st) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int64_t o = tb + 16 * st + 8 * h + 4 * hi;
        if (BC != BC_B2) x.p[2 * st + h] = *reinterpret_cast<const t4*>(Pl + o);
        if (NEED_DEN) x.q[2 * st + h] = *reinterpret_cast<const t4*>(Ql + o);
      }
    }
    if (BC == BC_B2) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int f = f0 + acc_row(r, hi);
        x.v[r] = ldc(a.V, (int64_t)f * a.ldv + ncol, ncol_ok && f < F);
      }
    }
  };

  const int ft_total = (F + kTile - 1) / kTile;
  const int t0 = g * a.tiles_per_group;
  const int t1 = min(ft_total, t0 + a.tiles_per_group);
  Kept cur, nxt;
  __syncthreads();
  if (t0 < t1) {
    load_tiles(t0 * kTile);
    if (wave_on) load_kept(t0 * kTile, cur);
    store_tiles(base0);
  }
  __syncthreads();

  for (int t = t0; t < t1; ++t) {
    const float* base = ((t - t0) & 1) ? base1 : base0;
    const bool more = t + 1 < t1;
    if (more) {
      load_tiles((t + 1) * kTile);
      if (wave_on) load_kept((t + 1) * kTile, nxt);
    }
    if (wave_on) {
      const int f0 = t * kTile;
      const float* c1s = base;
      const float* c2s = NEED_DEN ? base + kTile * CS : base;
#pragma unroll
      for (int st = 0; st < 2; ++st) {
        v8 pv, qv;
        if (BC == BC_B2) {
          float pa[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int r = 8 * st + e;
            const bool ok = ncol_ok && f0 + acc_row(r, hi) < F;
            pa[e] = ok ? cur.v[r] + a.kappa : 0.f;
          }
          range_check<T>(pa, rok);
          pv = to_low<T>(pa);
        } else {
          pv = __builtin_shufflevector(cur.p[2 * st], cur.p[2 * st + 1], 0, 1, 2, 3, 4, 5, 6, 7);
        }
        if (NEED_DEN) qv = __builtin_shufflevector(cur.q[2 * st], cur.q[2 * st + 1], 0, 1, 2, 3, 4, 5, 6, 7);
#pragma unroll
        for (int kb = 0; kb < KB; ++kb) {
          float b1[8], b2[8];
#pragma unroll
          for (int e = 0; e < 8; ++e) {
            const int row = acc_row(8 * st + e, hi) * CS + kb * 32 + li;
            b1[e] = c1s[row];
            b2[e] = c2s[row];
          }
          range_check<T>(b1, rok);
          if (NEED_DEN) range_check<T>(b2, rok);
          accN[kb] = LowP<T>::mfma(pv, to_low<T>(b1), accN[kb]);
          if (NEED_DEN) accD[kb] = LowP<T>::mfma(qv, to_low<T>(b2), accD[kb]);
        }
      }
    }
    if (more) {
      store_tiles(((t - t0 + 1) & 1) ? base1 : base0);
      cur = nxt;
    }
    __syncthreads();
  }

  if (!rok) set_flag(a.flags, 8u);  // operand outside the float16 range
  if constexpr (FINISH) {
    if (wave_on) finish_h_cols<KB>(a, uh, accN, accD, norm_s, csum_s, n0w);
    return;
  }
  if (wave_on) {
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int n = n0w + acc_row(r, hi);
        if (n < a.N) {
          const int64_t o = ((int64_t)g * a.N + n) * KP + kb * 32 + li;
          a.pnum[o] = accN[kb][r];
          if (NEED_DEN) a.pden[o] = accD[kb][r];
        }
      }
    }
  }
}

// LDS bytes a cols item needs.
template <int KB, bool C2_TILE>
constexpr int cols_item_lds() {
  return (2 * 32 * KB * kHS + 2 * kTile * (32 * KB + 4) * (C2_TILE ? 2 : 1)) * 4;
}

// ---------------------------------------------------------------------------
// cols item: H-step contractions (reduction over f) for 128 columns over the
// row tiles of one group.  Per tile the workgroup stages (LDS, double
// buffered) the transposed factor forming Lambda (KP x 32 from WT, unless
// LOAD_PQ) and chi_1, chi_2 (32 x KP, row-major with ld KP).  With LOAD_PQ the
// element-wise terms P, Q come from the tiles a rows item stored (no Lambda
// re-formation, no V pass).
// FINISH (one row group: the accumulators hold the whole H-step contractions of
// the item's columns): the item applies the H update to its columns in place,
// as update_h_cols_multi does, from the accumulators and the column norms and
// sums of W_new in norm_s / csum_s; `uh` points to the update's arguments.
// ---------------------------------------------------------------------------
template <int BC, int KB, int KIND, bool DUAL, bool LOAD_PQ, bool FINISH = false,
          class UHPtr = const UpdateHArgs*>
__device__ __forceinline__ void cols_item(const SweepColsArgs& a, int item, float* lds, UHPtr uh = nullptr,
                                          const float* norm_s = nullptr, const float* csum_s = nullptr) {
  constexpr int KP = 32 * KB;
  constexpr int K2MAX = KP / 2;
  constexpr int CS = KP + 4;  // LDS row stride of [f][KP] tiles
  constexpr bool NEED_DEN = (KIND == KIND_UPDATE) && (BC != BC_B1) && (BC != BC_B2G);
  constexpr bool C2_TILE = DUAL && NEED_DEN;
  // Lambda is formed from the staged factor unless P, Q are read (kept tiles)
  // or P = V needs no Lambda (Gram form at beta = 2)
  constexpr bool USE_LAM = !LOAD_PQ && (BC != BC_B2G);
  float* const Ws0 = lds;
  float* const Ws1 = lds + KP * kHS;
  float* const C1s0 = lds + 2 * KP * kHS;
  float* const C1s1 = C1s0 + kTile * CS;
  float* const C2s0 = C1s1 + kTile * CS;
  float* const C2s1 = C2s0 + kTile * CS;

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, hi = lane >> 5;
  const int cb = item / a.f_groups, g = item % a.f_groups;
  const int n0w = cb * kBlockRows + wave * kTile;
  const int ncol = n0w + li;
  const bool ncol_ok = ncol < a.N;
  const bool wave_on = n0w < a.N;
  const int K = a.K, F = a.F;
  const int K2 = (K + 1) >> 1;

  // B operand of Lambda = W H~: lane holds H~[2s + hi][ncol]
  float hB[USE_LAM ? K2MAX : 1];
  if (USE_LAM) {
#pragma unroll
    for (int s = 0; s < K2MAX; ++s) hB[s] = ldc(a.H, (int64_t)(2 * s + hi) * a.ldh + ncol, ncol_ok && 2 * s + hi < K);
#pragma unroll
    for (int s = 0; s < K2MAX; ++s) hB[s] = (ncol_ok && 2 * s + hi < K) ? hB[s] : 0.f;
  }
  f32x16 accN[KB], accD[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) { accN[kb][r] = 0.f; accD[kb][r] = 0.f; }
  }

  // staging: WT tile float4 j -> row k = e4 / 8, columns f0 + 4 (e4 % 8);
  //          chi tile float4 j -> row i = e4 / (KP/4), columns 4 (e4 % (KP/4))
  float4 wreg[USE_LAM ? KB : 1], c1reg[KB], c2reg[C2_TILE ? KB : 1];
  auto load_tiles = [&](int f0) {
    const bool full = f0 + kTile <= F;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e4 = tid + kBlock * j;
      if (USE_LAM) {
        const int k = e4 >> 3, f = f0 + 4 * (e4 & 7);
        const int64_t o = (int64_t)k * a.ldwt + f;
        if (full) {
          wreg[j] = ldc4(a.WT, o, true);
        } else {
          wreg[j].x = ldc(a.WT, o + 0, f + 0 < F);
          wreg[j].y = ldc(a.WT, o + 1, f + 1 < F);
          wreg[j].z = ldc(a.WT, o + 2, f + 2 < F);
          wreg[j].w = ldc(a.WT, o + 3, f + 3 < F);
        }
      }
      const int i = e4 / (KP / 4), c = 4 * (e4 % (KP / 4));
      const bool ok = f0 + i < F;
      const int64_t o = (int64_t)(f0 + i) * KP + c;
      c1reg[j] = ldc4(a.C1, o, ok);  // rows f >= F meet P = Q = 0
      if (C2_TILE) c2reg[j] = ldc4(a.C2, o, ok);
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e4 = tid + kBlock * j;
      if (USE_LAM) *reinterpret_cast<float4*>(&(buf ? Ws1 : Ws0)[(e4 >> 3) * kHS + 4 * (e4 & 7)]) = wreg[j];
      const int i = e4 / (KP / 4), c = 4 * (e4 % (KP / 4));
      *reinterpret_cast<float4*>(&(buf ? C1s1 : C1s0)[i * CS + c]) = c1reg[j];
      if (C2_TILE) *reinterpret_cast<float4*>(&(buf ? C2s1 : C2s0)[i * CS + c]) = c2reg[j];
    }
  };
  // per-wave tile data at the accumulator positions (register r: row
  // f0 + acc_row(r, hi), column ncol): V, or the stored P and Q
  auto load_v = [&](int f0, float (&v)[16], float (&w)[16]) {
    if (LOAD_PQ) {
      const int64_t tb = ((int64_t)(f0 >> 5) * a.NT + (n0w >> 5)) * (kTile * kTile) + li * kTile;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        if (BC != BC_B2) {
          const float4 x = *reinterpret_cast<const float4*>(a.Pst + tb + 8 * q + 4 * hi);
          v[4 * q + 0] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
        }
        if (NEED_DEN) {
          const float4 y = *reinterpret_cast<const float4*>(a.Qst + tb + 8 * q + 4 * hi);
          w[4 * q + 0] = y.x; w[4 * q + 1] = y.y; w[4 * q + 2] = y.z; w[4 * q + 3] = y.w;
        }
      }
      if (BC == BC_B2) {  // P = V + kappa: read V (masked where it is consumed)
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int f = f0 + acc_row(r, hi);
          v[r] = ldc(a.V, (int64_t)f * a.ldv + ncol, ncol_ok && f < F);
        }
      }
    } else {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int f = f0 + acc_row(r, hi);
        v[r] = ldc(a.V, (int64_t)f * a.ldv + ncol, ncol_ok && f < F);
      }
    }
  };

  const int ft_total = (F + kTile - 1) / kTile;
  const int t0 = g * a.tiles_per_group;
  const int t1 = min(ft_total, t0 + a.tiles_per_group);
  float vcur[16], vnext[16], wcur[16], wnext[16];  // w*: stored Q (LOAD_PQ only)
  __syncthreads();  // LDS may still be read by the previous item
  if (t0 < t1) {
    load_tiles(t0 * kTile);
    if (wave_on) load_v(t0 * kTile, vcur, wcur);
    store_tiles(0);
  }
  __syncthreads();

  for (int t = t0; t < t1; ++t) {
    const int buf = (t - t0) & 1;
    const bool more = t + 1 < t1;
    if (more) {
      load_tiles((t + 1) * kTile);
      if (wave_on) load_v((t + 1) * kTile, vnext, wnext);
    }
    if (wave_on) {
      const int f0 = t * kTile;
      const float* c1s = buf ? C1s1 : C1s0;
      const float* c2s = C2_TILE ? (buf ? C2s1 : C2s0) : c1s;
      float P[16], Q[16];
      if (LOAD_PQ) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          if (BC == BC_B2) {
            const bool ok = ncol_ok && f0 + acc_row(r, hi) < F;
            P[r] = ok ? vcur[r] + a.kappa : 0.f;
          } else {
            P[r] = vcur[r];
          }
          Q[r] = NEED_DEN ? wcur[r] : 0.f;
        }
      } else if (!USE_LAM) {  // Gram form at beta = 2: P = V + kappa
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const bool ok = ncol_ok && f0 + acc_row(r, hi) < F;
          P[r] = ok ? vcur[r] + a.kappa : 0.f;
          Q[r] = 0.f;
        }
      } else {
        const float* ws = buf ? Ws1 : Ws0;
        // Lambda tile: lam[r] = Lambda[f0 + acc_row(r, hi)][ncol]; A operand W[f0+li][2s+hi]
        f32x16 lam;
#pragma unroll
        for (int r = 0; r < 16; ++r) lam[r] = 0.f;
        {
          float av[4], an[4];
#pragma unroll
          for (int j = 0; j < 4; ++j) av[j] = ws[(2 * j + hi) * kHS + li];
#pragma unroll
          for (int b = 0; b < K2MAX / 4; ++b) {
            if (b + 1 < K2MAX / 4)
#pragma unroll
              for (int j = 0; j < 4; ++j) an[j] = ws[(2 * (4 * b + 4 + j) + hi) * kHS + li];
            if (4 * b < K2)
#pragma unroll
              for (int j = 0; j < 4; ++j) lam = mfma32(av[j], hB[4 * b + j], lam);
#pragma unroll
            for (int j = 0; j < 4; ++j) av[j] = an[j];
          }
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int f = f0 + acc_row(r, hi);
          const bool ok = ncol_ok && f < F;
          const float lk = lam[r] + a.kappa;
          const float vk = vcur[r] + a.kappa;
          if (KIND == KIND_UPDATE) {
            beta_terms<BC>(vk, lk, a.bm2, P[r], Q[r]);
            if (!ok) { P[r] = 0.f; Q[r] = 0.f; }
          } else {
            P[r] = ok ? pow_bm2<BC>(lk, a.bm2) * (lam[r] - vcur[r]) : 0.f;
          }
        }
      }
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
          const int row = acc_row(r, hi) * CS + kb * 32 + li;
          accN[kb] = mfma32(P[r], c1s[row], accN[kb]);
          if (NEED_DEN) accD[kb] = mfma32(Q[r], c2s[row], accD[kb]);
        }
      }
    }
    if (more) {
      store_tiles(buf ^ 1);
#pragma unroll
      for (int i = 0; i < 16; ++i) vcur[i] = vnext[i];
      if (LOAD_PQ)
#pragma unroll
        for (int i = 0; i < 16; ++i) wcur[i] = wnext[i];
    }
    __syncthreads();
  }

  if constexpr (FINISH) {
    if (wave_on) finish_h_cols<KB>(a, uh, accN, accD, norm_s, csum_s, n0w);
    return;
  }
  if (wave_on) {
    // accumulator (i = column offset n, j = li = k); each wave owns its columns
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int n = n0w + acc_row(r, hi);
        if (n < a.N) {
          const int64_t o = ((int64_t)g * a.N + n) * KP + kb * 32 + li;
          a.pnum[o] = accN[kb][r];
          if (NEED_DEN) a.pden[o] = accD[kb][r];
        }
      }
    }
  }
}

// ---------------------------------------------------------------------------
// W update for one unit of kUnitRows(KB) rows: W_new = W~ (num/den)^gamma with
// the partials summed in a fixed order (four thread slices take every fourth
// group, combined slice 0..3 through LDS), the chi terms (joint), the
// transposed copy of the factor that forms Lambda in a later H pass (when
// `write_wt`), and running column sums of W_new^2 and W_new in (nrm, cs) for
// the normalization (threads of slice 0 only).
// ---------------------------------------------------------------------------
constexpr int kSlices = 4;
template <int KB, int SL = kSlices, int BT = kBlock>
constexpr int unit_rows() { return BT / (32 * KB * SL) > 0 ? BT / (32 * KB * SL) : 1; }
template <int KB, int SL = kSlices, int BT = kBlock>
constexpr int unit_slices() { return BT / (32 * KB * unit_rows<KB, SL, BT>()); }
template <int KB>
constexpr int update_w_lds_floats() { return 2 * kBlock; }

// SL: thread slices sharing a row's group sums (more slices: fewer rows per unit,
// shorter per-thread sums for many groups); BT: threads of the workgroup.  `lds`
// holds 2 * BT doubles.
template <int KB, int SL = kSlices, int BT = kBlock>
__device__ __forceinline__ void update_w_unit(const UpdateWArgs& a, int unit, bool write_wt, float* lds,
                                              double den1, double& nrm, double& cs) {
  constexpr int KP = 32 * KB;
  constexpr int RU = unit_rows<KB, SL, BT>();
  constexpr int GS = unit_slices<KB, SL, BT>();
  constexpr int U = 8;  // groups per round
  const int tid = threadIdx.x;
  const int k = tid % KP, r = (tid / KP) % RU, gs = tid / (KP * RU);
  const int f = unit * RU + r;
  const bool fok = f < a.F;
  const int64_t gstride = (int64_t)a.F * KP;
  const int64_t base = (int64_t)f * KP + k;
  const float wtf = ldz(a.W, (int64_t)f * a.ldw + k, fok && k < a.K);  // issued with the partial loads
  double dn = 0.0, dd = 0.0;
  int g = gs;
  for (; g + (U - 1) * GS < a.n_groups; g += U * GS) {
    float xn[U], xd[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      xn[u] = ldc(a.pnum, (int64_t)(g + u * GS) * gstride + base, fok);
      xd[u] = a.beta_one ? 0.f : ldc(a.pden, (int64_t)(g + u * GS) * gstride + base, fok);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) { dn += (double)xn[u]; dd += (double)xd[u]; }
  }
  if (g < a.n_groups) {  // the remaining groups in one round of predicated loads
    float xn[U], xd[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool gu = fok && g + u * GS < a.n_groups;
      xn[u] = ldc(a.pnum, (int64_t)(g + u * GS) * gstride + base, gu);
      xd[u] = a.beta_one ? 0.f : ldc(a.pden, (int64_t)(g + u * GS) * gstride + base, gu);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (g + u * GS < a.n_groups) { dn += (double)xn[u]; dd += (double)xd[u]; }
    }
  }
  double* red = reinterpret_cast<double*>(lds);  // [2][GS][RU*KP]
  __syncthreads();  // red may still be read by the previous unit
  red[tid] = dn;
  red[BT + tid] = dd;
  __syncthreads();
  if (gs == 0) {
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int j = 0; j < GS; ++j) {
      num += red[j * KP * RU + tid];
      den += red[BT + j * KP * RU + tid];
    }
    float wn = 0.f, c1 = 0.f, c2 = 0.f;
    if (fok && k < a.K) {
      double gden = 0.0;
      if (a.gram) {  // Gram form at beta = 2: (W~ (H~ H~^T))[f][k], eight terms in flight
        const float* wr = a.W + (int64_t)f * a.ldw;
        double g8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        int l = 0;
        for (; l + 8 <= a.K; l += 8) {
#pragma unroll
          for (int j = 0; j < 8; ++j) g8[j] = fma((double)wr[l + j], a.gram[(l + j) * KP + k], g8[j]);
        }
        for (; l < a.K; ++l) g8[0] = fma((double)wr[l], a.gram[l * KP + k], g8[0]);
        gden = ((g8[0] + g8[1]) + (g8[2] + g8[3])) + ((g8[4] + g8[5]) + (g8[6] + g8[7]));
      }
      const double dsum = a.beta_one ? den1 : (a.gram ? gden : den);
      const double ratio = num / dsum;
      if (!(dsum > 0.0) || !isfinite(ratio)) set_flag(a.flags, 1u);
      const double rr = pow_gamma(ratio, a.gamma);
      const double wt = (double)wtf;
      const double wnew = wt * rr;
      wn = (float)wnew;
      if (a.joint) chi_terms(a.beta, wt, rr, wnew, c1, c2);
      nrm += (double)wn * (double)wn;
      cs += (double)wn;
    }
    if (fok) {
      const int64_t o = (int64_t)f * KP + k;
      a.Wn[o] = wn;
      if (a.joint) { a.C1[o] = c1; a.C2[o] = c2; }
      if (a.C0) a.C0[o] = wtf;
      if (write_wt) a.WT[(int64_t)k * a.ldt + f] = a.joint ? wtf : wn;
    }
  }
}

// W update of rows [f0, f0 + R) with every load of the rows in flight at once
// (the batched step's W-update item): thread (r, k) owns rows f0 + r + i RU,
// i < R / RU (RU = kBlock / KP), and sums each row's partial groups in order in
// float64, so the result equals update_w_unit's.  With `write_wt` the factor
// that forms Lambda in the H pass (W~ joint, W_new alternating) is written to
// the transposed copy through LDS ([R][KP + 1] floats), 32 consecutive rows of
// one column per wave store.
template <int KB, int R>
__device__ __forceinline__ void update_w_rows(const UpdateWArgs& a, int f0, bool write_wt, double den1,
                                              float* lds) {
  constexpr int KP = 32 * KB;
  constexpr int RU = kBlock / KP;
  constexpr int PER = R / RU;
  static_assert(PER * RU == R, "rows per item");
  const int tid = threadIdx.x;
  const int k = tid % KP, r = tid / KP;
  const bool kok = k < a.K;
  const int64_t gstride = (int64_t)a.F * KP;
  float wt[PER];
  bool ok[PER];
  double num[PER], den[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int f = f0 + r + i * RU;
    ok[i] = f < a.F;
    wt[i] = ldz(a.W, (int64_t)f * a.ldw + k, ok[i] && kok);
    num[i] = 0.0;
    den[i] = 0.0;
  }
  for (int g = 0; g < a.n_groups; ++g) {
    float xn[PER], xd[PER];
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int64_t o = (int64_t)g * gstride + (int64_t)(f0 + r + i * RU) * KP + k;
      xn[i] = ldc(a.pnum, o, ok[i]);
      xd[i] = a.beta_one ? 0.f : ldc(a.pden, o, ok[i]);
    }
#pragma unroll
    for (int i = 0; i < PER; ++i) { num[i] += (double)xn[i]; den[i] += (double)xd[i]; }
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int f = f0 + r + i * RU;
    float wn = 0.f, c1 = 0.f, c2 = 0.f;
    if (ok[i] && kok) {
      const double dsum = a.beta_one ? den1 : den[i];
      const double ratio = num[i] / dsum;
      if (!(dsum > 0.0) || !isfinite(ratio)) set_flag(a.flags, 1u);
      const double rr = pow_gamma(ratio, a.gamma);
      const double w0 = (double)wt[i];
      const double wnew = w0 * rr;
      wn = (float)wnew;
      if (a.joint) chi_terms(a.beta, w0, rr, wnew, c1, c2);
    }
    if (ok[i]) {
      const int64_t o = (int64_t)f * KP + k;
      a.Wn[o] = wn;
      if (a.joint) { a.C1[o] = c1; a.C2[o] = c2; }
      if (a.C0) a.C0[o] = wt[i];
    }
    if (write_wt) lds[(r + i * RU) * (KP + 1) + k] = a.joint ? wt[i] : wn;
  }
  if (write_wt) {
    __syncthreads();
    for (int e = tid; e < KP * R; e += kBlock) {
      const int kk = e / R, j = e % R;
      if (f0 + j < a.F) a.WT[(int64_t)kk * a.ldt + f0 + j] = lds[j * (KP + 1) + kk];
    }
  }
}

// Sum over groups of the beta = 1 row-sum partials of H~ (the W-step denominator).
template <int KB>
__device__ __forceinline__ double row_sum_den(const UpdateWArgs& a) {
  constexpr int KP = 32 * KB;
  const int k = threadIdx.x % KP;
  double d = 0.0;
  if (a.beta_one && k < a.K)
    for (int g = 0; g < a.n_groups; ++g) d += (double)a.prs[g * KP + k];
  return d;
}

// The same with all BT threads of the workgroup: thread (k, j) sums groups
// j, j + BT / KP, ... and the slices are combined through `scratch` (BT doubles)
// in a fixed order, so every thread returns the total for its k.
template <int KB, int BT>
__device__ __forceinline__ double row_sum_den_wide(const UpdateWArgs& a, double* scratch) {
  constexpr int KP = 32 * KB;
  constexpr int SLICES = BT / KP;
  const int k = threadIdx.x % KP, j = threadIdx.x / KP;
  double d = 0.0;
  if (a.beta_one && k < a.K)
    for (int g = j; g < a.n_groups; g += SLICES) d += (double)a.prs[g * KP + k];
  __syncthreads();
  scratch[threadIdx.x] = d;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < SLICES; ++i) t += scratch[i * KP + k];
  __syncthreads();
  return t;
}

// Column norms / sums of W_new from per-block partials pcol[b][2][KP] (b <
// nblocks), summed in a fixed order into norm_s / csum_s (LDS, KP each).
template <int KB>
__device__ __forceinline__ void reduce_columns(const double* pcol, int nblocks, double* scratch, float* norm_s,
                                               float* csum_s) {
  constexpr int KP = 32 * KB;
  constexpr int R = kBlock / KP;
  constexpr int U = 8;
  const int tid = threadIdx.x;
  const int k = tid % KP, part = tid / KP;
  double x = 0.0, y = 0.0;
  int b = part;
  for (; b + (U - 1) * R < nblocks; b += U * R) {
    double xs[U], ys[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      xs[u] = pcol[(int64_t)(b + u * R) * 2 * KP + k];
      ys[u] = pcol[(int64_t)(b + u * R) * 2 * KP + KP + k];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) { x += xs[u]; y += ys[u]; }
  }
  for (; b < nblocks; b += R) {
    x += pcol[(int64_t)b * 2 * KP + k];
    y += pcol[(int64_t)b * 2 * KP + KP + k];
  }
  __syncthreads();
  scratch[tid] = x;
  scratch[kBlock + tid] = y;
  __syncthreads();
  if (tid < KP) {
    double xs = 0.0, ys = 0.0;
    for (int j = 0; j < R; ++j) { xs += scratch[j * KP + tid]; ys += scratch[kBlock + j * KP + tid]; }
    norm_s[tid] = (float)sqrt(xs);
    csum_s[tid] = (float)ys;
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// H update for one 32-column tile: H_new = H~ (num/den)^gamma (times the column
// norm of W_new when normalizing), with den = column sums of W_new at beta = 1.
// ---------------------------------------------------------------------------
template <int KB>
__device__ __forceinline__ void update_h_tile(const UpdateHArgs& a, int ntile, const float* norm_s,
                                              const float* csum_s, double* S /* [KP][33] */) {
  constexpr int KP = 32 * KB;
  constexpr int PER = kTile * KP / kBlock;
  const int tid = threadIdx.x;
  const int k = tid % KP;
  const int n0 = ntile * kTile;
  double num[PER], den[PER];
  sum_partials<PER>(a.pnum, a.beta_one ? nullptr : a.pden, a.f_groups, (int64_t)a.N * KP, (int64_t)n0 * KP,
                    (int64_t)(min(a.N - n0, kTile)) * KP, num, den);
  // H~ entries this thread rewrites (kk = e / 32, n = n0 + e % 32), loaded up front
  float hv[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = tid + i * kBlock;
    const int kk = e / kTile, n = n0 + e % kTile;
    hv[i] = ldc(a.H, (int64_t)kk * a.ldh + n, kk < a.K && n < a.N);
  }
  double nk = 1.0;
  if (a.normalize && k < a.K) {
    const float x = norm_s[k];
    if (x > 0.f) nk = (double)x;
  }
  __syncthreads();  // S may still be read by the previous tile
#pragma unroll 1
  for (int i = 0; i < PER; ++i) {
    const int e = tid + i * kBlock;
    const int nl = e / KP, n = n0 + nl;
    double s = 0.0;
    if (n < a.N && k < a.K) {
      const double dd = a.beta_one ? (double)csum_s[k] : den[i];
      const double ratio = num[i] / dd;
      if (!(dd > 0.0) || !isfinite(ratio)) set_flag(a.flags, 1u);
      s = pow_gamma(ratio, a.gamma) * nk;
    }
    S[k * 33 + nl] = s;
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int e = tid + i * kBlock;
    const int kk = e / kTile, nl = e % kTile, n = n0 + nl;
    if (kk < a.K && n < a.N) a.H[(int64_t)kk * a.ldh + n] = (float)((double)hv[i] * S[kk * 33 + nl]);
  }
}

// H update of column units [u0, u1) (unit u: columns u * kBlock / KP + c, one
// thread per (k, c)), M units at a time with all their loads in flight together
// (with few row groups each unit alone is one short load round trip).
template <int KB, int M>
__device__ __forceinline__ void update_h_cols_multi(const UpdateHArgs& a, int u0, int u1, const float* norm_s,
                                                    const float* csum_s) {
  constexpr int KP = 32 * KB;
  constexpr int UC = kBlock / KP;
  const int tid = threadIdx.x;
  const int k = tid % KP;
  const int64_t gstride = (int64_t)a.N * KP;
  double nk = 1.0;
  if (a.normalize && k < a.K) {
    const float x = norm_s[k];
    if (x > 0.f) nk = (double)x;
  }
  for (int ub = u0; ub < u1; ub += M) {
    int n[M];
    bool ok[M];
    float hv[M];
    double num[M], den[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      n[m] = (ub + m) * UC + tid / KP;
      ok[m] = ub + m < u1 && n[m] < a.N && k < a.K;
      hv[m] = ldc(a.H, (int64_t)k * a.ldh + n[m], ok[m]);
      num[m] = 0.0;
      den[m] = 0.0;
    }
    for (int g = 0; g < a.f_groups; ++g) {
      float xn[M], xd[M];
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const int64_t o = (int64_t)g * gstride + (int64_t)n[m] * KP + k;
        xn[m] = ldc(a.pnum, o, ok[m]);
        xd[m] = a.beta_one ? 0.f : ldc(a.pden, o, ok[m]);
      }
#pragma unroll
      for (int m = 0; m < M; ++m) { num[m] += (double)xn[m]; den[m] += (double)xd[m]; }
    }
#pragma unroll
    for (int m = 0; m < M; ++m) {
      if (!ok[m]) continue;
      const double dd = a.beta_one ? (double)csum_s[k] : den[m];
      const double ratio = num[m] / dd;
      if (!(dd > 0.0) || !isfinite(ratio)) set_flag(a.flags, 1u);
      a.H[(int64_t)k * a.ldh + n[m]] = (float)((double)hv[m] * (pow_gamma(ratio, a.gamma) * nk));
    }
  }
}

// W <- W_new / norm (or W_new), entries e0, e0 + stride, ...
template <int KB>
__device__ __forceinline__ void write_w(const UpdateHArgs& a, const float* norm_s, int64_t e0, int64_t stride) {
  constexpr int KP = 32 * KB;
  const int64_t total = (int64_t)a.F * a.K;
  for (int64_t e = e0; e < total; e += stride) {
    const int f = (int)(e / a.K), kk = (int)(e % a.K);
    float w = a.Wn[(int64_t)f * KP + kk];
    if (a.normalize) {
      const float x = norm_s[kk];
      if (x > 0.f) w = (float)((double)w / (double)x);
    }
    a.W[(int64_t)f * a.ldw + kk] = w;
  }
}

}  // namespace nmf
