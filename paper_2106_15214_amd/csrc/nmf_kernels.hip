// HIP kernels for beta-NMF multiplicative updates on gfx950 (MI355X).
//
// Data layout: V (F x N), W (F x K), H (K x N), all float32 row-major.
// Lambda = W H is formed tile by tile on the matrix cores
// (v_mfma_f32_32x32x2_f32) and never written to memory.
//
// Two orientations of the pass over V:
//  * sweep_rows: each wave owns 32 rows f of V and walks 32-column tiles; the
//    contraction over n (P H^T, Q H^T: the W step) accumulates in registers.
//    Lambda^T is formed so that the accumulator layout (lane -> f, register
//    -> n) is directly the A operand of the next product.
//  * sweep_cols: each wave owns 32 columns n and walks 32-row tiles; the
//    contraction over f (chi_1^T P, chi_2^T Q: the H step) accumulates in
//    registers.  Lambda is formed with lane -> n, register -> f.
// Each workgroup writes one partial per output entry for its range of the
// contracted index; update kernels reduce the partials in a fixed order
// (deterministic results) and apply the multiplicative updates.
#include "nmf_internal.h"

namespace nmf {

typedef float f32x16 __attribute__((ext_vector_type(16)));

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
  return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

// Row (or column) offset held in accumulator register r by lane half `hi` of a
// 32x32 MFMA result: rows 8*(r/4) + 4*hi + r%4.
__device__ __forceinline__ int acc_row(int r, int hi) { return 8 * (r >> 2) + 4 * hi + (r & 3); }

// Lambda^(beta-2) for a smoothed Lambda (> 0).
template <int BC>
__device__ __forceinline__ float pow_bm2(float lam, float bm2) {
  if (BC == BC_B2) return 1.f;
  if (BC == BC_B1) return __builtin_amdgcn_rcpf(lam);
  if (BC == BC_B0) { float r = __builtin_amdgcn_rcpf(lam); return r * r; }
  if (BC == BC_B05) { float s = __builtin_amdgcn_rsqf(lam); return s * s * s; }
  if (BC == BC_B15) return __builtin_amdgcn_rsqf(lam);
  return __builtin_amdgcn_exp2f(bm2 * __builtin_amdgcn_logf(lam));
}

// P = v * lam^(beta-2), Q = lam^(beta-1) (v and lam include kappa).
template <int BC>
__device__ __forceinline__ void beta_terms(float v, float lam, float bm2, float& P, float& Q) {
  if (BC == BC_B2) { P = v; Q = lam; return; }
  if (BC == BC_B1) { P = v * __builtin_amdgcn_rcpf(lam); Q = 1.f; return; }
  if (BC == BC_B0) { float r = __builtin_amdgcn_rcpf(lam); Q = r; P = v * r * r; return; }
  if (BC == BC_B05) { float s = __builtin_amdgcn_rsqf(lam); Q = s; P = v * (s * s * s); return; }
  if (BC == BC_B15) { float s = __builtin_amdgcn_rsqf(lam); P = v * s; Q = lam * s; return; }
  float e = __builtin_amdgcn_exp2f(bm2 * __builtin_amdgcn_logf(lam));
  P = v * e;
  Q = lam * e;
}

// General-beta term of eq. (beta-div) (kept out of line: three float64 pows).
__device__ __noinline__ double d_beta_general(double v, double l, double beta) {
  if (v > 0.0)
    return pow(v, beta) / (beta * (beta - 1.0)) + pow(l, beta) / beta - v * pow(l, beta - 1.0) / (beta - 1.0);
  return beta > 0.0 ? pow(l, beta) / beta : __builtin_inf();
}

// d_beta(v | l) in float64 (v, l include kappa), paper eq. (beta-div);
// v = 0 takes the limit of the expression.
template <int BC>
__device__ __forceinline__ double d_beta(double v, double l, double beta) {
  if (BC == BC_B2) { double t = v - l; return 0.5 * t * t; }
  if (BC == BC_B1) return v > 0.0 ? v * log(v / l) - v + l : l;
  if (BC == BC_B0) { double r = v / l; return r - log(r) - 1.0; }
  if (BC == BC_B05) { double sy = sqrt(l); return -4.0 * sqrt(v) + 2.0 * sy + 2.0 * v / sy; }
  if (BC == BC_B15) { double sy = sqrt(l); return v * sqrt(v) / 0.75 + l * sy / 1.5 - 2.0 * v * sy; }
  return d_beta_general(v, l, beta);
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
  if (lane == 0) red[wave] = x;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kWaves; ++w) s += red[w];
  __syncthreads();
  return s;
}

// ---------------------------------------------------------------------------
// sweep_rows: W-step contractions (reduction over n), optional objective.
// A workgroup's four waves own four consecutive 32-row slabs of V and walk the
// same 32-column tiles in lockstep.  The H~ tile (KP x 32) is staged in LDS by
// the whole workgroup, double-buffered; each wave prefetches its next V tile
// into registers while the matrix cores work on the current one.
// ---------------------------------------------------------------------------
constexpr int kHS = 36;  // LDS row stride of [k][32] tiles: float4 and dword reads conflict-free

template <int BC, int KB, int KIND, bool OBJ>
__global__ __launch_bounds__(kBlock, sweep_rows_occupancy(KB)) void sweep_rows_kernel(SweepRowsArgs a) {
  constexpr int KP = 32 * KB;
  constexpr int K2MAX = KP / 2;
  constexpr bool CONTRACT = (KIND != KIND_OBJ);
  constexpr bool NEED_DEN = (KIND == KIND_UPDATE) && (BC != BC_B1);
  constexpr bool ROWSUM = (KIND == KIND_UPDATE) && (BC == BC_B1);
  __shared__ __align__(16) float Hs[2][KP * kHS];
  __shared__ double dred[kWaves];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, hi = lane >> 5;
  const int rb = blockIdx.x / a.n_groups, g = blockIdx.x % a.n_groups;
  const int f0 = rb * (kWaves * kTile) + wave * kTile;
  const int frow = f0 + li;
  const bool frow_ok = frow < a.F;
  const bool wave_on = f0 < a.F;
  const int K = a.K, N = a.N;
  const int K2 = (K + 1) >> 1;

  // B operand of Lambda^T = H~^T W~^T: lane holds W~[frow][2s + hi]
  float wB[K2MAX];
#pragma unroll
  for (int s = 0; s < K2MAX; ++s) {
    const int k = 2 * s + hi;
    wB[s] = (frow_ok && k < K) ? a.W[(int64_t)frow * a.ldw + k] : 0.f;
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
  double objsum = 0.0;

  // cooperative staging of the H~ tile: thread float4 j covers row (tid + 256 j) / 8,
  // columns 4 * ((tid + 256 j) % 8) .. + 3
  auto load_h = [&](int n0, float4 (&r)[KB]) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e4 = tid + kBlock * j;
      const int k = e4 >> 3, n = n0 + 4 * (e4 & 7);
      const float* src = a.H + (int64_t)k * a.ldh + n;
      if (k < K && a.hvec && n + 3 < N) {
        r[j] = *reinterpret_cast<const float4*>(src);
      } else {
        r[j].x = (k < K && n + 0 < N) ? src[0] : 0.f;
        r[j].y = (k < K && n + 1 < N) ? src[1] : 0.f;
        r[j].z = (k < K && n + 2 < N) ? src[2] : 0.f;
        r[j].w = (k < K && n + 3 < N) ? src[3] : 0.f;
      }
    }
  };
  auto store_h = [&](float* buf, const float4 (&r)[KB]) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e4 = tid + kBlock * j;
      *reinterpret_cast<float4*>(&buf[(e4 >> 3) * kHS + 4 * (e4 & 7)]) = r[j];
    }
  };
  const float* vrow = a.V + (int64_t)frow * a.ldv;
  // V at the accumulator positions: registers 4q..4q+3 are columns n0 + 8q + 4hi + 0..3
  auto load_v = [&](int n0, float (&v)[16]) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int nb = n0 + 8 * q + 4 * hi;
      if (a.vec4 && frow_ok && nb + 3 < N) {
        const float4 x = *reinterpret_cast<const float4*>(vrow + nb);
        v[4 * q + 0] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
      } else {
#pragma unroll
        for (int j = 0; j < 4; ++j) v[4 * q + j] = (frow_ok && nb + j < N) ? vrow[nb + j] : 0.f;
      }
    }
  };

  const int nt_total = (N + kTile - 1) / kTile;
  const int t0 = g * a.tiles_per_group;
  const int t1 = min(nt_total, t0 + a.tiles_per_group);
  float4 hreg[KB];
  float vcur[16], vnext[16];
  if (t0 < t1) {
    load_h(t0 * kTile, hreg);
    if (ROWSUM)
#pragma unroll
      for (int j = 0; j < KB; ++j) rsum[j] += (hreg[j].x + hreg[j].y) + (hreg[j].z + hreg[j].w);
    if (wave_on) load_v(t0 * kTile, vcur);
    store_h(Hs[0], hreg);
  }
  __syncthreads();

  for (int t = t0; t < t1; ++t) {
    const float* hs = Hs[(t - t0) & 1];
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
#pragma unroll
      for (int s = 0; s < K2MAX; ++s)
        if (s < K2) lam = mfma32(hs[(2 * s + hi) * kHS + li], wB[s], lam);

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
        if (OBJ && ok) objsum += d_beta<BC>((double)vk, (double)lk, a.beta);
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
      store_h(Hs[(t - t0 + 1) & 1], hreg);
      if (ROWSUM)
#pragma unroll
        for (int j = 0; j < KB; ++j) rsum[j] += (hreg[j].x + hreg[j].y) + (hreg[j].z + hreg[j].w);
#pragma unroll
      for (int i = 0; i < 16; ++i) vcur[i] = vnext[i];
    }
    __syncthreads();
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
  if (OBJ) {
    const double sum = block_sum(objsum, dred);
    if (tid == 0) a.pobj[blockIdx.x] = sum;
  }
}

// ---------------------------------------------------------------------------
// sweep_cols: H-step contractions (reduction over f).  The four waves own four
// 32-column slabs and walk the same 32-row tiles in lockstep.  Per tile the
// workgroup stages, double-buffered in LDS: the transposed factor forming
// Lambda (KP x 32, from WT), chi_1 and chi_2 (32 x KP, row-major with ld KP).
// ---------------------------------------------------------------------------
template <int BC, int KB, int KIND, bool DUAL>
__global__ __launch_bounds__(kBlock, sweep_cols_occupancy(BC, KB, KIND, DUAL)) void sweep_cols_kernel(SweepColsArgs a) {
  constexpr int KP = 32 * KB;
  constexpr int K2MAX = KP / 2;
  constexpr int CS = KP + 4;  // LDS row stride of [f][KP] tiles
  constexpr bool NEED_DEN = (KIND == KIND_UPDATE) && (BC != BC_B1);
  constexpr bool C2_TILE = DUAL && NEED_DEN;
  __shared__ __align__(16) float Ws[2][KP * kHS];
  __shared__ __align__(16) float C1s[2][kTile * CS];
  __shared__ __align__(16) float C2s[C2_TILE ? 2 : 1][C2_TILE ? kTile * CS : 4];

  const int tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6;
  const int li = lane & 31, hi = lane >> 5;
  const int cb = blockIdx.x / a.f_groups, g = blockIdx.x % a.f_groups;
  const int n0w = cb * (kWaves * kTile) + wave * kTile;
  const int ncol = n0w + li;
  const bool ncol_ok = ncol < a.N;
  const bool wave_on = n0w < a.N;
  const int K = a.K, F = a.F;
  const int K2 = (K + 1) >> 1;

  // B operand of Lambda = W H~: lane holds H~[2s + hi][ncol]
  float hB[K2MAX];
#pragma unroll
  for (int s = 0; s < K2MAX; ++s) {
    const int k = 2 * s + hi;
    hB[s] = (ncol_ok && k < K) ? a.H[(int64_t)k * a.ldh + ncol] : 0.f;
  }
  f32x16 accN[KB], accD[KB];
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) { accN[kb][r] = 0.f; accD[kb][r] = 0.f; }
  }

  // staging: WT tile thread float4 j -> row k = e4 / 8, columns f0 + 4 (e4 % 8);
  //          chi tile thread float4 j -> row i = e4 / (KP/4), columns 4 (e4 % (KP/4))
  float4 wreg[KB], c1reg[KB], c2reg[C2_TILE ? KB : 1];
  auto load_tiles = [&](int f0) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e4 = tid + kBlock * j;
      const int k = e4 >> 3, f = f0 + 4 * (e4 & 7);
      const float* src = a.WT + (int64_t)k * a.ldwt + f;
      if (f + 3 < F) {
        wreg[j] = *reinterpret_cast<const float4*>(src);
      } else {
        wreg[j].x = (f + 0 < F) ? src[0] : 0.f;
        wreg[j].y = (f + 1 < F) ? src[1] : 0.f;
        wreg[j].z = (f + 2 < F) ? src[2] : 0.f;
        wreg[j].w = (f + 3 < F) ? src[3] : 0.f;
      }
      const int i = e4 / (KP / 4), c = 4 * (e4 % (KP / 4));
      const bool ok = f0 + i < F;
      const int64_t o = (int64_t)(f0 + i) * KP + c;
      c1reg[j] = ok ? *reinterpret_cast<const float4*>(a.C1 + o) : make_float4(0.f, 0.f, 0.f, 0.f);
      if (C2_TILE) c2reg[j] = ok ? *reinterpret_cast<const float4*>(a.C2 + o) : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto store_tiles = [&](int buf) {
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const int e4 = tid + kBlock * j;
      *reinterpret_cast<float4*>(&Ws[buf][(e4 >> 3) * kHS + 4 * (e4 & 7)]) = wreg[j];
      const int i = e4 / (KP / 4), c = 4 * (e4 % (KP / 4));
      *reinterpret_cast<float4*>(&C1s[buf][i * CS + c]) = c1reg[j];
      if (C2_TILE) *reinterpret_cast<float4*>(&C2s[buf][i * CS + c]) = c2reg[j];
    }
  };
  // V at the accumulator positions: register r is row f0 + acc_row(r, hi), column ncol
  auto load_v = [&](int f0, float (&v)[16]) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int f = f0 + acc_row(r, hi);
      v[r] = (ncol_ok && f < F) ? a.V[(int64_t)f * a.ldv + ncol] : 0.f;
    }
  };

  const int ft_total = (F + kTile - 1) / kTile;
  const int t0 = g * a.tiles_per_group;
  const int t1 = min(ft_total, t0 + a.tiles_per_group);
  float vcur[16], vnext[16];
  if (t0 < t1) {
    load_tiles(t0 * kTile);
    if (wave_on) load_v(t0 * kTile, vcur);
    store_tiles(0);
  }
  __syncthreads();

  for (int t = t0; t < t1; ++t) {
    const int buf = (t - t0) & 1;
    const bool more = t + 1 < t1;
    if (more) {
      load_tiles((t + 1) * kTile);
      if (wave_on) load_v((t + 1) * kTile, vnext);
    }
    if (wave_on) {
      const int f0 = t * kTile;
      const float* ws = Ws[buf];
      const float* c1s = C1s[buf];
      const float* c2s = C2_TILE ? C2s[buf] : C1s[buf];
      // Lambda tile: lam[r] = Lambda[f0 + acc_row(r, hi)][ncol]; A operand W[f0+li][2s+hi]
      f32x16 lam;
#pragma unroll
      for (int r = 0; r < 16; ++r) lam[r] = 0.f;
#pragma unroll
      for (int s = 0; s < K2MAX; ++s)
        if (s < K2) lam = mfma32(ws[(2 * s + hi) * kHS + li], hB[s], lam);

      float P[16], Q[16];
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
    }
    __syncthreads();
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
// update_w: W_new = W~ (num/den)^gamma, chi terms, transposed copy of the factor
// that forms Lambda in the H pass, per-block column norm / sum partials.
// A block handles 32-row slabs (grid-stride).
// ---------------------------------------------------------------------------
__device__ __noinline__ double pow_out_of_line(double x, double y) { return pow(x, y); }

__device__ __forceinline__ double pow_gamma(double x, double g) {
  if (g == 1.0) return x;
  if (g == 0.5) return sqrt(x);
  return pow_out_of_line(x, g);
}

__device__ __forceinline__ void set_flag(unsigned* flags, unsigned bit) {
  __hip_atomic_fetch_or(flags, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// chi_1(W, W~) = W~^(2-b) / W^(1-b) = W~ r^(b-1) for b <= 2, else W;
// chi_2(W, W~) = W for b < 1, else W^b / W~^(b-1) = W~ r^b   (r = W / W~)
__device__ __forceinline__ void chi_terms(double beta, double wt, double r, double wnew, float& c1, float& c2) {
  double x1, x2;
  if (beta > 2.0) x1 = wnew;
  else if (beta == 2.0) x1 = wnew;
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

// Sums `groups` partial arrays (stride `gstride` floats) at offsets base + tid + i*kBlock
// (i < PER, entries below `limit`), four groups per round so that many loads
// are in flight; fixed order, float64 accumulation rounded once to float.
template <int PER>
__device__ __forceinline__ void sum_partials(const float* __restrict__ pn, const float* __restrict__ pd, int groups,
                                             int64_t gstride, int64_t base, int64_t limit, float (&num)[PER],
                                             float (&den)[PER]) {
  double sn[PER], sd[PER];
#pragma unroll
  for (int i = 0; i < PER; ++i) { sn[i] = 0.0; sd[i] = 0.0; }
  const int tid = threadIdx.x;
  int g = 0;
  for (; g + 4 <= groups; g += 4) {
    float xn[4][PER], xd[4][PER];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int i = 0; i < PER; ++i) {
        const int64_t e = tid + i * kBlock;
        const int64_t o = (int64_t)(g + u) * gstride + base + e;
        xn[u][i] = e < limit ? pn[o] : 0.f;
        xd[u][i] = (pd && e < limit) ? pd[o] : 0.f;
      }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int i = 0; i < PER; ++i) { sn[i] += (double)xn[u][i]; sd[i] += (double)xd[u][i]; }
  }
  for (; g < groups; ++g) {
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int64_t e = tid + i * kBlock;
      const int64_t o = (int64_t)g * gstride + base + e;
      sn[i] += e < limit ? (double)pn[o] : 0.0;
      sd[i] += (pd && e < limit) ? (double)pd[o] : 0.0;
    }
  }
#pragma unroll
  for (int i = 0; i < PER; ++i) { num[i] = (float)sn[i]; den[i] = (float)sd[i]; }
}

template <int KB>
__global__ __launch_bounds__(kBlock) void update_w_kernel(UpdateWArgs a) {
  constexpr int KP = 32 * KB;
  constexpr int PER = kTile * KP / kBlock;  // entries per thread per slab (4 KB)
  __shared__ float T[KP * 33];
  __shared__ double sn[kBlock], sc[kBlock];
  const int tid = threadIdx.x;
  const int k = tid % KP;  // the same k for all of a thread's entries (kBlock % KP == 0)
  const bool kok = k < a.K;
  double den1 = 0.0;
  if (a.beta_one && kok)
    for (int g = 0; g < a.n_groups; ++g) den1 += (double)a.prs[g * KP + k];

  double nrm = 0.0, cs = 0.0;
  const int slabs = (a.F + kTile - 1) / kTile;
  for (int sl = blockIdx.x; sl < slabs; sl += gridDim.x) {
    const int f0 = sl * kTile;
    float num[PER], den[PER];
    sum_partials<PER>(a.pnum, a.beta_one ? nullptr : a.pden, a.n_groups, (int64_t)a.F * KP,
                      (int64_t)f0 * KP, (int64_t)(min(a.F - f0, kTile)) * KP, num, den);
#pragma unroll 1
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * kBlock;
      const int fl = e / KP, f = f0 + fl;
      float wn = 0.f, c1 = 0.f, c2 = 0.f, wtf = 0.f;
      if (f < a.F && kok) {
        const double dd = a.beta_one ? den1 : (double)den[i];
        const double ratio = (double)num[i] / dd;
        if (!(dd > 0.0) || !isfinite(ratio)) set_flag(a.flags, 1u);
        const double r = pow_gamma(ratio, a.gamma);
        wtf = a.W[(int64_t)f * a.ldw + k];
        const double wt = (double)wtf;
        const double wnew = wt * r;
        wn = (float)wnew;
        if (a.joint) chi_terms(a.beta, wt, r, wnew, c1, c2);
        nrm += (double)wn * (double)wn;
        cs += (double)wn;
      }
      if (f < a.F) {
        const int64_t o = (int64_t)f * KP + k;
        a.Wn[o] = wn;
        if (a.joint) { a.C1[o] = c1; a.C2[o] = c2; }
      }
      T[k * 33 + fl] = a.joint ? wtf : wn;
    }
    __syncthreads();
    // transposed copy (KP x ldt) of the factor that forms Lambda in the H pass
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * kBlock;
      const int kk = e / kTile, fl = e % kTile;
      if (f0 + fl < a.F) a.WT[(int64_t)kk * a.ldt + f0 + fl] = T[kk * 33 + fl];
    }
    __syncthreads();
  }
  sn[tid] = nrm;
  sc[tid] = cs;
  __syncthreads();
  if (tid < KP) {
    double x = 0.0, y = 0.0;
    for (int j = 0; j < kBlock / KP; ++j) { x += sn[j * KP + tid]; y += sc[j * KP + tid]; }
    a.pcol[(int64_t)blockIdx.x * 2 * KP + tid] = x;
    a.pcol[(int64_t)blockIdx.x * 2 * KP + KP + tid] = y;
  }
}

// ---------------------------------------------------------------------------
// update_h: H_new = H~ (num/den)^gamma (* column norm), W <- W_new / norm
// ---------------------------------------------------------------------------
template <int KB>
__global__ __launch_bounds__(kBlock) void update_h_kernel(UpdateHArgs a) {
  constexpr int KP = 32 * KB;
  constexpr int PER = kTile * KP / kBlock;
  __shared__ double S[KP * 33];
  __shared__ double cn[kBlock], cc[kBlock];
  __shared__ float norm_s[KP], csum_s[KP];
  __shared__ double red[kWaves];
  const int tid = threadIdx.x;
  const int k = tid % KP;
  const int n0 = blockIdx.x * kTile;
  // column norms and sums of W_new from update_w's per-block partials (fixed order)
  {
    constexpr int R = kBlock / KP;
    const int part = tid / KP;
    double x = 0.0, y = 0.0;
    for (int b = part; b < a.pcol_blocks; b += R) {
      x += a.pcol[(int64_t)b * 2 * KP + k];
      y += a.pcol[(int64_t)b * 2 * KP + KP + k];
    }
    cn[tid] = x;
    cc[tid] = y;
    __syncthreads();
    if (tid < KP) {
      double xs = 0.0, ys = 0.0;
      for (int j = 0; j < R; ++j) { xs += cn[j * KP + tid]; ys += cc[j * KP + tid]; }
      norm_s[tid] = (float)sqrt(xs);
      csum_s[tid] = (float)ys;
    }
    __syncthreads();
  }
  if (blockIdx.x == 0 && a.d_obj) {
    double s = 0.0;
    for (int i = tid; i < a.nobj; i += kBlock) s += a.pobj[i];
    s = block_sum(s, red);
    if (tid == 0) {
      *a.d_obj = s;
      if (!isfinite(s)) set_flag(a.flags, 1u);
    }
  }
  if (n0 < a.N) {
    float num[PER], den[PER];
    sum_partials<PER>(a.pnum, a.beta_one ? nullptr : a.pden, a.f_groups, (int64_t)a.N * KP, (int64_t)n0 * KP,
                      (int64_t)(min(a.N - n0, kTile)) * KP, num, den);
    double nk = 1.0;
    if (a.normalize && k < a.K) {
      const float x = norm_s[k];
      if (x > 0.f) nk = (double)x;
    }
#pragma unroll 1
    for (int i = 0; i < PER; ++i) {
      const int e = tid + i * kBlock;
      const int nl = e / KP, n = n0 + nl;
      double s = 0.0;
      if (n < a.N && k < a.K) {
        const double dd = a.beta_one ? (double)csum_s[k] : (double)den[i];
        const double ratio = (double)num[i] / dd;
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
      if (kk < a.K && n < a.N) {
        float* h = a.H + (int64_t)kk * a.ldh + n;
        *h = (float)((double)*h * S[kk * 33 + nl]);
      }
    }
  }
  // normalized W (every block takes a strided share)
  const int64_t total = (int64_t)a.F * a.K;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + tid; e < total; e += (int64_t)gridDim.x * kBlock) {
    const int f = (int)(e / a.K), kk = (int)(e % a.K);
    float w = a.Wn[(int64_t)f * KP + kk];
    if (a.normalize) {
      const float x = norm_s[kk];
      if (x > 0.f) w = (float)((double)w / (double)x);
    }
    a.W[(int64_t)f * a.ldw + kk] = w;
  }
}

// Transposed copy WT[k][f] = W[f][k] (k < KP, zero-padded) and a row-major copy
// Wp[f][k] with leading dimension KP (zero-padded): the layouts the H pass stages.
__global__ __launch_bounds__(kBlock) void transpose_kernel(const float* W, int64_t ldw, int F, int K, int KP,
                                                           float* WT, int64_t ldt, float* Wp) {
  __shared__ float T[32 * 33];
  const int f0 = blockIdx.x * 32, k0 = blockIdx.y * 32;
  for (int e = threadIdx.x; e < 32 * 32; e += kBlock) {
    const int fl = e / 32, kl = e % 32;
    const int f = f0 + fl, k = k0 + kl;
    const float w = (f < F && k < K) ? W[(int64_t)f * ldw + k] : 0.f;
    T[kl * 33 + fl] = w;
    if (f < F) Wp[(int64_t)f * KP + k] = w;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 32 * 32; e += kBlock) {
    const int kl = e / 32, fl = e % 32;
    const int f = f0 + fl, k = k0 + kl;
    if (f < F) WT[(int64_t)k * ldt + f] = T[kl * 33 + fl];
  }
}

// ---------------------------------------------------------------------------
// small kernels: objective finalization, gradient write-out, domain scan
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void finalize_objective_kernel(const double* pobj, int n, double* out,
                                                                    unsigned* flags) {
  __shared__ double red[kWaves];
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) s += pobj[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    *out = s;
    if (!isfinite(s)) set_flag(flags, 1u);
  }
}

template <int KB>
__global__ __launch_bounds__(kBlock) void grad_w_kernel(const float* pnum, int F, int K, int n_groups,
                                                        double scale, float* dW, int64_t lddw) {
  constexpr int KP = 32 * KB;
  const int64_t total = (int64_t)F * K;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBlock) {
    const int f = (int)(e / K), k = (int)(e % K);
    double s = 0.0;
    for (int g = 0; g < n_groups; ++g) s += (double)pnum[((int64_t)g * F + f) * KP + k];
    dW[(int64_t)f * lddw + k] = (float)(scale * s);
  }
}

template <int KB>
__global__ __launch_bounds__(kBlock) void grad_h_kernel(const float* pnum, int N, int K, int f_groups,
                                                        double scale, float* dH, int64_t lddh) {
  constexpr int KP = 32 * KB;
  __shared__ float S[KP * 33];
  const int n0 = blockIdx.x * kTile;
  for (int e = threadIdx.x; e < kTile * KP; e += kBlock) {
    const int nl = e / KP, k = e % KP, n = n0 + nl;
    double s = 0.0;
    if (n < N && k < K)
      for (int g = 0; g < f_groups; ++g) s += (double)pnum[((int64_t)g * N + n) * KP + k];
    S[k * 33 + nl] = (float)(scale * s);
  }
  __syncthreads();
  for (int e = threadIdx.x; e < KP * kTile; e += kBlock) {
    const int k = e / kTile, nl = e % kTile, n = n0 + nl;
    if (k < K && n < N) dH[(int64_t)k * lddh + n] = S[k * 33 + nl];
  }
}

__global__ __launch_bounds__(kBlock) void validate_kernel(const float* V, int64_t ldv, const float* W, int64_t ldw,
                                                          const float* H, int64_t ldh, int F, int N, int K,
                                                          int zero_bad, unsigned* flags) {
  bool bad = false;
  const int64_t stride = (int64_t)gridDim.x * kBlock;
  const int64_t t0 = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  for (int64_t e = t0; e < (int64_t)F * N; e += stride) {
    const float v = V[(e / N) * ldv + e % N];
    bad |= !(v >= 0.f) || !isfinite(v) || (zero_bad && v == 0.f);
  }
  for (int64_t e = t0; e < (int64_t)F * K; e += stride) {
    const float w = W[(e / K) * ldw + e % K];
    bad |= !(w > 0.f) || !isfinite(w);
  }
  for (int64_t e = t0; e < (int64_t)K * N; e += stride) {
    const float h = H[(e / N) * ldh + e % N];
    bad |= !(h > 0.f) || !isfinite(h);
  }
  if (__any(bad) && (threadIdx.x & 63) == 0) set_flag(flags, 2u);
}

// ---------------------------------------------------------------------------
// launchers: map runtime (beta class, K block count, kind) to instantiations
// ---------------------------------------------------------------------------
template <int BC, int KB>
static hipError_t rows_kb(int kind, bool obj, int grid, hipStream_t s, const SweepRowsArgs& a) {
  if (kind == KIND_UPDATE) {
    if (obj) hipLaunchKernelGGL((sweep_rows_kernel<BC, KB, KIND_UPDATE, true>), dim3(grid), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((sweep_rows_kernel<BC, KB, KIND_UPDATE, false>), dim3(grid), dim3(kBlock), 0, s, a);
  } else if (kind == KIND_GRAD) {
    if (obj) hipLaunchKernelGGL((sweep_rows_kernel<BC, KB, KIND_GRAD, true>), dim3(grid), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((sweep_rows_kernel<BC, KB, KIND_GRAD, false>), dim3(grid), dim3(kBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL((sweep_rows_kernel<BC, KB, KIND_OBJ, true>), dim3(grid), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

template <int BC>
static hipError_t rows_bc(int kb, int kind, bool obj, int grid, hipStream_t s, const SweepRowsArgs& a) {
  switch (kb) {
    case 1: return rows_kb<BC, 1>(kind, obj, grid, s, a);
    case 2: return rows_kb<BC, 2>(kind, obj, grid, s, a);
    case 4: return rows_kb<BC, 4>(kind, obj, grid, s, a);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_rows(int bc, int kb, int kind, bool obj, int grid, hipStream_t s, const SweepRowsArgs& a) {
  switch (bc) {
    case BC_GEN: return rows_bc<BC_GEN>(kb, kind, obj, grid, s, a);
    case BC_B2: return rows_bc<BC_B2>(kb, kind, obj, grid, s, a);
    case BC_B1: return rows_bc<BC_B1>(kb, kind, obj, grid, s, a);
    case BC_B0: return rows_bc<BC_B0>(kb, kind, obj, grid, s, a);
    case BC_B05: return rows_bc<BC_B05>(kb, kind, obj, grid, s, a);
    case BC_B15: return rows_bc<BC_B15>(kb, kind, obj, grid, s, a);
  }
  return hipErrorInvalidValue;
}

template <int BC, int KB>
static hipError_t cols_kb(int kind, bool dual, int grid, hipStream_t s, const SweepColsArgs& a) {
  if (kind == KIND_UPDATE) {
    if (dual) hipLaunchKernelGGL((sweep_cols_kernel<BC, KB, KIND_UPDATE, true>), dim3(grid), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((sweep_cols_kernel<BC, KB, KIND_UPDATE, false>), dim3(grid), dim3(kBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL((sweep_cols_kernel<BC, KB, KIND_GRAD, false>), dim3(grid), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

template <int BC>
static hipError_t cols_bc(int kb, int kind, bool dual, int grid, hipStream_t s, const SweepColsArgs& a) {
  switch (kb) {
    case 1: return cols_kb<BC, 1>(kind, dual, grid, s, a);
    case 2: return cols_kb<BC, 2>(kind, dual, grid, s, a);
    case 4: return cols_kb<BC, 4>(kind, dual, grid, s, a);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_cols(int bc, int kb, int kind, bool dual, int grid, hipStream_t s, const SweepColsArgs& a) {
  switch (bc) {
    case BC_GEN: return cols_bc<BC_GEN>(kb, kind, dual, grid, s, a);
    case BC_B2: return cols_bc<BC_B2>(kb, kind, dual, grid, s, a);
    case BC_B1: return cols_bc<BC_B1>(kb, kind, dual, grid, s, a);
    case BC_B0: return cols_bc<BC_B0>(kb, kind, dual, grid, s, a);
    case BC_B05: return cols_bc<BC_B05>(kb, kind, dual, grid, s, a);
    case BC_B15: return cols_bc<BC_B15>(kb, kind, dual, grid, s, a);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_update_w(int kb, int grid, hipStream_t s, const UpdateWArgs& a) {
  switch (kb) {
    case 1: hipLaunchKernelGGL(update_w_kernel<1>, dim3(grid), dim3(kBlock), 0, s, a); break;
    case 2: hipLaunchKernelGGL(update_w_kernel<2>, dim3(grid), dim3(kBlock), 0, s, a); break;
    case 4: hipLaunchKernelGGL(update_w_kernel<4>, dim3(grid), dim3(kBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_update_h(int kb, int grid, hipStream_t s, const UpdateHArgs& a) {
  switch (kb) {
    case 1: hipLaunchKernelGGL(update_h_kernel<1>, dim3(grid), dim3(kBlock), 0, s, a); break;
    case 2: hipLaunchKernelGGL(update_h_kernel<2>, dim3(grid), dim3(kBlock), 0, s, a); break;
    case 4: hipLaunchKernelGGL(update_h_kernel<4>, dim3(grid), dim3(kBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_finalize_objective(hipStream_t s, const double* pobj, int n, double* out, unsigned* flags) {
  hipLaunchKernelGGL(finalize_objective_kernel, dim3(1), dim3(kBlock), 0, s, pobj, n, out, flags);
  return hipGetLastError();
}

hipError_t launch_grad_w(int kb, int grid, hipStream_t s, const float* pnum, int F, int K, int n_groups,
                         double scale, float* dW, int64_t lddw) {
  switch (kb) {
    case 1: hipLaunchKernelGGL(grad_w_kernel<1>, dim3(grid), dim3(kBlock), 0, s, pnum, F, K, n_groups, scale, dW, lddw); break;
    case 2: hipLaunchKernelGGL(grad_w_kernel<2>, dim3(grid), dim3(kBlock), 0, s, pnum, F, K, n_groups, scale, dW, lddw); break;
    case 4: hipLaunchKernelGGL(grad_w_kernel<4>, dim3(grid), dim3(kBlock), 0, s, pnum, F, K, n_groups, scale, dW, lddw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_grad_h(int kb, int grid, hipStream_t s, const float* pnum, int N, int K, int f_groups,
                         double scale, float* dH, int64_t lddh) {
  switch (kb) {
    case 1: hipLaunchKernelGGL(grad_h_kernel<1>, dim3(grid), dim3(kBlock), 0, s, pnum, N, K, f_groups, scale, dH, lddh); break;
    case 2: hipLaunchKernelGGL(grad_h_kernel<2>, dim3(grid), dim3(kBlock), 0, s, pnum, N, K, f_groups, scale, dH, lddh); break;
    case 4: hipLaunchKernelGGL(grad_h_kernel<4>, dim3(grid), dim3(kBlock), 0, s, pnum, N, K, f_groups, scale, dH, lddh); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_transpose(hipStream_t s, const float* W, int64_t ldw, int F, int K, int KP, float* WT,
                            int64_t ldt, float* Wp) {
  hipLaunchKernelGGL(transpose_kernel, dim3((F + 31) / 32, KP / 32), dim3(kBlock), 0, s, W, ldw, F, K, KP, WT, ldt, Wp);
  return hipGetLastError();
}

hipError_t launch_validate(hipStream_t s, const float* V, int64_t ldv, const float* W, int64_t ldw,
                           const float* H, int64_t ldh, int F, int N, int K, int zero_bad, unsigned* flags) {
  hipLaunchKernelGGL(validate_kernel, dim3(512), dim3(kBlock), 0, s, V, ldv, W, ldw, H, ldh, F, N, K, zero_bad, flags);
  return hipGetLastError();
}

}  // namespace nmf
