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

// d_beta(v | l) in float64 (v, l include kappa), paper eq. (beta-div);
// v = 0 takes the limit of the expression.
template <int BC>
__device__ __forceinline__ double d_beta(double v, double l, double beta) {
  if (BC == BC_B2) { double t = v - l; return 0.5 * t * t; }
  if (BC == BC_B1) return v > 0.0 ? v * log(v / l) - v + l : l;
  if (BC == BC_B0) { double r = v / l; return r - log(r) - 1.0; }
  if (BC == BC_B05) { double sy = sqrt(l); return -4.0 * sqrt(v) + 2.0 * sy + 2.0 * v / sy; }
  if (BC == BC_B15) { double sy = sqrt(l); return v * sqrt(v) / 0.75 + l * sy / 1.5 - 2.0 * v * sy; }
  if (v > 0.0)
    return pow(v, beta) / (beta * (beta - 1.0)) + pow(l, beta) / beta - v * pow(l, beta - 1.0) / (beta - 1.0);
  return beta > 0.0 ? pow(l, beta) / beta : __builtin_inf();
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
// sweep_rows: W-step contractions (reduction over n), optional objective
// ---------------------------------------------------------------------------
constexpr int kHsStride = 36;  // LDS row stride of the H~ tile; float4 reads conflict-free

template <int BC, int KB, int KIND, bool OBJ>
__global__ __launch_bounds__(kBlock) void sweep_rows_kernel(SweepRowsArgs a) {
  constexpr int KP = 32 * KB;
  constexpr int K2MAX = KP / 2;
  constexpr bool CONTRACT = (KIND != KIND_OBJ);
  constexpr bool NEED_DEN = (KIND == KIND_UPDATE) && (BC != BC_B1);
  constexpr bool ROWSUM = (KIND == KIND_UPDATE) && (BC == BC_B1);
  __shared__ __align__(16) float Hs[KP * kHsStride];
  __shared__ double red[kWaves];

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 31, hi = lane >> 5;
  const int rb = blockIdx.x / a.n_groups, gj = blockIdx.x % a.n_groups;
  const int f0 = rb * kRowsPerBlock + wave * kTile;
  const int frow = f0 + li;
  const bool frow_ok = frow < a.F;
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
  float rsum = 0.f;
  double objsum = 0.0;

  const int nt_total = (N + kTile - 1) / kTile;
  const int t_begin = gj * a.tiles_per_group;
  const int t_end = min(nt_total, t_begin + a.tiles_per_group);
  const float* vrow = a.V + (int64_t)frow * a.ldv;

  for (int t = t_begin; t < t_end; ++t) {
    const int n0 = t * kTile;
    // stage H~[0:KP, n0:n0+32] (zero outside K x N)
    for (int e = threadIdx.x; e < KP * kTile; e += kBlock) {
      const int k = e >> 5, c = e & 31;
      float h = 0.f;
      if (k < K && n0 + c < N) h = a.H[(int64_t)k * a.ldh + n0 + c];
      Hs[k * kHsStride + c] = h;
    }
    __syncthreads();
    if (ROWSUM && rb == 0 && threadIdx.x < KP) {
      float s = 0.f;
      for (int c = 0; c < kTile; ++c) s += Hs[threadIdx.x * kHsStride + c];
      rsum += s;
    }

    // Lambda^T tile: lam[r] = Lambda[frow][n0 + acc_row(r, hi)]
    f32x16 lam;
#pragma unroll
    for (int r = 0; r < 16; ++r) lam[r] = 0.f;
#pragma unroll
    for (int s = 0; s < K2MAX; ++s)
      if (s < K2) lam = mfma32(Hs[(2 * s + hi) * kHsStride + li], wB[s], lam);

    // V at the same positions: registers 4q..4q+3 are columns n0 + 8q + 4hi + 0..3
    float v[16];
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

    float P[16], Q[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int n = n0 + acc_row(r, hi);
      const bool ok = frow_ok && n < N;
      const float lk = lam[r] + a.kappa;
      const float vk = v[r] + a.kappa;
      if (KIND == KIND_UPDATE) {
        beta_terms<BC>(vk, lk, a.bm2, P[r], Q[r]);
        if (!ok) { P[r] = 0.f; Q[r] = 0.f; }
      } else if (KIND == KIND_GRAD) {
        P[r] = ok ? pow_bm2<BC>(lk, a.bm2) * (lam[r] - v[r]) : 0.f;
      }
      if (OBJ && ok) objsum += d_beta<BC>((double)vk, (double)lk, a.beta);
    }

    if (CONTRACT) {
#pragma unroll
      for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          // B operand: H~[kb*32 + li][n0 + 8q + 4hi + j]
          const float4 b = *reinterpret_cast<const float4*>(&Hs[(kb * 32 + li) * kHsStride + 8 * q + 4 * hi]);
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
    __syncthreads();
  }

  if (CONTRACT) {
    // accumulator (i = row offset f, j = li = column k)
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int f = f0 + acc_row(r, hi);
        if (f < a.F) {
          const int64_t o = ((int64_t)gj * a.F + f) * KP + kb * 32 + li;
          a.pnum[o] = accN[kb][r];
          if (NEED_DEN) a.pden[o] = accD[kb][r];
        }
      }
    }
  }
  if (ROWSUM && rb == 0 && threadIdx.x < KP) a.prs[gj * KP + threadIdx.x] = rsum;
  if (OBJ) {
    const double s = block_sum(objsum, red);
    if (threadIdx.x == 0) a.pobj[blockIdx.x] = s;
  }
}

// ---------------------------------------------------------------------------
// sweep_cols: H-step contractions (reduction over f)
// ---------------------------------------------------------------------------
template <int BC, int KB, int KIND, bool DUAL>
__global__ __launch_bounds__(kBlock) void sweep_cols_kernel(SweepColsArgs a) {
  constexpr int KP = 32 * KB;
  constexpr int WS = KP + 1;  // LDS row stride: A-operand reads conflict-free
  constexpr int K2MAX = KP / 2;
  constexpr bool NEED_DEN = (KIND == KIND_UPDATE) && (BC != BC_B1);
  __shared__ float Ws[kTile * WS];
  __shared__ float C1s[DUAL ? kTile * WS : 1];
  __shared__ float C2s[(DUAL && NEED_DEN) ? kTile * WS : 1];

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int li = lane & 31, hi = lane >> 5;
  const int cb = blockIdx.x / a.f_groups, gi = blockIdx.x % a.f_groups;
  const int n0w = cb * kRowsPerBlock + wave * kTile;
  const int ncol = n0w + li;
  const bool ncol_ok = ncol < a.N;
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

  const int ft_total = (F + kTile - 1) / kTile;
  const int t_begin = gi * a.tiles_per_group;
  const int t_end = min(ft_total, t_begin + a.tiles_per_group);
  const float* c1src = DUAL ? C1s : Ws;
  const float* c2src = DUAL ? C2s : Ws;

  for (int t = t_begin; t < t_end; ++t) {
    const int f0 = t * kTile;
    for (int e = threadIdx.x; e < kTile * KP; e += kBlock) {
      const int i = e / KP, k = e % KP;
      const bool ok = (f0 + i < F) && (k < K);
      Ws[i * WS + k] = ok ? a.WL[(int64_t)(f0 + i) * a.ldwl + k] : 0.f;
      if (DUAL) {
        C1s[i * WS + k] = ok ? a.C1[(int64_t)(f0 + i) * a.ldc + k] : 0.f;
        if (NEED_DEN) C2s[i * WS + k] = ok ? a.C2[(int64_t)(f0 + i) * a.ldc + k] : 0.f;
      }
    }
    __syncthreads();

    // Lambda tile: lam[r] = Lambda[f0 + acc_row(r, hi)][ncol]
    f32x16 lam;
#pragma unroll
    for (int r = 0; r < 16; ++r) lam[r] = 0.f;
#pragma unroll
    for (int s = 0; s < K2MAX; ++s)
      if (s < K2) lam = mfma32(Ws[li * WS + 2 * s + hi], hB[s], lam);

    float P[16], Q[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int f = f0 + acc_row(r, hi);
      const bool ok = ncol_ok && f < F;
      const float vv = ok ? a.V[(int64_t)f * a.ldv + ncol] : 0.f;
      const float lk = lam[r] + a.kappa;
      const float vk = vv + a.kappa;
      if (KIND == KIND_UPDATE) {
        beta_terms<BC>(vk, lk, a.bm2, P[r], Q[r]);
        if (!ok) { P[r] = 0.f; Q[r] = 0.f; }
      } else {
        P[r] = ok ? pow_bm2<BC>(lk, a.bm2) * (lam[r] - vv) : 0.f;
      }
    }

#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const int row = acc_row(r, hi) * WS + kb * 32 + li;
        accN[kb] = mfma32(P[r], c1src[row], accN[kb]);
        if (NEED_DEN) accD[kb] = mfma32(Q[r], c2src[row], accD[kb]);
      }
    }
    __syncthreads();
  }

  // accumulator (i = column offset n, j = li = k)
#pragma unroll
  for (int kb = 0; kb < KB; ++kb) {
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const int n = n0w + acc_row(r, hi);
      if (n < a.N) {
        const int64_t o = ((int64_t)gi * a.N + n) * KP + kb * 32 + li;
        a.pnum[o] = accN[kb][r];
        if (NEED_DEN) a.pden[o] = accD[kb][r];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// update_w: W_new = W~ (num/den)^gamma, chi terms, column norms / sums,
// objective finalization (last workgroup)
// ---------------------------------------------------------------------------
__device__ __forceinline__ double pow_gamma(double x, double g) {
  if (g == 1.0) return x;
  if (g == 0.5) return sqrt(x);
  return pow(x, g);
}

__device__ __forceinline__ void set_flag(unsigned* flags, unsigned bit) {
  __hip_atomic_fetch_or(flags, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Returns true in every thread of the last workgroup to arrive at `counter`.
__device__ __forceinline__ bool last_block(unsigned* counter) {
  __shared__ int is_last;
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned prev = __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    is_last = (prev == gridDim.x - 1);
  }
  __syncthreads();
  const bool r = is_last != 0;
  if (r) __threadfence();
  return r;
}

template <int KB>
__global__ __launch_bounds__(kBlock) void update_w_kernel(UpdateWArgs a) {
  constexpr int KP = 32 * KB;
  constexpr int RPS = kBlock / KP;  // rows per step
  __shared__ double sn[kBlock], sc[kBlock];
  __shared__ double red[kWaves];
  const int k = threadIdx.x % KP, rs = threadIdx.x / KP;
  const bool kok = k < a.K;
  double den1 = 0.0;
  if (a.beta_one && kok)
    for (int g = 0; g < a.n_groups; ++g) den1 += (double)a.prs[g * KP + k];

  double nrm = 0.0, cs = 0.0;
  for (int f = blockIdx.x * RPS + rs; f < a.F; f += gridDim.x * RPS) {
    float wn = 0.f, c1 = 0.f, c2 = 0.f;
    if (kok) {
      double num = 0.0, den = 0.0;
      for (int g = 0; g < a.n_groups; ++g) {
        const int64_t o = ((int64_t)g * a.F + f) * KP + k;
        num += (double)a.pnum[o];
        if (!a.beta_one) den += (double)a.pden[o];
      }
      if (a.beta_one) den = den1;
      const double ratio = num / den;
      if (!(den > 0.0) || !isfinite(ratio)) set_flag(a.flags, 1u);
      const double r = pow_gamma(ratio, a.gamma);
      const double wt = (double)a.W[(int64_t)f * a.ldw + k];
      const double wnew = wt * r;
      wn = (float)wnew;
      if (a.joint) {
        // chi_1(W, W~) = W~^(2-b) / W^(1-b) = W~ r^(b-1)  (b <= 2), else W
        // chi_2(W, W~) = W (b < 1), else W^b / W~^(b-1) = W~ r^b
        c1 = (float)(a.beta <= 2.0 ? (a.beta == 1.0 ? wt : wt * pow(r, a.beta - 1.0)) : wnew);
        c2 = (float)(a.beta < 1.0 ? wnew : (a.beta == 1.0 ? wnew : wt * pow(r, a.beta)));
      }
      nrm += (double)wn * (double)wn;
      cs += (double)wn;
    }
    const int64_t o = (int64_t)f * KP + k;
    a.Wn[o] = wn;
    if (a.joint) { a.C1[o] = c1; a.C2[o] = c2; }
  }
  sn[threadIdx.x] = nrm;
  sc[threadIdx.x] = cs;
  __syncthreads();
  if (threadIdx.x < KP) {
    double x = 0.0, y = 0.0;
    for (int j = 0; j < RPS; ++j) { x += sn[j * KP + threadIdx.x]; y += sc[j * KP + threadIdx.x]; }
    a.pcol[(int64_t)blockIdx.x * 2 * KP + threadIdx.x] = x;
    a.pcol[(int64_t)blockIdx.x * 2 * KP + KP + threadIdx.x] = y;
  }
  if (last_block(a.counter)) {
    const double* pc = a.pcol;
    if (threadIdx.x < KP) {
      double x = 0.0, y = 0.0;
      for (int b = 0; b < (int)gridDim.x; ++b) {
        x += pc[(int64_t)b * 2 * KP + threadIdx.x];
        y += pc[(int64_t)b * 2 * KP + KP + threadIdx.x];
      }
      a.norms[threadIdx.x] = (float)sqrt(x);
      a.csum[threadIdx.x] = (float)y;
    }
    if (a.d_obj) {
      double s = 0.0;
      for (int i = threadIdx.x; i < a.nobj; i += kBlock) s += a.pobj[i];
      s = block_sum(s, red);
      if (threadIdx.x == 0) {
        *a.d_obj = s;
        if (!isfinite(s)) set_flag(a.flags, 1u);
      }
    }
    if (threadIdx.x == 0) *a.counter = 0u;
  }
}

// ---------------------------------------------------------------------------
// update_h: H_new = H~ (num/den)^gamma (* column norm), W <- W_new / norm
// ---------------------------------------------------------------------------
template <int KB>
__global__ __launch_bounds__(kBlock) void update_h_kernel(UpdateHArgs a) {
  constexpr int KP = 32 * KB;
  __shared__ double S[KP * 33];
  const int n0 = blockIdx.x * kTile;
  if (n0 < a.N) {
    for (int e = threadIdx.x; e < kTile * KP; e += kBlock) {
      const int nl = e / KP, k = e % KP, n = n0 + nl;
      double s = 0.0;
      if (n < a.N && k < a.K) {
        double num = 0.0, den = 0.0;
        for (int g = 0; g < a.f_groups; ++g) {
          const int64_t o = ((int64_t)g * a.N + n) * KP + k;
          num += (double)a.pnum[o];
          if (!a.beta_one) den += (double)a.pden[o];
        }
        if (a.beta_one) den = (double)a.csum[k];
        const double ratio = num / den;
        if (!(den > 0.0) || !isfinite(ratio)) set_flag(a.flags, 1u);
        s = pow_gamma(ratio, a.gamma);
        if (a.normalize) {
          const float nk = a.norms[k];
          if (nk > 0.f) s *= (double)nk;
        }
      }
      S[k * 33 + nl] = s;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < KP * kTile; e += kBlock) {
      const int k = e / kTile, nl = e % kTile, n = n0 + nl;
      if (k < a.K && n < a.N) {
        float* h = a.H + (int64_t)k * a.ldh + n;
        *h = (float)((double)*h * S[k * 33 + nl]);
      }
    }
  }
  // normalized W (every block takes a strided share)
  const int64_t total = (int64_t)a.F * a.K;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < total; e += (int64_t)gridDim.x * kBlock) {
    const int f = (int)(e / a.K), k = (int)(e % a.K);
    float w = a.Wn[(int64_t)f * KP + k];
    if (a.normalize) {
      const float nk = a.norms[k];
      if (nk > 0.f) w = (float)((double)w / (double)nk);
    }
    a.W[(int64_t)f * a.ldw + k] = w;
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

hipError_t launch_validate(hipStream_t s, const float* V, int64_t ldv, const float* W, int64_t ldw,
                           const float* H, int64_t ldh, int F, int N, int K, int zero_bad, unsigned* flags) {
  hipLaunchKernelGGL(validate_kernel, dim3(512), dim3(kBlock), 0, s, V, ldv, W, ldw, H, ldh, F, N, K, zero_bad, flags);
  return hipGetLastError();
}

}  // namespace nmf
