// Update kernels of the streaming path (reduction of the partial contractions,
// multiplicative updates, normalization), transposition, gradient write-out,
// objective finalization and the domain scan.  The passes over V are in
// nmf_sweep_rows.hip and nmf_sweep_cols.hip; the device building blocks live in
// nmf_device.h.
#include <algorithm>

#include "nmf_device.h"

namespace nmf {

// W update.  Narrow: 256 threads, four thread slices per row.  Wide: 1024
// threads with the same rows per unit and four times as many slices, so that
// each thread sums a quarter of the groups -- for problems split into many
// groups, where the partial reads would otherwise take several rounds.
constexpr int kUpdateWThreadsWide = 1024;

template <int KB, int BT, int SL>
__global__ __launch_bounds__(BT) void update_w_kernel(UpdateWArgs a) {
  if (a.halt && *a.halt) return;
  constexpr int RU = unit_rows<KB, SL, BT>();
  static_assert(RU == unit_rows<KB>(), "rows per unit must match the host plan");
  __shared__ double lds[2 * BT];
  const double den1 = a.beta_one ? row_sum_den_wide<KB, BT>(a, lds) : 0.0;
  double nrm = 0.0, cs = 0.0;  // unused here: the H pass forms the column sums
  const int units = (a.F + RU - 1) / RU;
  for (int u = blockIdx.x; u < units; u += gridDim.x)
    update_w_unit<KB, SL, BT>(a, u, true, reinterpret_cast<float*>(lds), den1, nrm, cs);
}

// H update of kBlock / KP columns per workgroup (thread (k, c) owns H[k][n]).
// Every independent load -- the H~ entry, the first round of H partials, the
// first W_new entry of the write-back -- is issued before the column-sum
// reduction, so the kernel's latency is about one memory round trip plus the
// reduction.
template <int KB>
__global__ __launch_bounds__(kBlock) void update_h_kernel(UpdateHArgs a) {
  if (a.halt && *a.halt) return;
  constexpr int KP = 32 * KB;
  constexpr int UC = kBlock / KP;
  constexpr int U = 16;
  __shared__ double scratch[2 * kBlock];
  __shared__ float norm_s[KP], csum_s[KP];
  __shared__ double red[kWaves];
  const int tid = threadIdx.x;
  const int k = tid % KP, n = blockIdx.x * UC + tid / KP;
  const bool ok = n < a.N && k < a.K;
  const int64_t gstride = (int64_t)a.N * KP;
  const int64_t base = (int64_t)n * KP + k;
  const float hv = ldc(a.H, (int64_t)k * a.ldh + n, ok);
  float xn[U], xd[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const bool gu = ok && u < a.f_groups;
    xn[u] = ldc(a.pnum, (int64_t)u * gstride + base, gu);
    xd[u] = a.beta_one ? 0.f : ldc(a.pden, (int64_t)u * gstride + base, gu);
  }
  const int64_t total_w = (int64_t)a.F * a.K;
  const int64_t e0 = (int64_t)blockIdx.x * kBlock + tid, estride = (int64_t)gridDim.x * kBlock;
  const int f0 = (int)(e0 / (a.K > 0 ? a.K : 1)), kk0 = (int)(e0 % (a.K > 0 ? a.K : 1));
  const float w0 = ldc(a.Wn, (int64_t)f0 * KP + kk0, e0 < total_w);

  reduce_columns<KB>(a.pcol, a.pcol_blocks, scratch, norm_s, csum_s);
  if (blockIdx.x == 0 && a.d_obj) {
    double s = 0.0;
    for (int i = tid; i < a.nobj; i += kBlock) s += a.pobj[i];
    s = block_sum(s, red);
    if (tid == 0) {
      *a.d_obj = s;
      if (!isfinite(s)) set_flag(a.flags, 1u);
    }
  }
  // W <- W_new / norm: the first entry from the prefetched value, the rest (when
  // the grid is smaller than F * K) by write_w
  if (a.W && e0 < total_w) {
    float w = w0;
    if (a.normalize) {
      const float x = norm_s[kk0];
      if (x > 0.f) w = (float)((double)w / (double)x);
    }
    a.W[(int64_t)f0 * a.ldw + kk0] = w;
  }
  if (a.W && e0 + estride < total_w) write_w<KB>(a, norm_s, e0 + estride, estride);

  double num = 0.0, den = 0.0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (u < a.f_groups) { num += (double)xn[u]; den += (double)xd[u]; }
  }
  for (int g = U; g < a.f_groups; g += U) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool gu = ok && g + u < a.f_groups;
      xn[u] = ldc(a.pnum, (int64_t)(g + u) * gstride + base, gu);
      xd[u] = a.beta_one ? 0.f : ldc(a.pden, (int64_t)(g + u) * gstride + base, gu);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (g + u < a.f_groups) { num += (double)xn[u]; den += (double)xd[u]; }
    }
  }
  if (!ok) return;
  double gden = 0.0;
  if (a.gram) {  // Gram form at beta = 2: (G2 H~)[k][n], eight terms in flight
    double g8[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    int l = 0;
    for (; l + 8 <= a.K; l += 8) {
#pragma unroll
      for (int j = 0; j < 8; ++j) g8[j] = fma(a.gram[k * KP + l + j], (double)a.H[(int64_t)(l + j) * a.ldh + n], g8[j]);
    }
    for (; l < a.K; ++l) g8[0] = fma(a.gram[k * KP + l], (double)a.H[(int64_t)l * a.ldh + n], g8[0]);
    gden = ((g8[0] + g8[1]) + (g8[2] + g8[3])) + ((g8[4] + g8[5]) + (g8[6] + g8[7]));
  }
  const double dd = a.beta_one ? (double)csum_s[k] : (a.gram ? gden : den);
  const double ratio = num / dd;
  if (!(dd > 0.0) || !isfinite(ratio)) set_flag(a.flags, 1u);
  if (a.C1h) {  // sub-iteration: chi terms of H_new against H~ (no normalization)
    const double rr = pow_gamma(ratio, a.gamma);
    float c1, c2;
    chi_terms(a.beta, (double)hv, rr, (double)hv * rr, c1, c2);
    a.C1h[(int64_t)k * a.ldc + n] = c1;
    a.C2h[(int64_t)k * a.ldc + n] = c2;
    return;
  }
  double nk = 1.0;
  if (a.normalize) {
    const float x = norm_s[k];
    if (x > 0.f) nk = (double)x;
  }
  a.H[(int64_t)k * a.ldh + n] = (float)((double)hv * (pow_gamma(ratio, a.gamma) * nk));
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
    const float w = ldz(W, (int64_t)f * ldw + k, f < F && k < K);
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
                                                        double scale, const double* dscale, float* dW,
                                                        int64_t lddw) {
  constexpr int KP = 32 * KB;
  if (dscale) scale *= *dscale;
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
                                                        double scale, const double* dscale, float* dH,
                                                        int64_t lddh) {
  constexpr int KP = 32 * KB;
  if (dscale) scale *= *dscale;
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
hipError_t launch_update_w(int kb, int grid, hipStream_t s, const UpdateWArgs& a) {
  const bool wide = a.n_groups > 4 * kSlices;
  switch (kb) {
    case 1:
      if (wide) hipLaunchKernelGGL((update_w_kernel<1, kUpdateWThreadsWide, 4 * kSlices>), dim3(grid), dim3(kUpdateWThreadsWide), 0, s, a);
      else hipLaunchKernelGGL((update_w_kernel<1, kBlock, kSlices>), dim3(grid), dim3(kBlock), 0, s, a);
      break;
    case 2:
      if (wide) hipLaunchKernelGGL((update_w_kernel<2, kUpdateWThreadsWide, 4 * kSlices>), dim3(grid), dim3(kUpdateWThreadsWide), 0, s, a);
      else hipLaunchKernelGGL((update_w_kernel<2, kBlock, kSlices>), dim3(grid), dim3(kBlock), 0, s, a);
      break;
    case 4:
      if (wide) hipLaunchKernelGGL((update_w_kernel<4, kUpdateWThreadsWide, 4 * kSlices>), dim3(grid), dim3(kUpdateWThreadsWide), 0, s, a);
      else hipLaunchKernelGGL((update_w_kernel<4, kBlock, kSlices>), dim3(grid), dim3(kBlock), 0, s, a);
      break;
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

// ---------------------------------------------------------------------------
// Gram matrices of the beta = 2 Gram form (Table 2).  gram_kernel: block b
// takes a range of i (32 at a time staged in LDS) and writes its float64
// partial [KP][KP]; gram_finalize_kernel adds the partials in block order (one
// thread per entry, eight loads in flight).  Deterministic, no atomics.
// ---------------------------------------------------------------------------
constexpr int kGramBlocks = 64;
int gram_parts() { return kGramBlocks; }

template <bool COLS>
__global__ __launch_bounds__(kBlock) void gram_kernel(const float* X, int64_t ldx, const float* Y, int64_t ldy, int K,
                                                      int KP, int64_t len, double* part) {
  __shared__ float xs[32][65], ys[32][65];
  const int tid = threadIdx.x;
  const int64_t chunk = (len + gridDim.x - 1) / gridDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * chunk, i1 = min(len, i0 + chunk);
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int64_t b = i0; b < i1; b += 32) {
    __syncthreads();
    for (int e = tid; e < 32 * 64; e += kBlock) {
      int r, k;
      if (COLS) { k = e / 32; r = e % 32; }  // consecutive threads read consecutive columns of a row
      else { r = e / 64; k = e % 64; }       // consecutive threads read consecutive entries of a row
      const int64_t i = b + r;
      const bool ok = i < i1 && k < K;
      float x = 0.f, y = 0.f;
      if (ok) {
        x = COLS ? X[(int64_t)k * ldx + i] : X[i * ldx + k];
        y = COLS ? Y[(int64_t)k * ldy + i] : Y[i * ldy + k];
      }
      xs[r][k] = x;
      ys[r][k] = y;
    }
    __syncthreads();
    // thread owns pairs (k, l) = (4 (tid / 16) + q / 4, 4 (tid % 16) + q % 4), q < 16
#pragma unroll 4
    for (int r = 0; r < 32; ++r) {
#pragma unroll
      for (int q = 0; q < 16; ++q) {
        const int k = (tid >> 4) * 4 + (q >> 2), l = (tid & 15) * 4 + (q & 3);
        acc[q] = fma((double)xs[r][k], (double)ys[r][l], acc[q]);
      }
    }
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int k = (tid >> 4) * 4 + (q >> 2), l = (tid & 15) * 4 + (q & 3);
    if (k < KP && l < KP) part[(int64_t)blockIdx.x * KP * KP + k * KP + l] = acc[q];
  }
}

__global__ __launch_bounds__(kBlock) void gram_finalize_kernel(const double* part, int nparts, int KP, double* G) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= KP * KP) return;
  double s = 0.0;
  int b = 0;
  for (; b + 8 <= nparts; b += 8) {
    double x[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) x[r] = part[(int64_t)(b + r) * KP * KP + e];
    s += ((x[0] + x[1]) + (x[2] + x[3])) + ((x[4] + x[5]) + (x[6] + x[7]));
  }
  for (; b < nparts; ++b) s += part[(int64_t)b * KP * KP + e];
  G[e] = s;
}

hipError_t launch_gram(bool cols, hipStream_t s, const float* X, int64_t ldx, const float* Y, int64_t ldy, int K,
                       int KP, int64_t len, double* part, double* G) {
  if (K > 64 || KP > 64) return hipErrorInvalidValue;
  // about 64 entries of i per block, at most kGramBlocks blocks
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(kGramBlocks, (len + 63) / 64));
  if (cols) hipLaunchKernelGGL(gram_kernel<true>, dim3(grid), dim3(kBlock), 0, s, X, ldx, Y, ldy, K, KP, len, part);
  else hipLaunchKernelGGL(gram_kernel<false>, dim3(grid), dim3(kBlock), 0, s, X, ldx, Y, ldy, K, KP, len, part);
  hipLaunchKernelGGL(gram_finalize_kernel, dim3((KP * KP + kBlock - 1) / kBlock), dim3(kBlock), 0, s, part, grid,
                     KP, G);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Device-side outer loop: stopping rule of Sec. 4.1.2 on the objective trace
// ---------------------------------------------------------------------------
__global__ void run_init_kernel(unsigned* halt, int32_t* stop) {
  if (threadIdx.x == 0) {
    *halt = 0u;
    *stop = -1;
  }
}

__global__ __launch_bounds__(kBlock) void run_decide_kernel(const double* pobj, int n, double* trace, int t,
                                                            double eps, unsigned* halt, int32_t* stop,
                                                            unsigned* flags) {
  __shared__ double red[kWaves];
  if (*halt) return;  // uniform: the run stopped at an earlier iterate
  double s = 0.0;
  for (int i = threadIdx.x; i < n; i += kBlock) s += pobj[i];
  s = block_sum(s, red);
  if (threadIdx.x == 0) {
    trace[t] = s;
    if (!isfinite(s)) set_flag(flags, 1u);
    // relative decrease (D(previous) - D(current)) / D(current), as printed (no
    // absolute value): an increase also stops the run
    if (t >= 1 && (trace[t - 1] - s) / s <= eps) {
      *halt = 1u;
      *stop = t;
    }
  }
}

hipError_t launch_run_init(hipStream_t s, unsigned* halt, int32_t* stop) {
  hipLaunchKernelGGL(run_init_kernel, dim3(1), dim3(64), 0, s, halt, stop);
  return hipGetLastError();
}

hipError_t launch_run_decide(hipStream_t s, const double* pobj, int n, double* trace, int t, double eps,
                             unsigned* halt, int32_t* stop, unsigned* flags) {
  hipLaunchKernelGGL(run_decide_kernel, dim3(1), dim3(kBlock), 0, s, pobj, n, trace, t, eps, halt, stop, flags);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// KKT residuals (Sec. 4.1.5) from the gradient partials of the two passes:
// blocks [0, kKktBlocks) sum |min(w_fk, g_fk)| over W's entries, blocks
// [kKktBlocks, 2 kKktBlocks) |min(h_kn, g_kn)| over H's; block partials in
// float64, then one block adds them in a fixed order and divides by the entry
// counts F K and K N.
// ---------------------------------------------------------------------------
constexpr int kKktBlocks = 256;
int kkt_parts() { return 2 * kKktBlocks; }

template <int KB>
__global__ __launch_bounds__(kBlock) void kkt_kernel(const float* pnumw, int n_groups, const float* pnumh,
                                                     int f_groups, const float* W, int64_t ldw, const float* H,
                                                     int64_t ldh, int F, int N, int K, double* part) {
  constexpr int KP = 32 * KB;
  __shared__ double red[kWaves];
  const bool wpart = (int)blockIdx.x < kKktBlocks;
  const int b = wpart ? blockIdx.x : blockIdx.x - kKktBlocks;
  double s = 0.0;
  if (wpart) {
    const int64_t total = (int64_t)F * K;
    for (int64_t e = (int64_t)b * kBlock + threadIdx.x; e < total; e += (int64_t)kKktBlocks * kBlock) {
      const int f = (int)(e / K), k = (int)(e % K);
      double g = 0.0;
      for (int q = 0; q < n_groups; ++q) g += (double)pnumw[((int64_t)q * F + f) * KP + k];
      s += fabs(fmin((double)W[(int64_t)f * ldw + k], g));
    }
  } else {
    const int64_t total = (int64_t)K * N;
    for (int64_t e = (int64_t)b * kBlock + threadIdx.x; e < total; e += (int64_t)kKktBlocks * kBlock) {
      const int k = (int)(e / N), n = (int)(e % N);
      double g = 0.0;
      for (int q = 0; q < f_groups; ++q) g += (double)pnumh[((int64_t)q * N + n) * KP + k];
      s += fabs(fmin((double)H[(int64_t)k * ldh + n], g));
    }
  }
  s = block_sum(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

__global__ __launch_bounds__(kBlock) void kkt_finalize_kernel(const double* part, int F, int N, int K,
                                                              double* res) {
  __shared__ double red[kWaves];
  for (int h = 0; h < 2; ++h) {
    double s = 0.0;
    for (int i = threadIdx.x; i < kKktBlocks; i += kBlock) s += part[h * kKktBlocks + i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) res[h] = s / (h == 0 ? (double)F * K : (double)K * N);
  }
}

hipError_t launch_kkt(int kb, hipStream_t s, const float* pnumw, int n_groups, const float* pnumh, int f_groups,
                      const float* W, int64_t ldw, const float* H, int64_t ldh, int F, int N, int K, double* part,
                      double* res) {
  switch (kb) {
    case 1: hipLaunchKernelGGL(kkt_kernel<1>, dim3(2 * kKktBlocks), dim3(kBlock), 0, s, pnumw, n_groups, pnumh, f_groups, W, ldw, H, ldh, F, N, K, part); break;
    case 2: hipLaunchKernelGGL(kkt_kernel<2>, dim3(2 * kKktBlocks), dim3(kBlock), 0, s, pnumw, n_groups, pnumh, f_groups, W, ldw, H, ldh, F, N, K, part); break;
    case 4: hipLaunchKernelGGL(kkt_kernel<4>, dim3(2 * kKktBlocks), dim3(kBlock), 0, s, pnumw, n_groups, pnumh, f_groups, W, ldw, H, ldh, F, N, K, part); break;
    default: return hipErrorInvalidValue;
  }
  hipLaunchKernelGGL(kkt_finalize_kernel, dim3(1), dim3(kBlock), 0, s, part, F, N, K, res);
  return hipGetLastError();
}

hipError_t launch_finalize_objective(hipStream_t s, const double* pobj, int n, double* out, unsigned* flags) {
  hipLaunchKernelGGL(finalize_objective_kernel, dim3(1), dim3(kBlock), 0, s, pobj, n, out, flags);
  return hipGetLastError();
}

hipError_t launch_grad_w(int kb, int grid, hipStream_t s, const float* pnum, int F, int K, int n_groups,
                         double scale, const double* dscale, float* dW, int64_t lddw) {
  switch (kb) {
    case 1: hipLaunchKernelGGL(grad_w_kernel<1>, dim3(grid), dim3(kBlock), 0, s, pnum, F, K, n_groups, scale, dscale, dW, lddw); break;
    case 2: hipLaunchKernelGGL(grad_w_kernel<2>, dim3(grid), dim3(kBlock), 0, s, pnum, F, K, n_groups, scale, dscale, dW, lddw); break;
    case 4: hipLaunchKernelGGL(grad_w_kernel<4>, dim3(grid), dim3(kBlock), 0, s, pnum, F, K, n_groups, scale, dscale, dW, lddw); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_grad_h(int kb, int grid, hipStream_t s, const float* pnum, int N, int K, int f_groups,
                         double scale, const double* dscale, float* dH, int64_t lddh) {
  switch (kb) {
    case 1: hipLaunchKernelGGL(grad_h_kernel<1>, dim3(grid), dim3(kBlock), 0, s, pnum, N, K, f_groups, scale, dscale, dH, lddh); break;
    case 2: hipLaunchKernelGGL(grad_h_kernel<2>, dim3(grid), dim3(kBlock), 0, s, pnum, N, K, f_groups, scale, dscale, dH, lddh); break;
    case 4: hipLaunchKernelGGL(grad_h_kernel<4>, dim3(grid), dim3(kBlock), 0, s, pnum, N, K, f_groups, scale, dscale, dH, lddh); break;
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
