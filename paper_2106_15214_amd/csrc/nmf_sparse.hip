// beta = 1 (Kullback-Leibler) multiplicative updates for a V stored by its
// nonzeros, in both compressed orders: CSR (row_ptr, col_idx, row_val) and CSC
// (col_ptr, row_idx, col_val) hold the same entries.  Table 2's KL row
// (Sec. 3.3.1) needs V / (WH) only where v != 0:
//   W step (both methods):  numW = P H~^T,  P = V / (W~ H~) at the nonzeros;
//                           denW = the row sums of H~ (the same for every row);
//   H step, joint MM:       numH = W~^T P with the same P (chi_1 = W~ at beta = 1),
//                           denH = the column sums of W_new (chi_2 = W_new);
//   H step, alternating MU: numH = W_new^T P',  P' = V / (W_new H~) at the nonzeros,
//                           denH = the column sums of W_new.
// The objective D_1(V | W~H~) sums every [W~H~]_fn from factor sums and adds
// v log(v / [W~H~]_fn) - v at the nonzeros only.
//
// One wavefront owns one row of V (row pass, W numerators and the objective)
// or one column (column pass, H numerators), so no partial sums cross
// wavefronts and every sum has a fixed order.  Lane i takes the line's entries
// i, i + 64, ...: it gathers the K-vector of the other factor at the entry
// (a row of H~^T, or of W for the column pass; stored K4-padded so that 16-byte
// loads read it), forms lambda as its dot product with the line's own factor
// vector (in scalar registers), P = v / lambda, and adds P times the gathered
// vector to its own K partial sums.  At the end of the line the 64 partial
// vectors are summed through LDS (lane k sums column k).
// The joint step runs the row pass and the column pass in one launch (the
// column pass only needs W~ and H~); alternating MU runs the column pass after
// the W update, gathering W_new.  Arithmetic: lambda, P and the numerators in
// float32; the objective terms and every reduction of the denominators in
// float64.  K <= 64.
#include "nmf_device.h"

namespace nmf {

constexpr int kSpTile = 64;          // columns (rows) per workgroup of the transpose/copy blocks

__device__ __forceinline__ int k4_of(int K) { return (K + 3) & ~3; }

// out[k] = sum over b < nparts of parts[b * stride + k] for k < K4 (float64), by
// the whole workgroup: four slices of 64 threads take every fourth part, with
// eight loads in flight per round, and their sums are added in a fixed order
// (deterministic).  `scratch` is LDS [4][64]; out is LDS [64].  Contains
// barriers: every thread of the workgroup must call it.
__device__ __forceinline__ void sum_parts(const double* __restrict__ parts, int nparts, int64_t stride, int K4,
                                          double (*scratch)[64], double* out) {
  const int tid = threadIdx.x, k = tid & 63, sl = tid >> 6;
  double s = 0.0;
  if (k < K4) {
    int b = sl;
    for (; b + 28 < nparts; b += 32) {
      double x[8];
#pragma unroll
      for (int r = 0; r < 8; ++r) x[r] = parts[(int64_t)(b + 4 * r) * stride + k];
      s += ((x[0] + x[1]) + (x[2] + x[3])) + ((x[4] + x[5]) + (x[6] + x[7]));
    }
    for (; b < nparts; b += 4) s += parts[(int64_t)b * stride + k];
  }
  scratch[sl][k] = s;
  __syncthreads();
  if (tid < 64) out[tid] = (scratch[0][tid] + scratch[1][tid]) + (scratch[2][tid] + scratch[3][tid]);
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Preparation: HT = H~^T ([N][K4], zero padded), Wc = W~ ([F][K4]), and float64
// partial sums: prow[b][k] = sum of H~[k][n] over block b's 64 columns,
// pcw[b][k] = sum of W~[f][k] over block b's 64 rows.  Blocks [0, hb) do H,
// blocks [hb, hb + wb) do W.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void sparse_prep_kernel(SparseArgs a, int hb) {
  __shared__ float tile[64][kSpTile + 1];
  const int tid = threadIdx.x;
  const int K = a.K, K4 = k4_of(K);
  if ((int)blockIdx.x < hb) {
    const int n0 = blockIdx.x * kSpTile;
    for (int e = tid; e < 64 * kSpTile; e += kBlock) {
      const int k = e / kSpTile, c = e % kSpTile, n = n0 + c;
      tile[k][c] = (k < K && n < a.N) ? a.Hio[(int64_t)k * a.ldh + n] : 0.f;
    }
    __syncthreads();
    for (int e = tid; e < kSpTile * K4; e += kBlock) {
      const int c = e / K4, k = e % K4, n = n0 + c;
      if (n < a.N) a.HT[(int64_t)n * K4 + k] = tile[k][c];
    }
    if (tid < K4) {
      double s = 0.0;
      for (int c = 0; c < kSpTile; ++c) s += (double)tile[tid][c];
      a.prow[(int64_t)blockIdx.x * K4 + tid] = s;
    }
  } else {
    const int b = blockIdx.x - hb;
    const int f0 = b * kSpTile;
    for (int e = tid; e < kSpTile * K4; e += kBlock) {
      const int r = e / K4, k = e % K4, f = f0 + r;
      const float x = (k < K && f < a.F) ? a.Wio[(int64_t)f * a.ldw + k] : 0.f;
      tile[k][r] = x;
      if (f < a.F) a.Wc[(int64_t)f * K4 + k] = x;
    }
    __syncthreads();
    if (tid < K4) {
      double s = 0.0;
      for (int r = 0; r < kSpTile; ++r) s += (double)tile[tid][r];
      a.pcw[(int64_t)b * K4 + tid] = s;
    }
  }
}

// ---------------------------------------------------------------------------
// One line (row or column) of V: out[k] = sum over the line's entries e of
// (v_e / lambda_e) * G[idx_e][k], lambda_e = <U, G[idx_e]>, where U is the line's
// own factor vector (4 KQ floats, kept in scalar registers).  Lane i takes entries
// i, i + 64, ... and keeps its own K-vector of partial sums in registers; at
// the end of the line the 64 partial vectors go through LDS and lane k sums
// column k (consecutive lanes read consecutive words).  Returns the sum in
// lane k < 4 KQ.  With OBJ, v log(v / lambda) - v (float64) is added to `obj`
// per lane.  Indices are clamped to [0, limit) and the caller clamps the
// entry range to [0, nnz]: a malformed compressed matrix gives wrong numbers
// (nmf_sparse_validate flags it), never an access outside the arrays.
// ---------------------------------------------------------------------------
template <int KQ, bool OBJ>
__device__ __forceinline__ float sparse_line(int64_t e0, int64_t e1, const int32_t* __restrict__ idx,
                                             const float* __restrict__ val, const float* __restrict__ G, int limit,
                                             const float* __restrict__ Urow, float* T, double& obj) {
  const int lane = threadIdx.x & 63;
  // the line's own factor vector is the same for every lane: kept in scalar
  // registers, it costs no vector registers and no LDS traffic per entry
  float u[4 * KQ];
#pragma unroll
  for (int i = 0; i < 4 * KQ; ++i) u[i] = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(Urow[i])));
  float4 acc[KQ];
#pragma unroll
  for (int q = 0; q < KQ; ++q) acc[q] = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int64_t c0 = e0; c0 < e1; c0 += 64) {
    const bool ok = c0 + lane < e1;
    const int64_t e = ok ? c0 + lane : c0;
    const int j = min(max(idx[e], 0), limit - 1);
    const float v = val[e];
    const float4* g = reinterpret_cast<const float4*>(G + (int64_t)j * (4 * KQ));
    float4 x[KQ];
#pragma unroll
    for (int q = 0; q < KQ; ++q) x[q] = g[q];
    float lam = 0.f;
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      lam = fmaf(u[4 * q + 0], x[q].x, lam);
      lam = fmaf(u[4 * q + 1], x[q].y, lam);
      lam = fmaf(u[4 * q + 2], x[q].z, lam);
      lam = fmaf(u[4 * q + 3], x[q].w, lam);
    }
    const float p = (ok && v != 0.f) ? v * __builtin_amdgcn_rcpf(lam) : 0.f;
    if (OBJ && ok && v > 0.f) obj += kl_nz((double)v, (double)lam);
#pragma unroll
    for (int q = 0; q < KQ; ++q) {
      acc[q].x = fmaf(p, x[q].x, acc[q].x);
      acc[q].y = fmaf(p, x[q].y, acc[q].y);
      acc[q].z = fmaf(p, x[q].z, acc[q].z);
      acc[q].w = fmaf(p, x[q].w, acc[q].w);
    }
  }
  // lanes i and i + 32 first (cross-half swap), then the 32 half-row vectors
  // through LDS: lane k sums column k
  constexpr int ST = 4 * KQ + 4;  // LDS row stride (floats)
#pragma unroll
  for (int q = 0; q < KQ; ++q) {
    acc[q].x += __shfl_xor(acc[q].x, 32, 64);
    acc[q].y += __shfl_xor(acc[q].y, 32, 64);
    acc[q].z += __shfl_xor(acc[q].z, 32, 64);
    acc[q].w += __shfl_xor(acc[q].w, 32, 64);
  }
  if (lane < 32) {
    float* trow = T + lane * ST;
#pragma unroll
    for (int q = 0; q < KQ; ++q) *reinterpret_cast<float4*>(trow + 4 * q) = acc[q];
  }
  wave_lds_sync();
  float s[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) s[r] = 0.f;
  if (lane < 4 * KQ) {
#pragma unroll
    for (int i = 0; i < 32; i += 8)
#pragma unroll
      for (int r = 0; r < 8; ++r) s[r] += T[(i + r) * ST + lane];
  }
  wave_lds_sync();  // T is reused by the wave's next line
  return ((s[0] + s[1]) + (s[2] + s[3])) + ((s[4] + s[5]) + (s[6] + s[7]));
}

// Row pass over blocks [0, rb) (four rows per workgroup, one per wave) and,
// unless `cols_first` < 0, column pass over the following blocks; with
// `cols_first` > 0 the whole grid is the column pass.  Row pass: numW, the
// objective partial of the block (pobj[block], float64, when a.pobj != null).
// Column pass: numH gathering a.Wg (W~ for joint MM, W_new for alternating MU).
// One instantiation per KQ = K4 / 4, so each has its own register budget.
template <int KQ>
__global__ __launch_bounds__(kBlock) void sparse_pass_kernel(SparseArgs a, int rb, int cols_first) {
  constexpr int K4 = 4 * KQ;
  __shared__ __align__(16) float T[kWaves][32 * (K4 + 4)];
  __shared__ double red[kWaves];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double obj = 0.0;
  const bool row_block = cols_first == 0 && (int)blockIdx.x < rb;
  if (row_block) {
    const int f = blockIdx.x * kWaves + wave;
    if (f < a.F) {
      const float* U = a.Wc + (int64_t)f * K4;
      const int64_t e0 = min(max(a.row_ptr[f], (int64_t)0), a.nnz);
      const int64_t e1 = min(max(a.row_ptr[f + 1], e0), a.nnz);
      const float acc = a.pobj ? sparse_line<KQ, true>(e0, e1, a.col_idx, a.row_val, a.HT, a.N, U, T[wave], obj)
                               : sparse_line<KQ, false>(e0, e1, a.col_idx, a.row_val, a.HT, a.N, U, T[wave], obj);
      if (lane < K4) a.numW[(int64_t)f * K4 + lane] = acc;
    }
    if (a.pobj) {
      const double s = block_sum(obj, red);
      if (tid == 0) a.pobj[blockIdx.x] = s;
    }
  } else {
    const int n = ((int)blockIdx.x - (cols_first ? 0 : rb)) * kWaves + wave;
    if (n < a.N) {
      const float* U = a.HT + (int64_t)n * K4;
      const int64_t e0 = min(max(a.col_ptr[n], (int64_t)0), a.nnz);
      const int64_t e1 = min(max(a.col_ptr[n + 1], e0), a.nnz);
      const float acc = sparse_line<KQ, false>(e0, e1, a.row_idx, a.col_val, a.Wg, a.F, U, T[wave], obj);
      if (lane < K4) a.numH[(int64_t)n * K4 + lane] = acc;
    }
  }
}

template <int KQ>
void launch_pass_kq(hipStream_t s, const SparseArgs& a, int grid, int rb, int cols_first) {
  hipLaunchKernelGGL(sparse_pass_kernel<KQ>, dim3(grid), dim3(kBlock), 0, s, a, rb, cols_first);
}

void launch_pass(hipStream_t s, const SparseArgs& a, int grid, int rb, int cols_first) {
  switch ((a.K + 3) / 4) {
#define NMF_SP_CASE(q) \
    case q: launch_pass_kq<q>(s, a, grid, rb, cols_first); break;
    NMF_SP_CASE(1) NMF_SP_CASE(2) NMF_SP_CASE(3) NMF_SP_CASE(4) NMF_SP_CASE(5) NMF_SP_CASE(6) NMF_SP_CASE(7)
    NMF_SP_CASE(8) NMF_SP_CASE(9) NMF_SP_CASE(10) NMF_SP_CASE(11) NMF_SP_CASE(12) NMF_SP_CASE(13)
    NMF_SP_CASE(14) NMF_SP_CASE(15)
#undef NMF_SP_CASE
    default: launch_pass_kq<16>(s, a, grid, rb, cols_first); break;
  }
}

// ---------------------------------------------------------------------------
// W update: W_new = W~ numW / rowsum(H~) (gamma = 1 at beta = 1), written to
// a.Wn ([F][K4]); per-block float64 partials of the column sums of W_new and of
// its squares (pcol[b][0][k], pcol[b][1][k]).  Block b owns 64 rows.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void sparse_update_w_kernel(SparseArgs a, int hb) {
  __shared__ double den_s[64];
  __shared__ double cs[4][64], cq[4][64];
  const int tid = threadIdx.x;
  const int K = a.K, K4 = k4_of(K);
  sum_parts(a.prow, hb, K4, K4, cs, den_s);
  const int k = tid % 64, sl = tid / 64;
  double s1 = 0.0, s2 = 0.0;
  bool bad = false;
  if (k < K4) {
    const double den = den_s[k];
    for (int r = sl; r < kSpTile; r += 4) {
      const int f = blockIdx.x * kSpTile + r;
      if (f >= a.F) break;
      float wn = 0.f;
      if (k < K) {
        const double num = (double)a.numW[(int64_t)f * K4 + k];
        const double ratio = num / den;
        if (!(den > 0.0) || !isfinite(ratio)) bad = true;
        wn = (float)((double)a.Wc[(int64_t)f * K4 + k] * ratio);
        s1 += (double)wn;
        s2 += (double)wn * (double)wn;
      }
      a.Wn[(int64_t)f * K4 + k] = wn;
    }
  }
  if (bad) set_flag(a.flags, 1u);
  if (k < 64) { cs[sl][k] = s1; cq[sl][k] = s2; }
  __syncthreads();
  if (tid < K4) {
    a.pcol[((int64_t)blockIdx.x * 2 + 0) * K4 + tid] = cs[0][tid] + cs[1][tid] + cs[2][tid] + cs[3][tid];
    a.pcol[((int64_t)blockIdx.x * 2 + 1) * K4 + tid] = cq[0][tid] + cq[1][tid] + cq[2][tid] + cq[3][tid];
  }
}

// ---------------------------------------------------------------------------
// H update and write-back: colsum_k = sum_f W_new[f][k], n_k = ||W_new[:,k]||;
// H[k][n] = H~[k][n] numH[n][k] / colsum_k (times n_k when normalizing);
// W[f][k] = W_new[f][k] / n_k (unchanged where n_k = 0; plain W_new without
// normalization).  Blocks [0, nb) own 64 columns of H, blocks [nb, nb + wb)
// 64 rows of W.  Block 0 also writes the objective of the entry iterate:
// sum of the row-pass partials plus sum_k colsum(W~)_k rowsum(H~)_k.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kBlock) void sparse_update_h_kernel(SparseArgs a, int nb, int uwb, int hb, int wcb,
                                                                 int pob) {
  __shared__ float tile[64][kSpTile + 1];
  __shared__ double csum[64], nrm[64], sw_s[64], sh_s[64];
  __shared__ double scratch[4][64];
  __shared__ double red[kWaves];
  const int tid = threadIdx.x;
  const int K = a.K, K4 = k4_of(K);
  sum_parts(a.pcol, uwb, 2 * K4, K4, scratch, csum);
  sum_parts(a.pcol + K4, uwb, 2 * K4, K4, scratch, nrm);
  if (tid < K4) nrm[tid] = a.normalize ? sqrt(nrm[tid]) : 1.0;
  const bool obj_block = blockIdx.x == 0 && a.d_obj;
  if (obj_block) {
    sum_parts(a.pcw, wcb, K4, K4, scratch, sw_s);
    sum_parts(a.prow, hb, K4, K4, scratch, sh_s);
  }
  __syncthreads();
  if ((int)blockIdx.x < nb) {
    const int n0 = blockIdx.x * kSpTile;
    for (int e = tid; e < kSpTile * K4; e += kBlock) {
      const int c = e / K4, k = e % K4, n = n0 + c;
      tile[k][c] = n < a.N ? a.numH[(int64_t)n * K4 + k] : 0.f;
    }
    __syncthreads();
    bool bad = false;
    for (int e = tid; e < K * kSpTile; e += kBlock) {
      const int k = e / kSpTile, c = e % kSpTile, n = n0 + c;
      if (n >= a.N) continue;
      const double den = csum[k];
      const double ratio = (double)tile[k][c] / den;
      if (!(den > 0.0) || !isfinite(ratio)) bad = true;
      const double sc = nrm[k] > 0.0 ? nrm[k] : 1.0;
      float* h = a.Hio + (int64_t)k * a.ldh + n;
      *h = (float)((double)*h * ratio * sc);
    }
    if (bad) set_flag(a.flags, 1u);
  } else {
    const int f0 = (blockIdx.x - nb) * kSpTile;
    for (int e = tid; e < kSpTile * K; e += kBlock) {
      const int r = e / K, k = e % K, f = f0 + r;
      if (f >= a.F) break;
      const double sc = nrm[k] > 0.0 ? nrm[k] : 1.0;
      a.Wio[(int64_t)f * a.ldw + k] = (float)((double)a.Wn[(int64_t)f * K4 + k] / sc);
    }
  }
  if (obj_block) {
    double s = 0.0;
    for (int i = tid; i < pob; i += kBlock) s += a.pobj[i];
    if (tid < K4) s += sw_s[tid] * sh_s[tid];
    s = block_sum(s, red);
    if (tid == 0) {
      *a.d_obj = s;
      if (!isfinite(s)) set_flag(a.flags, 1u);
    }
  }
}

// Objective of the entry iterate alone: sum of the row-pass partials plus
// sum_k colsum(W~)_k rowsum(H~)_k, written to *out.
__global__ __launch_bounds__(kBlock) void sparse_objective_kernel(SparseArgs a, int hb, int wcb, int pob,
                                                                  double* out) {
  __shared__ double red[kWaves];
  __shared__ double sw_s[64], sh_s[64], scratch[4][64];
  const int tid = threadIdx.x, K4 = k4_of(a.K);
  sum_parts(a.pcw, wcb, K4, K4, scratch, sw_s);
  sum_parts(a.prow, hb, K4, K4, scratch, sh_s);
  double s = 0.0;
  for (int i = tid; i < pob; i += kBlock) s += a.pobj[i];
  if (tid < K4) s += sw_s[tid] * sh_s[tid];
  s = block_sum(s, red);
  if (tid == 0) {
    *out = s;
    if (!isfinite(s)) set_flag(a.flags, 1u);
  }
}

// Structure and value scan of both compressed orders: pointers start at 0, end
// at nnz and never decrease, indices lie in range and ascend within a line,
// values are finite and >= 0.  Any violation sets NMF_FLAG_DOMAIN.  (That the
// two orders hold the same entries is the caller's promise.)
__global__ __launch_bounds__(kBlock) void sparse_validate_kernel(SparseArgs a) {
  bool bad = false;
  const int64_t t0 = (int64_t)blockIdx.x * kBlock + threadIdx.x, st = (int64_t)gridDim.x * kBlock;
  if (t0 == 0)
    bad |= a.row_ptr[0] != 0 || a.row_ptr[a.F] != a.nnz || a.col_ptr[0] != 0 || a.col_ptr[a.N] != a.nnz;
  for (int64_t i = t0; i < a.F; i += st) bad |= a.row_ptr[i + 1] < a.row_ptr[i];
  for (int64_t i = t0; i < a.N; i += st) bad |= a.col_ptr[i + 1] < a.col_ptr[i];
  for (int64_t e = t0; e < a.nnz; e += st) {
    const int c = a.col_idx[e], r = a.row_idx[e];
    const float v = a.row_val[e], w = a.col_val[e];
    bad |= c < 0 || c >= a.N || r < 0 || r >= a.F || !(v >= 0.f) || !(w >= 0.f) || !isfinite(v) || !isfinite(w);
  }
  // ascending indices within each line
  for (int64_t f = t0; f < a.F; f += st) {
    const int64_t e0 = min(max(a.row_ptr[f], (int64_t)0), a.nnz), e1 = min(max(a.row_ptr[f + 1], e0), a.nnz);
    for (int64_t e = e0 + 1; e < e1; ++e) bad |= a.col_idx[e] <= a.col_idx[e - 1];
  }
  for (int64_t n = t0; n < a.N; n += st) {
    const int64_t e0 = min(max(a.col_ptr[n], (int64_t)0), a.nnz), e1 = min(max(a.col_ptr[n + 1], e0), a.nnz);
    for (int64_t e = e0 + 1; e < e1; ++e) bad |= a.row_idx[e] <= a.row_idx[e - 1];
  }
  if (bad) set_flag(a.flags, 2u);
}

hipError_t launch_sparse_validate(hipStream_t s, const SparseArgs& a) {
  hipLaunchKernelGGL(sparse_validate_kernel, dim3(512), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

int sparse_blocks(int F, int N, int* hb, int* wcb, int* rb, int* cb) {
  *hb = (N + kSpTile - 1) / kSpTile;
  *wcb = (F + kSpTile - 1) / kSpTile;
  *rb = (F + kWaves - 1) / kWaves;
  *cb = (N + kWaves - 1) / kWaves;
  return 0;
}

hipError_t launch_sparse_prep(hipStream_t s, const SparseArgs& a) {
  int hb, wcb, rb, cb;
  sparse_blocks(a.F, a.N, &hb, &wcb, &rb, &cb);
  hipLaunchKernelGGL(sparse_prep_kernel, dim3(hb + wcb), dim3(kBlock), 0, s, a, hb);
  return hipGetLastError();
}

hipError_t launch_sparse_pass(hipStream_t s, const SparseArgs& a, bool rows, bool cols) {
  int hb, wcb, rb, cb;
  sparse_blocks(a.F, a.N, &hb, &wcb, &rb, &cb);
  if (rows) launch_pass(s, a, rb + (cols ? cb : 0), rb, 0);
  else if (cols) launch_pass(s, a, cb, 0, 1);
  return hipGetLastError();
}

hipError_t launch_sparse_update_w(hipStream_t s, const SparseArgs& a) {
  int hb, wcb, rb, cb;
  sparse_blocks(a.F, a.N, &hb, &wcb, &rb, &cb);
  hipLaunchKernelGGL(sparse_update_w_kernel, dim3(wcb), dim3(kBlock), 0, s, a, hb);
  return hipGetLastError();
}

hipError_t launch_sparse_update_h(hipStream_t s, const SparseArgs& a) {
  int hb, wcb, rb, cb;
  sparse_blocks(a.F, a.N, &hb, &wcb, &rb, &cb);
  hipLaunchKernelGGL(sparse_update_h_kernel, dim3(hb + wcb), dim3(kBlock), 0, s, a, hb, wcb, hb, wcb,
                     a.pobj ? rb : 0);
  return hipGetLastError();
}

// Objective only: preparation (factor sums, HT, Wc) and the row pass.
hipError_t launch_sparse_objective(hipStream_t s, const SparseArgs& a, double* d_out) {
  const int hb = (a.N + kSpTile - 1) / kSpTile;
  const int wcb = (a.F + kSpTile - 1) / kSpTile;
  const int rb = (a.F + kWaves - 1) / kWaves;
  hipLaunchKernelGGL(sparse_prep_kernel, dim3(hb + wcb), dim3(kBlock), 0, s, a, hb);
  launch_pass(s, a, rb, rb, 0);
  hipLaunchKernelGGL(sparse_objective_kernel, dim3(1), dim3(kBlock), 0, s, a, hb, wcb, rb, d_out);
  return hipGetLastError();
}

}  // namespace nmf
