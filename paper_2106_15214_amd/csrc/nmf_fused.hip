// One outer iteration of the multiplicative-update method in a single
// cooperative launch: every workgroup takes part in the four phases
//   1. W pass    (rows items: Lambda~, P, Q, W-step contractions, objective;
//                 joint mode also stores P and Q tile by tile)
//   2. W update  (partials reduced by all workgroups; chi terms; column sums)
//   3. H pass    (cols items: joint mode contracts the stored P, Q with chi_1,
//                 chi_2 -- V~ and its element-wise terms are formed once per
//                 outer iteration, as in Algorithm 2; alternating mode forms
//                 Lambda' = W_new H~ again, as in Algorithm 1)
//   4. H update  (partials reduced; normalization; objective total)
// separated by grid barriers.  It replaces three launches by grid barriers; on
// MI355X the barriers cost more than the launches they replace, so the default
// path selection uses the four-launch streaming path, and this one is kept as an
// opt-in alternative (same results to rounding).
#include <hip/hip_cooperative_groups.h>

#include "nmf_device.h"

namespace nmf {

// Grid-wide barrier of the cooperative launch (all workgroups co-resident).
__device__ __forceinline__ bool grid_barrier() {
  cooperative_groups::this_grid().sync();
  return true;
}

template <int BC, int KB, bool JOINT>
constexpr int fused_lds_floats() {
  constexpr bool C2_TILE = JOINT && (BC != BC_B1);
  constexpr int a = rows_item_lds<KB>() / 4;
  constexpr int b = cols_item_lds<KB, C2_TILE>() / 4;
  constexpr int c = 32 * KB * 33 * 2;  // update_h's [KP][33] doubles
  return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

template <int BC, int KB, bool JOINT, bool OBJ>
__global__ __launch_bounds__(kBlock, 1) void fused_step_kernel(FusedArgs f) {
  constexpr int KP = 32 * KB;
  __shared__ __align__(16) float lds[fused_lds_floats<BC, KB, JOINT>()];
  __shared__ double scratch[2 * kBlock];
  __shared__ float norm_s[KP], csum_s[KP];
  __shared__ double red[kWaves];
  const int G = gridDim.x;
  const int tid = threadIdx.x;
  unsigned* flags = f.uw.flags;
  // phase-boundary stamps (100 MHz constant clock), workgroup 0 only
  auto stamp = [&](int i) {
    if (f.stamps && blockIdx.x == 0 && tid == 0) f.stamps[i] = wall_clock64();
  };
  stamp(0);

  // 1. W pass
  double objsum = 0.0;
  for (int item = blockIdx.x; item < f.n_items_w; item += G)
    rows_item<BC, KB, KIND_UPDATE, OBJ, JOINT>(f.r, item, lds, objsum);
  if (OBJ) {
    const double sum = block_sum(objsum, red);
    if (tid == 0) f.r.pobj[blockIdx.x] = sum;
  }
  stamp(1);
  grid_barrier();
  stamp(2);

  // 2. W update (the alternating H pass forms Lambda' from W_new^T)
  {
    const int k = tid % KP;
    double den1 = 0.0;
    if (f.uw.beta_one && k < f.uw.K)
      for (int g = 0; g < f.uw.n_groups; ++g) den1 += (double)f.uw.prs[g * KP + k];
    double nrm = 0.0, cs = 0.0;
    const int units = (f.uw.F + unit_rows<KB>() - 1) / unit_rows<KB>();
    for (int u = blockIdx.x; u < units; u += G) update_w_unit<KB>(f.uw, u, !JOINT, lds, den1, nrm, cs);
    __syncthreads();
    scratch[tid] = nrm;
    scratch[kBlock + tid] = cs;
    __syncthreads();
    if (tid < KP) {
      double x = 0.0, y = 0.0;
      for (int j = 0; j < kBlock / KP; ++j) { x += scratch[j * KP + tid]; y += scratch[kBlock + j * KP + tid]; }
      f.uw.pcol[(int64_t)blockIdx.x * 2 * KP + tid] = x;
      f.uw.pcol[(int64_t)blockIdx.x * 2 * KP + KP + tid] = y;
    }
  }
  stamp(3);
  grid_barrier();
  stamp(4);

  // 3. H pass, and the column norms / sums of W_new (one column per workgroup)
  for (int item = blockIdx.x; item < f.n_items_h; item += G)
    cols_item<BC, KB, KIND_UPDATE, JOINT, JOINT>(f.c, item, lds);
  for (int k = blockIdx.x; k < KP; k += G) {
    double x = 0.0, y = 0.0;
    for (int b = tid; b < G; b += kBlock) {
      x += f.uw.pcol[(int64_t)b * 2 * KP + k];
      y += f.uw.pcol[(int64_t)b * 2 * KP + KP + k];
    }
    x = block_sum(x, red);
    y = block_sum(y, red);
    if (tid == 0) {
      f.colsum[k] = (float)sqrt(x);
      f.colsum[KP + k] = (float)y;
    }
  }
  stamp(5);
  grid_barrier();
  stamp(6);

  // 4. H update, normalized W, objective total
  if (tid < KP) {
    norm_s[tid] = f.colsum[tid];
    csum_s[tid] = f.colsum[KP + tid];
  }
  __syncthreads();
  if (OBJ && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = tid; i < G; i += kBlock) s += f.r.pobj[i];
    s = block_sum(s, red);
    if (tid == 0) {
      *f.uh.d_obj = s;
      if (!isfinite(s)) set_flag(flags, 1u);
    }
  }
  double* S = reinterpret_cast<double*>(lds);
  for (int nt = blockIdx.x; nt < f.ntiles; nt += G) update_h_tile<KB>(f.uh, nt, norm_s, csum_s, S);
  write_w<KB>(f.uh, norm_s, (int64_t)blockIdx.x * kBlock + tid, (int64_t)G * kBlock);
  stamp(7);
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <int BC, int KB, bool JOINT, bool OBJ>
static const void* fused_fn() {
  return reinterpret_cast<const void*>(&fused_step_kernel<BC, KB, JOINT, OBJ>);
}

template <int BC, int KB>
static const void* fused_pick2(bool joint, bool obj) {
  if (joint) return obj ? fused_fn<BC, KB, true, true>() : fused_fn<BC, KB, true, false>();
  return obj ? fused_fn<BC, KB, false, true>() : fused_fn<BC, KB, false, false>();
}

template <int BC>
static const void* fused_pick1(int kb, bool joint, bool obj) {
  switch (kb) {
    case 1: return fused_pick2<BC, 1>(joint, obj);
    case 2: return fused_pick2<BC, 2>(joint, obj);
  }
  return nullptr;
}

static const void* fused_pick(int bc, int kb, bool joint, bool obj) {
  switch (bc) {
    case BC_GEN: return fused_pick1<BC_GEN>(kb, joint, obj);
    case BC_B2: return fused_pick1<BC_B2>(kb, joint, obj);
    case BC_B1: return fused_pick1<BC_B1>(kb, joint, obj);
    case BC_B0: return fused_pick1<BC_B0>(kb, joint, obj);
    case BC_B05: return fused_pick1<BC_B05>(kb, joint, obj);
    case BC_B15: return fused_pick1<BC_B15>(kb, joint, obj);
  }
  return nullptr;
}

int fused_max_blocks(int bc, int kb, bool joint, bool obj, int num_cus) {
  const void* fn = fused_pick(bc, kb, joint, obj);
  if (!fn) return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0) != hipSuccess) return 0;
  return per_cu * num_cus;
}

hipError_t launch_fused(int bc, int kb, bool joint, bool obj, int grid, hipStream_t s, const FusedArgs& a) {
  const void* fn = fused_pick(bc, kb, joint, obj);
  if (!fn) return hipErrorNotSupported;
  FusedArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBlock), args, 0, s);
}

}  // namespace nmf
