// The W pass with bfloat16 / float16 matrix products (float32 accumulation,
// float32 element-wise terms, float64 objective).  With STORE_PQ (joint mode)
// it keeps P, Q in the product type for the H pass.
#include "nmf_device.h"

namespace nmf {

template <int BC, int KB, bool OBJ, class T, bool PQ>
__global__ __launch_bounds__(kBlock, 2) void sweep_rows_lp_kernel(SweepRowsArgs a) {
  if (a.halt && *a.halt) return;
  __shared__ __align__(16) float lds[rows_item_lds<KB>() / 4];
  __shared__ double dred[kWaves];
  double objsum = 0.0;
  rows_item_lp<BC, KB, OBJ, T, PQ>(a, blockIdx.x, lds, objsum);
  if (OBJ) {
    const double sum = block_sum(objsum, dred);
    if (threadIdx.x == 0) a.pobj[blockIdx.x] = sum;
  }
}

template <int BC, int KB, class T>
static hipError_t rows_lp3(bool obj, bool pq, int grid, hipStream_t s, const SweepRowsArgs& a) {
  if (pq) {
    if (obj) hipLaunchKernelGGL((sweep_rows_lp_kernel<BC, KB, true, T, true>), dim3(grid), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((sweep_rows_lp_kernel<BC, KB, false, T, true>), dim3(grid), dim3(kBlock), 0, s, a);
  } else {
    if (obj) hipLaunchKernelGGL((sweep_rows_lp_kernel<BC, KB, true, T, false>), dim3(grid), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((sweep_rows_lp_kernel<BC, KB, false, T, false>), dim3(grid), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

template <class T, int BC>
static hipError_t rows_lp2(int kb, bool obj, bool pq, int grid, hipStream_t s, const SweepRowsArgs& a) {
  if (kb == 1) return rows_lp3<BC, 1, T>(obj, pq, grid, s, a);
  if (kb == 2) return rows_lp3<BC, 2, T>(obj, pq, grid, s, a);
  return hipErrorInvalidValue;
}

template <class T>
static hipError_t rows_lp1(int bc, int kb, bool obj, bool pq, int grid, hipStream_t s, const SweepRowsArgs& a) {
  switch (bc) {
    case BC_GEN: return rows_lp2<T, BC_GEN>(kb, obj, pq, grid, s, a);
    case BC_B2: return rows_lp2<T, BC_B2>(kb, obj, pq, grid, s, a);
    case BC_B1: return rows_lp2<T, BC_B1>(kb, obj, pq, grid, s, a);
    case BC_B0: return rows_lp2<T, BC_B0>(kb, obj, pq, grid, s, a);
    case BC_B05: return rows_lp2<T, BC_B05>(kb, obj, pq, grid, s, a);
    case BC_B15: return rows_lp2<T, BC_B15>(kb, obj, pq, grid, s, a);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_rows_lp(int prec, int bc, int kb, bool obj, bool pq, int grid, hipStream_t s,
                                const SweepRowsArgs& a) {
  if (prec == 1) return rows_lp1<__bf16>(bc, kb, obj, pq, grid, s, a);
  if (prec == 2) return rows_lp1<_Float16>(bc, kb, obj, pq, grid, s, a);
  return hipErrorInvalidValue;
}

}  // namespace nmf
