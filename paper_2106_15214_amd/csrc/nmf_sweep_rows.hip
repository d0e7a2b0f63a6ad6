// The W pass of the streaming path: one pass over V along rows per launch
// (rows items of nmf_device.h).  With STORE_PQ (joint mode) it also keeps the
// element-wise terms P, Q of the tilde iterate for the H pass.
#include "nmf_device.h"

namespace nmf {

template <int BC, int KB, int KIND, bool OBJ, bool STORE_PQ>
__global__ __launch_bounds__(kBlock, sweep_rows_occupancy(KB)) void sweep_rows_kernel(SweepRowsArgs a) {
  if (a.halt && *a.halt) return;
  __shared__ __align__(16) float lds[rows_item_lds<KB>() / 4];
  __shared__ double dred[kWaves];
  double objsum = 0.0;
  rows_item<BC, KB, KIND, OBJ, STORE_PQ>(a, blockIdx.x, lds, objsum);
  if (OBJ) {
    const double sum = block_sum(objsum, dred);
    if (threadIdx.x == 0) a.pobj[blockIdx.x] = sum;
  }
}

// The W pass of a later joint sub-iteration (contractions of the kept P, Q tiles).
template <int BC, int KB>
__global__ __launch_bounds__(kBlock, sweep_rows_occupancy(KB)) void sweep_rows_pq_kernel(SweepRowsArgs a) {
  if (a.halt && *a.halt) return;
  __shared__ __align__(16) float lds[rows_pq_item_lds<KB>() / 4];
  rows_pq_item<BC, KB>(a, blockIdx.x, lds);
}

template <int BC>
static hipError_t rows_pq_bc(int kb, int grid, hipStream_t s, const SweepRowsArgs& a) {
  switch (kb) {
    case 1: hipLaunchKernelGGL((sweep_rows_pq_kernel<BC, 1>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 2: hipLaunchKernelGGL((sweep_rows_pq_kernel<BC, 2>), dim3(grid), dim3(kBlock), 0, s, a); break;
    case 4: hipLaunchKernelGGL((sweep_rows_pq_kernel<BC, 4>), dim3(grid), dim3(kBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sweep_rows_pq(int bc, int kb, int grid, hipStream_t s, const SweepRowsArgs& a) {
  switch (bc) {
    case BC_GEN: return rows_pq_bc<BC_GEN>(kb, grid, s, a);
    case BC_B2: return rows_pq_bc<BC_B2>(kb, grid, s, a);
    case BC_B1: return rows_pq_bc<BC_B1>(kb, grid, s, a);
    case BC_B0: return rows_pq_bc<BC_B0>(kb, grid, s, a);
    case BC_B05: return rows_pq_bc<BC_B05>(kb, grid, s, a);
    case BC_B15: return rows_pq_bc<BC_B15>(kb, grid, s, a);
  }
  return hipErrorInvalidValue;
}

// launchers: map runtime (beta class, K block count, kind) to instantiations
template <int BC, int KB>
static hipError_t rows_kb(int kind, bool obj, bool pq, int grid, hipStream_t s, const SweepRowsArgs& a) {
  if (kind == KIND_UPDATE) {
    if (pq) {
      if (obj) hipLaunchKernelGGL((sweep_rows_kernel<BC, KB, KIND_UPDATE, true, true>), dim3(grid), dim3(kBlock), 0, s, a);
      else hipLaunchKernelGGL((sweep_rows_kernel<BC, KB, KIND_UPDATE, false, true>), dim3(grid), dim3(kBlock), 0, s, a);
    } else {
      if (obj) hipLaunchKernelGGL((sweep_rows_kernel<BC, KB, KIND_UPDATE, true, false>), dim3(grid), dim3(kBlock), 0, s, a);
      else hipLaunchKernelGGL((sweep_rows_kernel<BC, KB, KIND_UPDATE, false, false>), dim3(grid), dim3(kBlock), 0, s, a);
    }
  } else if (kind == KIND_GRAD) {
    if (obj) hipLaunchKernelGGL((sweep_rows_kernel<BC, KB, KIND_GRAD, true, false>), dim3(grid), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((sweep_rows_kernel<BC, KB, KIND_GRAD, false, false>), dim3(grid), dim3(kBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL((sweep_rows_kernel<BC, KB, KIND_OBJ, true, false>), dim3(grid), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

template <int BC>
static hipError_t rows_bc(int kb, int kind, bool obj, bool pq, int grid, hipStream_t s, const SweepRowsArgs& a) {
  switch (kb) {
    case 1: return rows_kb<BC, 1>(kind, obj, pq, grid, s, a);
    case 2: return rows_kb<BC, 2>(kind, obj, pq, grid, s, a);
    case 4: return rows_kb<BC, 4>(kind, obj, pq, grid, s, a);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_rows(int bc, int kb, int kind, bool obj, bool pq, int grid, hipStream_t s,
                             const SweepRowsArgs& a) {
  if (bc == BC_B2G) {  // Gram form at beta = 2: update passes with K <= 64, no kept P, Q
    if (kind != KIND_UPDATE || pq || kb > 2) return hipErrorInvalidValue;
    if (kb == 1) {
      if (obj) hipLaunchKernelGGL((sweep_rows_kernel<BC_B2G, 1, KIND_UPDATE, true, false>), dim3(grid), dim3(kBlock), 0, s, a);
      else hipLaunchKernelGGL((sweep_rows_kernel<BC_B2G, 1, KIND_UPDATE, false, false>), dim3(grid), dim3(kBlock), 0, s, a);
    } else {
      if (obj) hipLaunchKernelGGL((sweep_rows_kernel<BC_B2G, 2, KIND_UPDATE, true, false>), dim3(grid), dim3(kBlock), 0, s, a);
      else hipLaunchKernelGGL((sweep_rows_kernel<BC_B2G, 2, KIND_UPDATE, false, false>), dim3(grid), dim3(kBlock), 0, s, a);
    }
    return hipGetLastError();
  }
  switch (bc) {
    case BC_GEN: return rows_bc<BC_GEN>(kb, kind, obj, pq, grid, s, a);
    case BC_B2: return rows_bc<BC_B2>(kb, kind, obj, pq, grid, s, a);
    case BC_B1: return rows_bc<BC_B1>(kb, kind, obj, pq, grid, s, a);
    case BC_B0: return rows_bc<BC_B0>(kb, kind, obj, pq, grid, s, a);
    case BC_B05: return rows_bc<BC_B05>(kb, kind, obj, pq, grid, s, a);
    case BC_B15: return rows_bc<BC_B15>(kb, kind, obj, pq, grid, s, a);
  }
  return hipErrorInvalidValue;
}

}  // namespace nmf
