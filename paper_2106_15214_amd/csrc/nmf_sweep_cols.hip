// The H pass of the streaming path: one pass over V along columns per launch
// (cols items of nmf_device.h).  With LOAD_PQ (joint mode) it contracts the
// element-wise terms P, Q kept by the W pass instead of forming Lambda again.
#include "nmf_device.h"

namespace nmf {

template <int BC, int KB, int KIND, bool DUAL, bool LOAD_PQ>
__global__ __launch_bounds__(kBlock, sweep_cols_occupancy(BC, KB, KIND, DUAL)) void sweep_cols_kernel(
    SweepColsArgs a) {
  if (a.halt && *a.halt) return;
  constexpr bool C2_TILE = DUAL && (KIND == KIND_UPDATE) && (BC != BC_B1);
  __shared__ __align__(16) float lds[cols_item_lds<KB, C2_TILE>() / 4];
  static_assert(cols_item_lds<KB, C2_TILE>() >= 2 * kBlock * 8, "column partial scratch");
  if (KIND == KIND_UPDATE) cols_prologue<KB>(a, blockIdx.x, lds);
  cols_item<BC, KB, KIND, DUAL, LOAD_PQ>(a, blockIdx.x, lds);
}

template <int BC, int KB>
static hipError_t cols_kb(int kind, bool dual, bool pq, int grid, hipStream_t s, const SweepColsArgs& a) {
  if (kind == KIND_UPDATE) {
    if (dual && pq) hipLaunchKernelGGL((sweep_cols_kernel<BC, KB, KIND_UPDATE, true, true>), dim3(grid), dim3(kBlock), 0, s, a);
    else if (dual) hipLaunchKernelGGL((sweep_cols_kernel<BC, KB, KIND_UPDATE, true, false>), dim3(grid), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((sweep_cols_kernel<BC, KB, KIND_UPDATE, false, false>), dim3(grid), dim3(kBlock), 0, s, a);
  } else {
    hipLaunchKernelGGL((sweep_cols_kernel<BC, KB, KIND_GRAD, false, false>), dim3(grid), dim3(kBlock), 0, s, a);
  }
  return hipGetLastError();
}

template <int BC>
static hipError_t cols_bc(int kb, int kind, bool dual, bool pq, int grid, hipStream_t s, const SweepColsArgs& a) {
  switch (kb) {
    case 1: return cols_kb<BC, 1>(kind, dual, pq, grid, s, a);
    case 2: return cols_kb<BC, 2>(kind, dual, pq, grid, s, a);
    case 4: return cols_kb<BC, 4>(kind, dual, pq, grid, s, a);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_cols(int bc, int kb, int kind, bool dual, bool pq, int grid, hipStream_t s,
                             const SweepColsArgs& a) {
  if (bc == BC_B2G) {  // Gram form at beta = 2: numerators chi_1^T V only (C1 = W_new in both modes)
    if (kind != KIND_UPDATE || pq || kb > 2) return hipErrorInvalidValue;
    if (kb == 1) hipLaunchKernelGGL((sweep_cols_kernel<BC_B2G, 1, KIND_UPDATE, false, false>), dim3(grid), dim3(kBlock), 0, s, a);
    else hipLaunchKernelGGL((sweep_cols_kernel<BC_B2G, 2, KIND_UPDATE, false, false>), dim3(grid), dim3(kBlock), 0, s, a);
    return hipGetLastError();
  }
  switch (bc) {
    case BC_GEN: return cols_bc<BC_GEN>(kb, kind, dual, pq, grid, s, a);
    case BC_B2: return cols_bc<BC_B2>(kb, kind, dual, pq, grid, s, a);
    case BC_B1: return cols_bc<BC_B1>(kb, kind, dual, pq, grid, s, a);
    case BC_B0: return cols_bc<BC_B0>(kb, kind, dual, pq, grid, s, a);
    case BC_B05: return cols_bc<BC_B05>(kb, kind, dual, pq, grid, s, a);
    case BC_B15: return cols_bc<BC_B15>(kb, kind, dual, pq, grid, s, a);
  }
  return hipErrorInvalidValue;
}

}  // namespace nmf
