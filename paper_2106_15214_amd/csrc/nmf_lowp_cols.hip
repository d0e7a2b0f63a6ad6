// The H pass with bfloat16 / float16 matrix products.  Joint mode with kept
// P, Q (PQ) contracts them directly; otherwise Lambda (joint: W~ H~, from the
// row-major W~ copy; alternating: W_new H~) is formed from split operands.
#include "nmf_device.h"

namespace nmf {

template <int BC, int KB, bool DUAL, class T>
__global__ __launch_bounds__(kBlock, 2) void sweep_cols_lp_kernel(SweepColsArgs a) {
  if (a.halt && *a.halt) return;
  __shared__ __align__(16) float lds[cols_item_lp_lds<KB, DUAL && (BC != BC_B1)>() / 4];
  static_assert(cols_item_lp_lds<KB, DUAL && (BC != BC_B1)>() >= 2 * kBlock * 8, "column partial scratch");
  cols_prologue<KB>(a, blockIdx.x, lds);
  cols_item_lp<BC, KB, DUAL, T>(a, blockIdx.x, lds);
}

template <int BC, int KB, class T>
__global__ __launch_bounds__(kBlock, 2) void sweep_cols_lp_pq_kernel(SweepColsArgs a) {
  if (a.halt && *a.halt) return;
  __shared__ __align__(16) float lds[cols_item_lp_lds<KB, BC != BC_B1>() / 4];
  static_assert(cols_item_lp_lds<KB, BC != BC_B1>() >= 2 * kBlock * 8, "column partial scratch");
  cols_prologue<KB>(a, blockIdx.x, lds);
  cols_item_lp_pq<BC, KB, T>(a, blockIdx.x, lds);
}

template <int BC, int KB, class T>
static hipError_t cols_lp3(bool dual, bool pq, int grid, hipStream_t s, const SweepColsArgs& a) {
  if (dual && pq) hipLaunchKernelGGL((sweep_cols_lp_pq_kernel<BC, KB, T>), dim3(grid), dim3(kBlock), 0, s, a);
  else if (dual) hipLaunchKernelGGL((sweep_cols_lp_kernel<BC, KB, true, T>), dim3(grid), dim3(kBlock), 0, s, a);
  else hipLaunchKernelGGL((sweep_cols_lp_kernel<BC, KB, false, T>), dim3(grid), dim3(kBlock), 0, s, a);
  return hipGetLastError();
}

template <class T, int BC>
static hipError_t cols_lp2(int kb, bool dual, bool pq, int grid, hipStream_t s, const SweepColsArgs& a) {
  if (kb == 1) return cols_lp3<BC, 1, T>(dual, pq, grid, s, a);
  if (kb == 2) return cols_lp3<BC, 2, T>(dual, pq, grid, s, a);
  return hipErrorInvalidValue;
}

template <class T>
static hipError_t cols_lp1(int bc, int kb, bool dual, bool pq, int grid, hipStream_t s, const SweepColsArgs& a) {
  switch (bc) {
    case BC_GEN: return cols_lp2<T, BC_GEN>(kb, dual, pq, grid, s, a);
    case BC_B2: return cols_lp2<T, BC_B2>(kb, dual, pq, grid, s, a);
    case BC_B1: return cols_lp2<T, BC_B1>(kb, dual, pq, grid, s, a);
    case BC_B0: return cols_lp2<T, BC_B0>(kb, dual, pq, grid, s, a);
    case BC_B05: return cols_lp2<T, BC_B05>(kb, dual, pq, grid, s, a);
    case BC_B15: return cols_lp2<T, BC_B15>(kb, dual, pq, grid, s, a);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_sweep_cols_lp(int prec, int bc, int kb, bool dual, bool pq, int grid, hipStream_t s,
                                const SweepColsArgs& a) {
  if (prec == 1) return cols_lp1<__bf16>(bc, kb, dual, pq, grid, s, a);
  if (prec == 2) return cols_lp1<_Float16>(bc, kb, dual, pq, grid, s, a);
  return hipErrorInvalidValue;
}

}  // namespace nmf
