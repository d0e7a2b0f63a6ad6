// Dispatch of the batched persistent step (kernels in nmf_batched.h,
// instantiated per precision in nmf_batched_f32.hip and nmf_batched_bf16.hip).
// The objective of every problem's entry iterate is always formed; writing it
// out is optional.
#include "nmf_batched.h"

namespace nmf {

static const void* batched_pick(int prec, bool joint) {
  switch (prec) {
    case 0: return batched_kernel_f32(joint);
    case 1: return batched_kernel_bf16(joint);
  }
  return nullptr;
}

int batched_max_blocks(int prec, bool joint, int num_cus) {
  const void* fn = batched_pick(prec, joint);
  if (!fn) return 0;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, kBlock, 0) != hipSuccess) return 0;
  return per_cu * num_cus;
}

hipError_t launch_batched(int prec, bool joint, int grid, hipStream_t s, const BatchArgs& a) {
  const void* fn = batched_pick(prec, joint);
  if (!fn) return hipErrorNotSupported;
  BatchArgs copy = a;
  void* args[] = {&copy};
  return hipLaunchKernel(fn, dim3(grid), dim3(kBlock), args, 0, s);
}

}  // namespace nmf
