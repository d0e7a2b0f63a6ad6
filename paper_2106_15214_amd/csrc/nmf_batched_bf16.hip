// Batched persistent step with bfloat16 matrix products.
#include "nmf_batched.h"

namespace nmf {

const void* batched_kernel_bf16(bool joint) {
  return joint ? reinterpret_cast<const void*>(&batched_step_kernel<1, true, true>)
               : reinterpret_cast<const void*>(&batched_step_kernel<1, false, true>);
}

}  // namespace nmf
