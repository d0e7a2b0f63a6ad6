// Batched persistent step with float32 matrix products.
#include "nmf_batched.h"

namespace nmf {

const void* batched_kernel_f32(bool joint) {
  return joint ? reinterpret_cast<const void*>(&batched_step_kernel<0, true, true>)
               : reinterpret_cast<const void*>(&batched_step_kernel<0, false, true>);
}

}  // namespace nmf
