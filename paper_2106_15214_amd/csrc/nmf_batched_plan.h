// Device-side planner of nmf_beta_step_batched (nmf_batched_plan.hip).
#pragma once

#include "nmf_plan.h"

namespace nmf {

struct BatchPlanArgs {
  const nmf_problem* problems;  // [count] descriptors in device memory
  int count;                    // descriptors available
  const int* d_count;           // nullable: descriptors used (0 .. count), read on the device
  const int* tiles;             // [kBatchBuckets] tiles per pass item of each bucket
  int joint;
  nmf_step_opts opts;
  char* work;                   // problem workspaces
  int64_t work_bytes;
  int64_t max_items;
  // planner scratch: [count] or [4 count]
  int64_t* s_bytes;
  int64_t* s_items;
  int64_t* s_off;
  int* s_order;
  // outputs read by the persistent kernel
  BatchProblem* desc;   // [count]
  int2* list;           // [max_items]
  unsigned* done;       // [4 count]
  unsigned* next;
  unsigned* exited;
  int* counts;          // [0] items listed, [1] problems
  unsigned* flags;
};

hipError_t launch_batch_plan(hipStream_t s, const BatchPlanArgs& a);

}  // namespace nmf
