// Many beta-NMF problems of uneven sizes, each with its own beta and rank, in
// one persistent launch.  Workgroups take work items from a queue listed
// phase-major over all problems:
//   W-pass items  (rows items: Lambda~ tiles, P, Q, W-step partials, objective;
//                  in joint mode P and Q are kept for the H pass)
//   W-update items (partials reduced, W_new, chi terms; 64 rows each, all loads
//                  in flight together)
//   H-pass items  (cols items: H-step partials from the kept P, Q in joint mode,
//                  column sums of W_new)
//   H-update units (H_new, normalization, W write-back, objective total)
// A problem whose rows take one column group has no W-update items: its W-pass
// items apply the W update.  If its columns also take one row group it
// has no H-update items either: its W-pass items also write the column
// partials of W_new and its H-pass items apply the H update and write W back.
// A per-problem counter of finished items per phase replaces grid barriers: an
// item waits until its problem's nearest earlier phase that has items is
// complete.  Every item it can wait for was taken from the queue before it by a
// running workgroup, so the wait ends without co-residency of the grid.
#pragma once

#include "nmf_device.h"
#include "nmf_plan.h"

namespace nmf {

// Largest LDS footprint of any item: the float32 joint H pass at KB = 2.
constexpr int kBatchLdsBytes = cols_item_lds<2, true>();
static_assert(cols_item_lp_lds<2, true>() <= kBatchLdsBytes, "batched LDS");
static_assert(rows_item_lds<2>() <= kBatchLdsBytes, "batched LDS");
static_assert(2 * kBlock * 8 <= kBatchLdsBytes, "batched LDS");
static_assert(kBatchWRows * (64 + 1) * 4 <= kBatchLdsBytes, "batched LDS");

// Joint MM keeps P, Q between its passes only at K > 32 (two K blocks) and
// beta != 1; elsewhere its H pass forms Lambda~ again from a copy of W~.  The
// same rule as batch_keeps_pq, fixed per instantiation.
template <int BC, int KB, int PREC, bool JOINT>
constexpr bool kKeepPQ = JOINT && KB > 1 && BC != BC_B1;

// Descriptors never change during the launch: reading them through the
// constant address space lets the compiler keep their fields in scalar
// registers.
typedef const __attribute__((address_space(4))) BatchProblem* ConstProblemPtr;

// Copies a descriptor field group out of constant memory (dword by dword).
template <class T>
__device__ __forceinline__ T load_const(const __attribute__((address_space(4))) T* p) {
  static_assert(sizeof(T) % 4 == 0, "dword copy");
  T r;
  const __attribute__((address_space(4))) uint32_t* s = (const __attribute__((address_space(4))) uint32_t*)p;
  uint32_t* d = reinterpret_cast<uint32_t*>(&r);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = s[i];
  return r;
}

// W-pass item of a problem whose rows take one column group: the item applies
// the W update from its accumulators; its objective terms are added to
// the caller's objsum.  A function of its own, so that its registers are
// allocated apart from the other phases'.  (Like batch_item it is handed a
// reference into its caller's frame, which keeps the call from being marked as
// one that could skip the caller's frame; such calls make the callee save the
// callee-saved registers it uses, hundreds of bytes per lane per item.)
template <int BC, int KB, int PREC, bool JOINT, bool OBJ>
__device__ __noinline__ void batch_wpass_fused(ConstProblemPtr P, int item, float* lds, double& objsum) {
  const SweepRowsArgs ra = load_const(&P->ra);
  constexpr bool KEEP = kKeepPQ<BC, KB, PREC, JOINT>;
  if constexpr (PREC == 0)
    rows_item<BC, KB, KIND_UPDATE, OBJ, KEEP, true, JOINT && !KEEP>(ra, item, lds, objsum, &P->ua);
  else rows_item_lp<BC, KB, OBJ, __bf16, KEEP, true, JOINT && !KEEP>(ra, item, lds, objsum, &P->ua);
}

// H-pass item of a problem whose W-pass items applied the W update and
// whose columns take one row group: the column norms and sums of W_new from
// the W pass's row-block partials, the H-step contractions of the item's
// columns, the H update of those columns, this item's share of the W
// write-back, and (item 0) the objective total.
template <int BC, int KB, int PREC, bool JOINT, bool OBJ>
__device__ __noinline__ void batch_hpass_fused(ConstProblemPtr P, int prob, int item, const BatchArgs& b,
                                               float* lds, double* red, float* norm_s, float* csum_s) {
  reduce_columns<KB>(P->ha.pcol, P->ha.pcol_blocks, reinterpret_cast<double*>(lds), norm_s, csum_s);
  {
    const SweepColsArgs ca = load_const(&P->ca);
    constexpr bool KEEP = kKeepPQ<BC, KB, PREC, JOINT>;
    if constexpr (PREC == 0) cols_item<BC, KB, KIND_UPDATE, JOINT, KEEP, true>(ca, item, lds, &P->ha, norm_s, csum_s);
    else if constexpr (KEEP) cols_item_lp_pq<BC, KB, __bf16, true>(ca, item, lds, &P->ha, norm_s, csum_s);
    else cols_item_lp<BC, KB, JOINT, __bf16, true>(ca, item, lds, &P->ha, norm_s, csum_s);
  }
  const UpdateHArgs ha = load_const(&P->ha);
  const int items = P->items[PH_HPASS];
  write_w<KB>(ha, norm_s, (int64_t)item * kBlock + threadIdx.x, (int64_t)items * kBlock);
  if (OBJ && item == 0 && b.d_obj) {
    double s = 0.0;
    for (int i = threadIdx.x; i < ha.nobj; i += kBlock) s += ha.pobj[i];
    s = block_sum(s, red);
    if (threadIdx.x == 0) {
      b.d_obj[prob] = s;
      if (!isfinite(s)) set_flag(b.flags, 1u);
    }
  }
}

// One work item.  Not inlined: each (beta class, K block, phase) path is its
// own function with its own register allocation, so the persistent kernel's
// budget is the largest single path and not the union of all of them inlined
// into one body (which spilled heavily); this is what lets two workgroups share
// a compute unit.
template <int BC, int KB, int PREC, bool JOINT, bool OBJ>
__device__ __noinline__ void batch_item(ConstProblemPtr P, int prob, int phase, int item, const BatchArgs& b,
                                           float* lds, double* red, float* norm_s, float* csum_s) {
  if (phase == PH_WPASS) {
    const SweepRowsArgs ra = load_const(&P->ra);
    double objsum = 0.0;
    if constexpr (PREC == 0) rows_item<BC, KB, KIND_UPDATE, OBJ, kKeepPQ<BC, KB, PREC, JOINT>>(ra, item, lds, objsum);
    else if constexpr (PREC == 1) rows_item_lp<BC, KB, OBJ, __bf16, kKeepPQ<BC, KB, PREC, JOINT>>(ra, item, lds, objsum);
    else rows_item_lp<BC, KB, OBJ, _Float16, JOINT>(ra, item, lds, objsum);
    if (OBJ) {
      const double sum = block_sum(objsum, red);
      if (threadIdx.x == 0) ra.pobj[item] = sum;
    }
  } else if (phase == PH_WUPDATE) {
    // the transposed factor that forms Lambda in the H pass (W_new for
    // alternating MU, W~ for joint MM without kept P, Q); a joint H pass that
    // contracts the kept P, Q never forms Lambda again
    const UpdateWArgs ua = load_const(&P->ua);
    update_w_rows<KB, kBatchWRows>(ua, item * kBatchWRows, !kKeepPQ<BC, KB, PREC, JOINT>, row_sum_den<KB>(ua), lds);
  } else if (phase == PH_HPASS) {
    const SweepColsArgs ca = load_const(&P->ca);
    cols_prologue<KB>(ca, item, lds);
    if constexpr (PREC == 0) cols_item<BC, KB, KIND_UPDATE, JOINT, kKeepPQ<BC, KB, PREC, JOINT>>(ca, item, lds);
    else if constexpr (PREC == 1) {
      if constexpr (kKeepPQ<BC, KB, PREC, JOINT>) cols_item_lp_pq<BC, KB, __bf16>(ca, item, lds);
      else cols_item_lp<BC, KB, JOINT, __bf16>(ca, item, lds);
    } else {
      if constexpr (JOINT) cols_item_lp_pq<BC, KB, _Float16>(ca, item, lds);
      else cols_item_lp<BC, KB, false, _Float16>(ca, item, lds);
    }
  } else {
    const UpdateHArgs ha = load_const(&P->ha);
    reduce_columns<KB>(ha.pcol, ha.pcol_blocks, reinterpret_cast<double*>(lds), norm_s, csum_s);
    if (OBJ && item == 0 && b.d_obj) {
      double s = 0.0;
      for (int i = threadIdx.x; i < ha.nobj; i += kBlock) s += ha.pobj[i];
      s = block_sum(s, red);
      if (threadIdx.x == 0) {
        b.d_obj[prob] = s;
        if (!isfinite(s)) set_flag(b.flags, 1u);
      }
    }
    const int items = P->items[PH_HUPDATE];
    write_w<KB>(ha, norm_s, (int64_t)item * kBlock + threadIdx.x, (int64_t)items * kBlock);
    const int per = P->per_item[PH_HUPDATE];
    const int u1 = min(P->units[PH_HUPDATE], (item + 1) * per);
    update_h_cols_multi<KB, 8>(ha, item * per, u1, norm_s, csum_s);
  }
}

template <int KB, int PREC, bool JOINT, bool OBJ>
__device__ __forceinline__ void batch_item_bc(int bc, ConstProblemPtr P, int prob, int phase, int item,
                                              const BatchArgs& b, float* lds, double* red, float* norm_s,
                                              float* csum_s) {
  switch (bc) {
    case BC_GEN: batch_item<BC_GEN, KB, PREC, JOINT, OBJ>(P, prob, phase, item, b, lds, red, norm_s, csum_s); break;
    case BC_B2: batch_item<BC_B2, KB, PREC, JOINT, OBJ>(P, prob, phase, item, b, lds, red, norm_s, csum_s); break;
    case BC_B1: batch_item<BC_B1, KB, PREC, JOINT, OBJ>(P, prob, phase, item, b, lds, red, norm_s, csum_s); break;
    case BC_B0: batch_item<BC_B0, KB, PREC, JOINT, OBJ>(P, prob, phase, item, b, lds, red, norm_s, csum_s); break;
    case BC_B05: batch_item<BC_B05, KB, PREC, JOINT, OBJ>(P, prob, phase, item, b, lds, red, norm_s, csum_s); break;
    default: batch_item<BC_B15, KB, PREC, JOINT, OBJ>(P, prob, phase, item, b, lds, red, norm_s, csum_s); break;
  }
}

template <int KB, int PREC, bool JOINT, bool OBJ>
__device__ __forceinline__ void batch_wpass_fused_bc(int bc, ConstProblemPtr P, int item, float* lds,
                                                     double& objsum) {
  switch (bc) {
    case BC_GEN: batch_wpass_fused<BC_GEN, KB, PREC, JOINT, OBJ>(P, item, lds, objsum); break;
    case BC_B2: batch_wpass_fused<BC_B2, KB, PREC, JOINT, OBJ>(P, item, lds, objsum); break;
    case BC_B1: batch_wpass_fused<BC_B1, KB, PREC, JOINT, OBJ>(P, item, lds, objsum); break;
    case BC_B0: batch_wpass_fused<BC_B0, KB, PREC, JOINT, OBJ>(P, item, lds, objsum); break;
    case BC_B05: batch_wpass_fused<BC_B05, KB, PREC, JOINT, OBJ>(P, item, lds, objsum); break;
    default: batch_wpass_fused<BC_B15, KB, PREC, JOINT, OBJ>(P, item, lds, objsum); break;
  }
}

template <int KB, int PREC, bool JOINT, bool OBJ>
__device__ __forceinline__ void batch_hpass_fused_bc(int bc, ConstProblemPtr P, int prob, int item,
                                                     const BatchArgs& b, float* lds, double* red, float* norm_s,
                                                     float* csum_s) {
  switch (bc) {
    case BC_GEN: batch_hpass_fused<BC_GEN, KB, PREC, JOINT, OBJ>(P, prob, item, b, lds, red, norm_s, csum_s); break;
    case BC_B2: batch_hpass_fused<BC_B2, KB, PREC, JOINT, OBJ>(P, prob, item, b, lds, red, norm_s, csum_s); break;
    case BC_B1: batch_hpass_fused<BC_B1, KB, PREC, JOINT, OBJ>(P, prob, item, b, lds, red, norm_s, csum_s); break;
    case BC_B0: batch_hpass_fused<BC_B0, KB, PREC, JOINT, OBJ>(P, prob, item, b, lds, red, norm_s, csum_s); break;
    case BC_B05: batch_hpass_fused<BC_B05, KB, PREC, JOINT, OBJ>(P, prob, item, b, lds, red, norm_s, csum_s); break;
    default: batch_hpass_fused<BC_B15, KB, PREC, JOINT, OBJ>(P, prob, item, b, lds, red, norm_s, csum_s); break;
  }
}

template <int PREC, bool JOINT, bool OBJ>
__global__ __launch_bounds__(kBlock, 2) void batched_step_kernel(BatchArgs b) {
  __shared__ __align__(16) float lds[kBatchLdsBytes / 4];
  __shared__ double red[kWaves];
  __shared__ float norm_s[64], csum_s[64];
  __shared__ int2 entry;
  __shared__ int last;
  const int tid = threadIdx.x;
  const ConstProblemPtr probs = (ConstProblemPtr)b.probs;
  // a batch planned on the device publishes its sizes in memory
  const int total = b.counts ? b.counts[0] : b.total;
  const int nprob = b.counts ? b.counts[1] : b.nprob;

  for (;;) {
    __syncthreads();  // every thread has read the previous entry
    if (tid == 0) {
      const unsigned idx = atomicAdd(b.next, 1u);
      entry = idx < (unsigned)total ? b.list[idx] : make_int2(-1, 0);
    }
    __syncthreads();
    const int prob = __builtin_amdgcn_readfirstlane(entry.x);
    const int code = __builtin_amdgcn_readfirstlane(entry.y);
    if (prob < 0) break;
    const int phase = code >> 24, item = code & 0xffffff;
    ConstProblemPtr P = probs + prob;

    // wait until the nearest earlier phase of this problem that has items is
    // complete (bounded)
    if (phase > 0) {
      if (tid == 0) {
        int pq = phase - 1;
        while (pq > 0 && P->items[pq] == 0) --pq;
        const unsigned need = (unsigned)P->items[pq];
        unsigned* cnt = b.done + 4 * prob + pq;
        unsigned polls = 0;
        // polled with read-modify-write atomics, which are performed where the
        // producers' increments are, never served from a cached copy
        while (__hip_atomic_fetch_add(cnt, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
          if (++polls > b.spin_limit) {
            set_flag(b.flags, 4u);  // gave up waiting: this launch's results are invalid
            break;
          }
          // once any wait has given up, later waits do not spin again
          if ((polls & 1023u) == 0u &&
              (__hip_atomic_fetch_or(b.flags, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & 4u))
            break;
          __builtin_amdgcn_s_sleep(2);
        }
      }
      __syncthreads();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");  // the finished items' writes are visible
    }

    const int kb = P->kb, bc = P->bc;
    bool fused_item = false;
    if constexpr (PREC <= 1) {
      if (phase == PH_WPASS && P->wfused) {
        double objsum = 0.0;
        if (kb == 1) batch_wpass_fused_bc<1, PREC, JOINT, OBJ>(bc, P, item, lds, objsum);
        else batch_wpass_fused_bc<2, PREC, JOINT, OBJ>(bc, P, item, lds, objsum);
        if (OBJ) {
          const double sum = block_sum(objsum, red);
          if (tid == 0) P->ra.pobj[item] = sum;
        }
        fused_item = true;
      } else if (phase == PH_HPASS && P->hfused) {
        if (kb == 1) batch_hpass_fused_bc<1, PREC, JOINT, OBJ>(bc, P, prob, item, b, lds, red, norm_s, csum_s);
        else batch_hpass_fused_bc<2, PREC, JOINT, OBJ>(bc, P, prob, item, b, lds, red, norm_s, csum_s);
        fused_item = true;
      }
    }
    if (!fused_item) {
      if (kb == 1) batch_item_bc<1, PREC, JOINT, OBJ>(bc, P, prob, phase, item, b, lds, red, norm_s, csum_s);
      else batch_item_bc<2, PREC, JOINT, OBJ>(bc, P, prob, phase, item, b, lds, red, norm_s, csum_s);
    }

    // nothing in the launch waits for the H update (its writes are read by the
    // next launch), so only the first three phases publish their items
    if (phase != PH_HUPDATE) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");  // this item's writes before its count
      __syncthreads();
      if (tid == 0) atomicAdd(b.done + 4 * prob + phase, 1u);
    }
  }

  // the last workgroup out resets the queue and the counters for the next launch
  if (tid == 0) {
    __threadfence();
    last = atomicAdd(b.exited, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (last) {
    __threadfence();
    // atomic exchanges: the counters are only ever accessed atomically
    for (int i = tid; i < 4 * nprob; i += kBlock)
      (void)__hip_atomic_exchange(b.done + i, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (tid == 0) {
      (void)__hip_atomic_exchange(b.next, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      (void)__hip_atomic_exchange(b.exited, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// per-precision entry points (one translation unit each, to keep builds parallel)
const void* batched_kernel_f32(bool joint);
const void* batched_kernel_bf16(bool joint);

}  // namespace nmf
