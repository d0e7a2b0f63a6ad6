// Device-side planning of a batched step whose problem descriptors live in
// device memory (nmf_beta_step_batched).  One workgroup reads the descriptors,
// checks them, plans every problem's splits and workspace with the functions
// the host planner uses (nmf_plan.h), lays the workspaces out one after
// another, writes the kernel descriptors and the work queue (phase by phase,
// larger problems first, ties by index: the order nmf_batch_create uses), and
// zeroes the completion counters.  The persistent kernel then reads the item
// and problem counts from device memory.  Nothing is allocated and the host
// never waits, so the two launches can be captured in a graph and replayed
// after the descriptors change.
#include "nmf_batched_plan.h"

namespace nmf {

namespace {

constexpr int kPlanThreads = 1024;
constexpr int kPlanWaves = kPlanThreads / 64;
constexpr int kStage = 256;  // descriptors staged in LDS per round of the pairwise checks

// Exclusive prefix sum of x[0..n) in place, by the whole workgroup: one
// contiguous segment per thread, the segment totals scanned across each wave
// with shuffles and across the waves by one wave, the offsets added back.
// *total receives the sum.  seg holds kPlanWaves values.
__device__ void block_exclusive_scan(int64_t* x, int n, int64_t* seg, int64_t* total) {
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int per = (n + kPlanThreads - 1) / kPlanThreads;
  const int i0 = min(n, tid * per), i1 = min(n, i0 + per);
  int64_t s = 0;
  for (int i = i0; i < i1; ++i) {
    const int64_t v = x[i];
    x[i] = s;
    s += v;
  }
  // inclusive scan of the segment totals within the wave
  int64_t inc = s;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int64_t y = __shfl_up(inc, d, 64);
    if (lane >= d) inc += y;
  }
  if (lane == 63) seg[wave] = inc;
  __syncthreads();
  if (wave == 0) {
    const int64_t w = lane < kPlanWaves ? seg[lane] : 0;
    int64_t wi = w;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const int64_t y = __shfl_up(wi, d, 64);
      if (lane >= d) wi += y;
    }
    if (lane < kPlanWaves) seg[lane] = wi - w;  // exclusive wave offsets
    if (lane == 63) *total = wi;
  }
  __syncthreads();
  const int64_t off = seg[wave] + inc - s;
  for (int i = i0; i < i1; ++i) x[i] += off;
  __syncthreads();
}

// Byte span of a row-major rows x cols matrix with leading dimension ld.
__device__ uint64_t span_end(const void* p, int64_t rows, int64_t cols, int64_t ld) {
  return (uint64_t)(uintptr_t)p + (uint64_t)((rows - 1) * ld + cols) * sizeof(float);
}
__device__ bool overlap(uint64_t alo, uint64_t ahi, uint64_t blo, uint64_t bhi) { return alo < bhi && blo < ahi; }

struct Spans {
  int64_t key;  // F N K of a valid problem, -1 otherwise (ranked last)
  uint64_t wlo, whi, hlo, hhi, vlo, vhi;
};

// The host checks of nmf_beta_step's arguments for one descriptor (sizes,
// leading dimensions, pointers, beta, the problem's own matrices disjoint),
// with K <= 64 as in every batch; an invalid descriptor gets key -1.
__device__ Spans spans_of(const nmf_problem& q) {
  Spans s{-1, 0, 0, 0, 0, 0, 0};
  const bool ok = q.V && q.W && q.H && q.F >= 1 && q.N >= 1 && q.K >= 1 && q.K <= 64 && q.F <= INT32_MAX &&
                  q.N <= INT32_MAX && q.ldv >= q.N && q.ldw >= q.K && q.ldh >= q.N && isfinite(q.beta);
  if (!ok) return s;
  s.wlo = (uintptr_t)q.W;
  s.whi = span_end(q.W, q.F, q.K, q.ldw);
  s.hlo = (uintptr_t)q.H;
  s.hhi = span_end(q.H, q.K, q.N, q.ldh);
  s.vlo = (uintptr_t)q.V;
  s.vhi = span_end(q.V, q.F, q.N, q.ldv);
  if (overlap(s.vlo, s.vhi, s.wlo, s.whi) || overlap(s.vlo, s.vhi, s.hlo, s.hhi) ||
      overlap(s.wlo, s.whi, s.hlo, s.hhi))
    return Spans{-1, 0, 0, 0, 0, 0, 0};
  s.key = q.F * q.N * q.K;
  return s;
}

__global__ __launch_bounds__(kPlanThreads) void batch_plan_kernel(BatchPlanArgs a) {
  __shared__ Spans stage[kStage];
  __shared__ int rpart[kPlanThreads];
  __shared__ int64_t seg[kPlanWaves];
  __shared__ int64_t tot_bytes, tot_items[4];
  __shared__ int bad;
  const int tid = threadIdx.x;
  int P = a.count;
  if (tid == 0) bad = 0;
  if (a.d_count) {
    const int n = *a.d_count;
    if (n < 0 || n > a.count) {
      if (tid == 0) bad = 1;
      P = 0;
    } else {
      P = n;
    }
  }
  __syncthreads();

  // each problem: workspace bytes and items per phase (zero if invalid)
  for (int i = tid; i < P; i += kPlanThreads) {
    const nmf_problem q = a.problems[i];
    const Spans sp = spans_of(q);
    int64_t bytes = 0, items[4] = {0, 0, 0, 0};
    if (sp.key < 0) {
      atomicOr(&bad, 1);
    } else {
      const Plan p = make_batch_plan(q.F, q.N, q.K, q.beta, a.tiles[bucket_of(q.F, q.N, q.K, q.beta)], a.joint != 0,
                                   a.opts.precision);
      bytes = (int64_t)align_up(p.total);
      int units[4], per_item[4], it[4];
      batch_phases(p, q.F, a.opts.precision, units, per_item, it);
      for (int ph = 0; ph < 4; ++ph) items[ph] = it[ph];
    }
    a.s_bytes[i] = bytes;
    for (int ph = 0; ph < 4; ++ph) a.s_items[4 * (int64_t)i + ph] = items[ph];
  }

  // rank by size (larger first, ties by index) and cross-problem overlaps, with
  // the other problems' spans staged through LDS kStage at a time.  With at
  // most kPlanThreads / 2 problems two threads share a problem, each checking
  // every other staged descriptor; their rank counts are added through LDS.
  const int split = P <= kPlanThreads / 2 ? 2 : 1;
  const int span = kPlanThreads / split;  // problems per round
  const int part = tid / span, lt = tid % span;
  for (int ib = 0; ib < P; ib += span) {
    const int i = ib + lt;
    const bool act = i < P;
    const Spans me = act ? spans_of(a.problems[i]) : Spans{-1, 0, 0, 0, 0, 0, 0};
    int r = 0;
    bool ov = false;
    for (int jb = 0; jb < P; jb += kStage) {
      __syncthreads();
      if (tid < kStage) {
        const int j = jb + tid;
        stage[tid] = j < P ? spans_of(a.problems[j]) : Spans{-2, 0, 0, 0, 0, 0, 0};
      }
      __syncthreads();
      const int nj = min(kStage, P - jb);
      if (act)
        for (int t = part; t < nj; t += split) {
          const Spans& o = stage[t];
          const int j2 = jb + t;
          r += (o.key > me.key) || (o.key == me.key && j2 < i);
          if (j2 != i)
            ov |= overlap(me.wlo, me.whi, o.wlo, o.whi) || overlap(me.wlo, me.whi, o.hlo, o.hhi) ||
                  overlap(me.hlo, me.hhi, o.hlo, o.hhi) || overlap(me.vlo, me.vhi, o.wlo, o.whi) ||
                  overlap(me.vlo, me.vhi, o.hlo, o.hhi);
        }
    }
    __syncthreads();
    rpart[tid] = r;
    __syncthreads();
    if (act && part == 0) {
      int rr = 0;
      for (int q = 0; q < split; ++q) rr += rpart[q * span + lt];
      a.s_order[rr] = i;
    }
    if (act && ov) atomicOr(&bad, 1);
  }
  __syncthreads();

  // workspace offsets, and item offsets phase by phase in rank order
  block_exclusive_scan(a.s_bytes, P, seg, &tot_bytes);
  for (int ph = 0; ph < 4; ++ph) {
    int64_t* off = a.s_off + (int64_t)ph * P;
    for (int r = tid; r < P; r += kPlanThreads) off[r] = a.s_items[4 * (int64_t)a.s_order[r] + ph];
    __syncthreads();
    block_exclusive_scan(off, P, seg, &tot_items[ph]);
  }
  const int64_t n_items = tot_items[0] + tot_items[1] + tot_items[2] + tot_items[3];
  const bool fits = !bad && tot_bytes <= a.work_bytes && n_items <= a.max_items;
  if (!fits) P = 0;

  // descriptors, queue entries, cleared counters
  int64_t phase_base[4];
  phase_base[0] = 0;
  for (int ph = 1; ph < 4; ++ph) phase_base[ph] = phase_base[ph - 1] + tot_items[ph - 1];
  for (int r = tid; r < P; r += kPlanThreads) {
    const int i = a.s_order[r];
    const nmf_problem q = a.problems[i];
    const Plan p = make_batch_plan(q.F, q.N, q.K, q.beta, a.tiles[bucket_of(q.F, q.N, q.K, q.beta)], a.joint != 0,
                                   a.opts.precision);
    const BatchProblem d = make_batch_problem(p, a.work + a.s_bytes[i], a.flags, q, a.joint != 0, a.opts);
    a.desc[i] = d;
    for (int ph = 0; ph < 4; ++ph) {
      int2* out = a.list + phase_base[ph] + a.s_off[(int64_t)ph * P + r];
      for (int it = 0; it < d.items[ph]; ++it) out[it] = make_int2(i, (ph << 24) | it);
      a.done[4 * (int64_t)i + ph] = 0u;
    }
  }
  if (tid == 0) {
    if (!fits) __hip_atomic_fetch_or(a.flags, 16u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // NMF_FLAG_SKIPPED
    *a.next = 0u;
    *a.exited = 0u;
    a.counts[0] = fits ? (int)n_items : 0;
    a.counts[1] = P;
  }
}

}  // namespace

hipError_t launch_batch_plan(hipStream_t s, const BatchPlanArgs& a) {
  hipLaunchKernelGGL(batch_plan_kernel, dim3(1), dim3(kPlanThreads), 0, s, a);
  return hipGetLastError();
}

}  // namespace nmf
