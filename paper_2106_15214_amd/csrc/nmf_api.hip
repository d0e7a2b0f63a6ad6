// Host side of the beta-NMF library: argument checks, context and workspace,
// launch planning and the C ABI declared in include/nmf_beta.h.
#include <hip/hip_runtime.h>

#include <unistd.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "nmf_batched_plan.h"
#include "nmf_beta.h"
#include "nmf_internal.h"
#include "nmf_plan.h"

using namespace nmf;

namespace {


struct TimedLaunch {
  hipEvent_t start, stop;
};

// Workspace of nmf_beta_step_noalloc: one fixed array per GPU, allocated with
// the code object when the library is loaded on a device and held until the
// process ends.  In host code `scratch` names a host-side stand-in, not device
// memory: its device address is looked up per device (hipGetSymbolAddress) at
// context creation and only that address is ever handed to kernels.
constexpr size_t kScratchBytes = size_t(NMF_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

}  // namespace

struct nmf_ctx_s {
  int device = 0;
  int num_cus = 256;
  char* ws = nullptr;  // workspace base
  size_t ws_bytes = 0;
  char* scratch = nullptr;  // this device's fixed scratch array (nmf_beta_step_noalloc)
  // A call was recorded into a stream capture: a graph may hold kernels that
  // point into the workspace, so it is never moved again (growth is refused).
  bool captured = false;
  int target_blocks = 0;  // 0: cost model
  int min_tiles = 1;
  int path = NMF_PATH_AUTO;
  int fused_grid[2][6][2][2] = {};  // cached cooperative capacity per instantiation (+1)
  uint32_t profile_mask = 0;
  std::vector<TimedLaunch> pending[NMF_KERNEL_COUNT];
  std::vector<hipEvent_t> event_pool;
  double prof_ms[NMF_KERNEL_COUNT] = {};
  int64_t prof_count[NMF_KERNEL_COUNT] = {};
  int batch_tiles[kBatchBuckets] = {};  // tiles per pass item of each batch bucket (set at creation)
  int batch_grid[2][2] = {};            // persistent batched grid per (precision, mode), 0 = not yet known
  // batched region of nmf_beta_step_batched (nmf_reserve_batched): header
  // (flags, queue position, exits, counts) | tile table | done counters |
  // descriptors | queue | planner scratch | problem workspaces
  char* bmem = nullptr;
  size_t bbytes = 0;
  int b_max_problems = 0;
  int64_t b_max_items = 0, b_work_bytes = 0;
  size_t bo_tiles = 0, bo_done = 0, bo_desc = 0, bo_list = 0, bo_sbytes = 0, bo_sitems = 0, bo_soff = 0,
         bo_sorder = 0, bo_work = 0;
  bool b_captured = false;  // a batched call was captured: the region never moves again
};

struct nmf_batch_s {
  int device = 0;
  int count = 0;
  int mode = NMF_JOINT;
  int prec = NMF_FP32;
  int grid = 0;
  int64_t total = 0;
  char* mem = nullptr;  // header | counters | descriptors | queue | problem workspaces
  size_t bytes = 0;
  BatchArgs args{};
};

namespace {

constexpr size_t kHaltOffset = 128;  // halt word of the device-side outer loop (nmf_beta_run)
constexpr int kFusedMaxPerCU = 8;      // bound on co-resident fused workgroups per CU (workspace sizing)
constexpr int kUpdateWBlocks = 4096;  // W-update workgroups at most (one unit of rows each, or more)



// Number of groups the contracted dimension (`tiles` 32-wide tiles) is split
// into, for `blocks` workgroups along the other dimension.  Minimizes a cost in
// tile-times: resident rounds x (tiles per group + 2 for prologue/epilogue)
// plus the partial-sum traffic (two arrays of groups * out_len * KP floats,
// written and read at ~24 MB per tile-time).
int choose_groups(const nmf_ctx_s* c, int64_t tiles, int64_t blocks, int64_t out_len, int KB, int64_t slots,
                  int* per_group) {
  const int64_t min_tpg = std::max(1, c->min_tiles);
  int64_t best_g = 1;
  const int64_t gcap = std::max<int64_t>(1, cdiv(4 * std::max<int64_t>(slots, 2 * (int64_t)c->num_cus), blocks));
  if (c->target_blocks > 0) {
    best_g = std::max<int64_t>(1, std::min<int64_t>(std::min(cdiv(tiles, min_tpg), gcap), cdiv(c->target_blocks, blocks)));
  } else {
    double best = 1e300;
    const int64_t gmax = std::min<int64_t>(cdiv(tiles, min_tpg), gcap);
    for (int64_t g = 1; g <= gmax; ++g) {
      const int64_t tpg = cdiv(tiles, g);
      if (g > 1 && cdiv(tiles, tpg) < g) continue;  // same split as a smaller g
      const double rounds = (double)cdiv(blocks * g, slots);
      const double partial = 4.0 * (double)g * out_len * 32 * KB * 4 / 24.0e6;
      const double cost = rounds * (tpg + 2.0) + partial;
      if (cost < best) { best = cost; best_g = g; }
    }
  }
  const int64_t tpg = cdiv(tiles, best_g);
  *per_group = (int)tpg;
  return (int)cdiv(tiles, tpg);
}



// Largest problem (F N entries) run as one fused launch: its P and Q tiles
// (8 bytes per entry) stay well inside the 256 MB last-level cache.
constexpr int64_t kFusedMaxEntries = int64_t(1) << 24;
// Largest problem (F N entries) whose joint streaming step keeps P and Q in the
// workspace between the passes (two float arrays of F N entries): the H pass
// then contracts them instead of forming Lambda~ and its powers a second time.
constexpr int64_t kPQMaxEntries = int64_t(1) << 28;
// Largest number of sub-iterations L accepted in one step.
constexpr int kMaxInnerIters = 1000;

int fused_capacity(nmf_ctx_s* c, int bc, int kb, bool joint, bool obj) {
  int& slot = c->fused_grid[kb - 1][bc][joint][obj];
  if (slot == 0) slot = 1 + std::min(fused_max_blocks(bc, kb, joint, obj, c->num_cus), kFusedMaxPerCU * c->num_cus);
  return slot - 1;
}


Plan make_plan(const nmf_ctx_s* c, int64_t F, int64_t N, int64_t K, int cols_occ = 2, int fused_grid = 0,
               bool pq = false, bool inner = false) {
  Plan p{};
  p.pq = pq && fused_grid == 0;
  p.KB = kblocks_for(K);
  p.KP = 32 * p.KB;
  p.fused = fused_grid > 0;
  p.fused_grid = fused_grid;
  const int64_t rows_slots = p.fused ? fused_grid : (int64_t)c->num_cus * sweep_rows_occupancy(p.KB);
  const int64_t cols_slots =
      p.fused ? fused_grid : (int64_t)c->num_cus * std::min(cols_occ, sweep_rows_occupancy(p.KB));
  p.row_blocks = (int)cdiv(F, kBlockRows);
  p.n_groups = choose_groups(c, cdiv(N, kTile), p.row_blocks, F, p.KB, rows_slots, &p.tiles_n);
  p.col_blocks = (int)cdiv(N, kBlockRows);
  p.f_groups = choose_groups(c, cdiv(F, kTile), p.col_blocks, N, p.KB, cols_slots, &p.tiles_f);
  p.uw_blocks = p.fused ? fused_grid : (int)std::min<int64_t>(kUpdateWBlocks, cdiv(F, update_w_unit_rows(p.KB)));
  p.uh_blocks = p.fused ? (int)cdiv(N, kTile) : (int)cdiv(N, kBlock / p.KP);
  return finish_plan(p, F, N, inner);
}


// Workspace size covering every call with F <= maxF, N <= maxN, K <= maxK under
// the current launch settings.  choose_groups keeps blocks * groups <= 4 * slots
// + blocks, so a partial array holds at most (4 * slots + blocks) * 128 rows
// (or columns), and never more than tiles * extent.
size_t plan_bound(const nmf_ctx_s* c, int64_t maxF, int64_t maxN, int64_t maxK) {
  const int64_t KP = 32 * kblocks_for(maxK);
  const int64_t slots = 2 * (int64_t)c->num_cus;
  const int64_t cap_blocks = 4 * slots;
  auto rows_bound = [&](int64_t extent, int64_t other) {
    const int64_t tiles = cdiv(other, kTile);
    const int64_t a = (cap_blocks + cdiv(extent, kBlockRows)) * kBlockRows;
    return std::min<int64_t>(a, tiles * extent);
  };
  Sizes z{};
  z.pobj = sizeof(double) * (size_t)(cap_blocks + cdiv(maxF, kBlockRows) + 4 * c->num_cus);
  z.pnum = sizeof(float) * (size_t)(rows_bound(maxF, maxN) * KP);
  z.prs = sizeof(float) * (size_t)((cap_blocks + 1) * KP);
  z.fk = sizeof(float) * (size_t)(maxF * KP);
  z.wt = sizeof(float) * (size_t)(KP * cdiv(maxF, 4) * 4);
  // fused: one row per workgroup; streaming: f_groups * col_parts <= 2 * row tiles + 1
  const int64_t pcol_rows = std::max<int64_t>(kFusedMaxPerCU * (int64_t)c->num_cus, 2 * cdiv(maxF, kTile) + 1);
  z.pcol = sizeof(double) * (size_t)(pcol_rows * 2 * KP);
  z.pnumh = sizeof(float) * (size_t)(rows_bound(maxN, maxF) * KP);
  const int64_t ft = cdiv(maxF, kTile), nt = cdiv(maxN, kTile);
  // P, Q tiles: every problem within the bounds that keeps them has F N <= kPQMaxEntries
  // (or the smaller single-launch limit), padded to whole 32 x 32 tiles
  const int64_t pq_cap = kPQMaxEntries + kTile * (maxF + maxN) + kTile * kTile;
  z.pq = sizeof(float) * (size_t)std::min<int64_t>(ft * nt * kTile * kTile, pq_cap);
  z.kn = sizeof(float) * (size_t)(KP * (cdiv(maxN, 4) * 4));  // chi(H) terms of joint sub-iterations
  return layout(z, Plan{}).total;
}

bool is_fin(double x) { return std::isfinite(x); }

bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  if (!a || !b || !na || !nb) return false;
  const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
  return a0 < b0 + nb && b0 < a0 + na;
}

size_t span_bytes(int64_t rows, int64_t cols, int64_t ld) {
  return (size_t)(((rows - 1) * ld + cols) * (int64_t)sizeof(float));
}

nmf_status check_mats(int64_t F, int64_t N, int64_t K, const float* V, int64_t ldv, const float* W, int64_t ldw,
                      const float* H, int64_t ldh) {
  if (!V || !W || !H) return NMF_ERR_NULL;
  if (F < 1 || N < 1 || K < 1) return NMF_ERR_SHAPE;
  if (F > INT32_MAX || N > INT32_MAX) return NMF_ERR_SHAPE;
  if (ldv < N || ldw < K || ldh < N) return NMF_ERR_SHAPE;
  if (K > 128) return NMF_ERR_UNSUPPORTED;
  const size_t sv = span_bytes(F, N, ldv), sw = span_bytes(F, K, ldw), sh = span_bytes(K, N, ldh);
  if (overlaps(V, sv, W, sw) || overlaps(V, sv, H, sh) || overlaps(W, sw, H, sh)) return NMF_ERR_ALIAS;
  return NMF_OK;
}

nmf_status check_opts(const nmf_step_opts* o) {
  if (!o) return NMF_OK;
  if (o->precision != NMF_FP32 && o->precision != NMF_BF16 && o->precision != NMF_FP16) return NMF_ERR_UNSUPPORTED;
  if (!is_fin(o->kappa) || o->kappa < 0.f) return NMF_ERR_BETA;
  if (o->inner_iters < 1 || o->inner_iters > kMaxInnerIters) return NMF_ERR_ARG;
  if (o->normalize != 0 && o->normalize != 1) return NMF_ERR_ARG;
  if (o->exponent != NMF_EXPONENT_MM && o->exponent != NMF_EXPONENT_ONE) return NMF_ERR_ARG;
  if (o->gram != 0 && o->gram != 1) return NMF_ERR_ARG;
  return NMF_OK;
}

nmf_status hip_status(hipError_t e) { return e == hipSuccess ? NMF_OK : NMF_ERR_HIP; }

// Ensures the workspace holds `bytes`; reallocates (blocking) unless the stream
// is being captured or a call was captured before (a graph may still point
// into the current workspace, so it must stay where it is).
nmf_status ensure_ws(nmf_ctx_s* c, hipStream_t s, size_t bytes) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return NMF_ERR_HIP;
  if (cs != hipStreamCaptureStatusNone) c->captured = true;
  if (c->ws_bytes >= bytes) return NMF_OK;
  if (cs != hipStreamCaptureStatusNone || c->captured) return NMF_ERR_WORKSPACE;
  if (hipSetDevice(c->device) != hipSuccess) return NMF_ERR_HIP;
  uint32_t flags_keep = 0;
  if (c->ws) {
    if (hipDeviceSynchronize() != hipSuccess) return NMF_ERR_HIP;
    (void)hipMemcpy(&flags_keep, c->ws, sizeof(uint32_t), hipMemcpyDeviceToHost);
    (void)hipFree(c->ws);
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  const size_t want = align_up(bytes + bytes / 8);
  void* p = nullptr;
  if (hipMalloc(&p, want) != hipSuccess) return NMF_ERR_HIP;
  if (hipMemset(p, 0, kHeaderBytes) != hipSuccess) { (void)hipFree(p); return NMF_ERR_HIP; }
  if (flags_keep && hipMemcpy(p, &flags_keep, sizeof(uint32_t), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(p);
    return NMF_ERR_HIP;
  }
  c->ws = (char*)p;
  c->ws_bytes = want;
  return NMF_OK;
}

unsigned* flags_ptr(nmf_ctx_s* c) { return (unsigned*)c->ws; }

// Device address of `scratch` on device `dev`, which must be current: looked up
// once per device and kept (each GPU holds its own copy at its own address).
nmf_status scratch_setup(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return NMF_ERR_NO_DEVICE;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return NMF_ERR_HIP;
    g_scratch[dev] = (char*)ptr;
  }
  *out = g_scratch[dev];
  return NMF_OK;
}

hipEvent_t get_event(nmf_ctx_s* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// Runs `launch` between two events when the kernel is selected for timing.
template <class Fn>
hipError_t timed(nmf_ctx_s* c, int kernel, hipStream_t s, Fn&& launch) {
  const bool on = (c->profile_mask >> kernel) & 1u;
  if (!on) return launch();
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  (void)hipStreamIsCapturing(s, &cs);
  if (cs != hipStreamCaptureStatusNone) return launch();
  TimedLaunch t{get_event(c), get_event(c)};
  (void)hipEventRecord(t.start, s);
  hipError_t e = launch();
  (void)hipEventRecord(t.stop, s);
  c->pending[kernel].push_back(t);
  return e;
}


// Byte ranges [lo, hi) of caller memory written (W, H) or read (V) by a batch.
struct Span {
  uintptr_t lo, hi;
  int prob;
};

nmf_status check_batch_alias(const nmf_problem* pr, int count) {
  std::vector<Span> wr, rd;
  for (int i = 0; i < count; ++i) {
    const nmf_problem& q = pr[i];
    wr.push_back({(uintptr_t)q.W, (uintptr_t)q.W + span_bytes(q.F, q.K, q.ldw), i});
    wr.push_back({(uintptr_t)q.H, (uintptr_t)q.H + span_bytes(q.K, q.N, q.ldh), i});
    rd.push_back({(uintptr_t)q.V, (uintptr_t)q.V + span_bytes(q.F, q.N, q.ldv), i});
  }
  std::sort(wr.begin(), wr.end(), [](const Span& a, const Span& b) { return a.lo < b.lo; });
  for (size_t i = 1; i < wr.size(); ++i)
    if (wr[i].lo < wr[i - 1].hi) return NMF_ERR_ALIAS;
  for (const Span& v : rd) {
    // first writable span ending after v.lo
    auto it = std::upper_bound(wr.begin(), wr.end(), v.lo, [](uintptr_t x, const Span& b) { return x < b.lo; });
    if (it != wr.begin() && std::prev(it)->hi > v.lo) return NMF_ERR_ALIAS;
    if (it != wr.end() && it->lo < v.hi) return NMF_ERR_ALIAS;
  }
  return NMF_OK;
}

// measured best on the 512-problem workload among 96..256 (160 and 256 tie):
// more problems take one group per pass and skip the update phases
constexpr int kBatchTilesDefault = 256;
constexpr unsigned kBatchSpinLimit = 1u << 22;

// Alternating MU with L > 1 sub-iterations (Algorithm 1, any product type): L W
// updates, each forming WH from the latest W (the first from the caller's W,
// the later ones from W_new in the workspace, which the update rewrites in
// place), then L H updates against the final W_new, each forming W_new H from
// the latest H.  Only the first W pass forms the objective of the entry
// iterate; only the last H update normalizes, writes W and the objective.
// Device-side outer loop (nmf_beta_run): every step kernel is gated by *halt,
// and after the W pass of iterate t (which forms its objective partials) a
// decide kernel writes trace[t] and applies the stopping rule.
struct RunCtl {
  unsigned* halt;
  double* trace;
  int t;
  double eps;
  int32_t* stop;
};

hipError_t run_decide_after_w(const RunCtl* run, hipStream_t s, const StepArgs& sa) {
  if (!run) return hipSuccess;
  return launch_run_decide(s, sa.ra.pobj, sa.sw_grid, run->trace, run->t, run->eps, run->halt, run->stop,
                           sa.ra.flags);
}

// Launches fn, between two timing events when the kernel is selected for
// profiling and the call may use them (`quiet`: never, no event is created).
template <class Fn>
hipError_t run_k(nmf_ctx_s* c, bool quiet, int kernel, hipStream_t s, Fn&& fn) {
  return quiet ? fn() : timed(c, kernel, s, fn);
}

nmf_status inner_steps(nmf_ctx_s* c, hipStream_t s, const Plan& p, const StepArgs& sa, int bc, bool want_obj,
                              int L, int prec, bool quiet, const RunCtl* run) {
  for (int l = 0; l < L; ++l) {
    SweepRowsArgs ra = sa.ra;
    UpdateWArgs ua = sa.ua;
    if (l > 0) {
      ra.W = sa.ua.Wn; ra.ldw = p.KP;
      ua.W = sa.ua.Wn; ua.ldw = p.KP;
    }
    hipError_t e = run_k(c, quiet, NMF_KERNEL_SWEEP_W, s, [&] {
      const bool obj = want_obj && l == 0;
      return prec == NMF_FP32 ? launch_sweep_rows(bc, p.KB, KIND_UPDATE, obj, false, sa.sw_grid, s, ra)
                              : launch_sweep_rows_lp(prec, bc, p.KB, obj, false, sa.sw_grid, s, ra);
    });
    if (e == hipSuccess && l == 0) e = run_decide_after_w(run, s, sa);
    if (e != hipSuccess) return NMF_ERR_HIP;
    e = run_k(c, quiet, NMF_KERNEL_UPDATE_W, s, [&] { return launch_update_w(p.KB, p.uw_blocks, s, ua); });
    if (e != hipSuccess) return NMF_ERR_HIP;
  }
  for (int l = 0; l < L; ++l) {
    UpdateHArgs ha = sa.ha;
    if (l + 1 < L) {
      ha.normalize = 0;
      ha.d_obj = nullptr;
    }
    hipError_t e = run_k(c, quiet, NMF_KERNEL_SWEEP_H, s, [&] {
      return prec == NMF_FP32 ? launch_sweep_cols(bc, p.KB, KIND_UPDATE, false, false, sa.sh_grid, s, sa.ca)
                              : launch_sweep_cols_lp(prec, bc, p.KB, false, false, sa.sh_grid, s, sa.ca);
    });
    if (e != hipSuccess) return NMF_ERR_HIP;
    e = run_k(c, quiet, NMF_KERNEL_UPDATE_H, s, [&] { return launch_update_h(p.KB, p.uh_blocks, s, ha); });
    if (e != hipSuccess) return NMF_ERR_HIP;
  }
  return NMF_OK;
}

// Joint MM with L > 1 sub-iterations (Algorithm 2, float32 products, P and Q
// kept between the passes).  Sub-iteration l updates W from W~ with the
// contractions P chi_1(H_l, H~)^T, Q chi_2(H_l, H~)^T -- the first W pass forms
// V~, P, Q and contracts them with H_1 = H~; later ones contract the kept tiles
// with the chi(H) terms -- then H from H~ with chi(W_{l+1}, W~).  The H updates
// before the last write chi_1(H_{l+1}, H~), chi_2(H_{l+1}, H~) to the workspace
// instead of H; the last writes H, normalizes, writes W and the objective.
nmf_status inner_steps_joint(nmf_ctx_s* c, hipStream_t s, const Plan& p, const StepArgs& sa, int bc, bool want_obj,
                             int L, char* ws, bool quiet, const RunCtl* run) {
  float* const C1h = (float*)(ws + p.o_c1h);
  float* const C2h = (float*)(ws + p.o_c2h);
  for (int l = 0; l < L; ++l) {
    hipError_t e;
    if (l == 0) {
      e = run_k(c, quiet, NMF_KERNEL_SWEEP_W, s, [&] {
        return launch_sweep_rows(bc, p.KB, KIND_UPDATE, want_obj, true, sa.sw_grid, s, sa.ra);
      });
      if (e == hipSuccess) e = run_decide_after_w(run, s, sa);
    } else {
      SweepRowsArgs rq = sa.ra;
      rq.H = C1h; rq.ldh = p.ldc;
      rq.W = C2h; rq.ldw = p.ldc;
      e = run_k(c, quiet, NMF_KERNEL_SWEEP_W, s, [&] { return launch_sweep_rows_pq(bc, p.KB, sa.sw_grid, s, rq); });
    }
    if (e != hipSuccess) return NMF_ERR_HIP;
    e = run_k(c, quiet, NMF_KERNEL_UPDATE_W, s, [&] { return launch_update_w(p.KB, p.uw_blocks, s, sa.ua); });
    if (e != hipSuccess) return NMF_ERR_HIP;
    e = run_k(c, quiet, NMF_KERNEL_SWEEP_H, s, [&] {
      return launch_sweep_cols(bc, p.KB, KIND_UPDATE, true, true, sa.sh_grid, s, sa.ca);
    });
    if (e != hipSuccess) return NMF_ERR_HIP;
    UpdateHArgs ha = sa.ha;
    if (l + 1 < L) {
      ha.C1h = C1h; ha.C2h = C2h; ha.ldc = p.ldc;
      ha.W = nullptr; ha.d_obj = nullptr; ha.normalize = 0;
    }
    e = run_k(c, quiet, NMF_KERNEL_UPDATE_H, s, [&] { return launch_update_h(p.KB, p.uh_blocks, s, ha); });
    if (e != hipSuccess) return NMF_ERR_HIP;
  }
  return NMF_OK;
}

// One outer iteration (nmf_beta_step).  no_alloc: the workspace is this
// device's fixed scratch array (never grown), `flags` the status word, the
// single-launch path and the kernel timing events are not used, and the joint
// step keeps P, Q between its passes only when they fit in the scratch.
nmf_status step_impl(nmf_ctx_t c, void* stream, int64_t F, int64_t N, int64_t K, const float* V, int64_t ldv,
                     float* W, int64_t ldw, float* H, int64_t ldh, double beta, int32_t mode,
                     const nmf_step_opts* opts, double* d_objective, bool no_alloc, unsigned* flags,
                     const RunCtl* run = nullptr) {
  if (!c) return NMF_ERR_NULL;
  nmf_status st = nmf_check_step_args(F, N, K, V, ldv, W, ldw, H, ldh, beta, mode, opts);
  if (st != NMF_OK) return st;
  nmf_step_opts o;
  nmf_default_opts(&o);
  if (opts) o = *opts;
  hipStream_t s = (hipStream_t)stream;
  const bool gram = o.gram != 0;
  const int bc = gram ? BC_B2G : beta_class(beta);
  const bool joint = (mode == NMF_JOINT);
  const bool want_obj = d_objective != nullptr || run != nullptr;
  const int prec = opts ? opts->precision : NMF_FP32;
  if (hipSetDevice(c->device) != hipSuccess) return NMF_ERR_HIP;
  // path: one cooperative launch for problems whose P, Q tiles stay cache
  // resident (not under stream capture), else four streaming launches
  const int L = o.inner_iters;
  int fused_grid = 0;
  if (!no_alloc && !run && !gram && c->path == NMF_PATH_FUSED && L == 1 && prec == NMF_FP32 && kblocks_for(K) <= 2 &&
      F * N <= kFusedMaxEntries) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cs) != hipSuccess) return NMF_ERR_HIP;
    if (cs == hipStreamCaptureStatusNone) fused_grid = fused_capacity(c, bc, kblocks_for(K), joint, want_obj);
  }
  if (!no_alloc && !run && !gram && c->path == NMF_PATH_FUSED && fused_grid <= 0) return NMF_ERR_UNSUPPORTED;
  // the Gram form at beta = 2 keeps nothing between the passes (P = V)
  bool use_pq = joint && !gram && fused_grid == 0 && F * N <= kPQMaxEntries;
  const bool dual = joint && !gram;
  const int cols_occ = sweep_cols_occupancy(bc, kblocks_for(K), KIND_UPDATE, dual);
  Plan p = make_plan(c, F, N, K, cols_occ, fused_grid, use_pq, joint && L > 1);
  // Gram region after the plan: G(H~) and G2 ([KP][KP] float64 each) and the
  // Gram kernels' block partials
  const size_t gram_bytes = gram ? sizeof(double) * (size_t)(2 + gram_parts()) * p.KP * p.KP : 0;
  char* ws = nullptr;
  if (no_alloc) {
    if (p.total + gram_bytes > kScratchBytes && use_pq && L == 1) {
      use_pq = false;  // the H pass forms Lambda~ again instead of reading kept P, Q
      p = make_plan(c, F, N, K, cols_occ, 0, false, false);
    }
    if (align_up(p.total) + gram_bytes > kScratchBytes) return NMF_ERR_WORKSPACE;
    if (!c->scratch) return NMF_ERR_HIP;
    ws = c->scratch;
  } else {
    if ((st = ensure_ws(c, s, align_up(p.total) + gram_bytes)) != NMF_OK) return st;
    ws = c->ws;
    flags = flags_ptr(c);
  }
  double* const G1 = gram ? (double*)(ws + align_up(p.total)) : nullptr;
  double* const G2 = G1 ? G1 + (size_t)p.KP * p.KP : nullptr;
  double* const Gpart = G2 ? G2 + (size_t)p.KP * p.KP : nullptr;
  const bool quiet = no_alloc;

  StepArgs sa = make_step_args(p, ws, flags, F, N, K, V, ldv, W, ldw, H, ldh, beta, joint, prec, o, d_objective);
  SweepRowsArgs& ra = sa.ra;
  UpdateWArgs& ua = sa.ua;
  SweepColsArgs& ca = sa.ca;
  UpdateHArgs& ha = sa.ha;
  if (run) {
    ra.halt = ua.halt = ca.halt = ha.halt = run->halt;
    ha.d_obj = nullptr;  // the decide kernel writes the trace
  }
  if (gram) {
    ua.gram = G1;
    ha.gram = G2;
  }
  const int sw_grid = sa.sw_grid, sh_grid = sa.sh_grid;

  if (p.fused) {
    // joint: the H pass contracts the P, Q tiles stored by the W pass
    ra.NT = (int)cdiv(N, kTile);
    ra.Pst = (float*)(ws + p.o_pst);
    ra.Qst = (float*)(ws + p.o_qst);
    ca.NT = ra.NT; ca.Pst = ra.Pst; ca.Qst = ra.Qst;
    ha.nobj = p.fused_grid;
    FusedArgs fa{};
    fa.r = ra; fa.uw = ua; fa.c = ca; fa.uh = ha;
    fa.n_items_w = sw_grid;
    fa.n_items_h = sh_grid;
    fa.slabs = (int)cdiv(F, kTile);
    fa.ntiles = (int)cdiv(N, kTile);
    fa.bar = (unsigned*)(ws + 8);
    fa.colsum = (float*)(ws + p.o_colsum);
    fa.spin_limit = 1u << 22;
    fa.stamps = ((c->profile_mask >> NMF_KERNEL_FUSED_STEP) & 1u) ? (unsigned long long*)(ws + 64) : nullptr;
    return hip_status(timed(c, NMF_KERNEL_FUSED_STEP, s, [&] {
      return launch_fused(bc, p.KB, joint, want_obj, p.fused_grid, s, fa);
    }));
  }
  if (p.pq) {
    ra.NT = (int)cdiv(N, kTile);
    ra.Pst = (float*)(ws + p.o_pst);
    ra.Qst = (float*)(ws + p.o_qst);
    ca.NT = ra.NT; ca.Pst = ra.Pst; ca.Qst = ra.Qst;
  }
  if (L > 1)
    return joint ? inner_steps_joint(c, s, p, sa, bc, want_obj, L, ws, quiet, run)
                 : inner_steps(c, s, p, sa, bc, want_obj, L, prec, quiet, run);
  if (gram) {  // H~ H~^T for the W-step denominators
    if (launch_gram(true, s, H, ldh, H, ldh, (int)K, p.KP, N, Gpart, G1) != hipSuccess)
      return NMF_ERR_HIP;
  }
  hipError_t e = run_k(c, quiet, NMF_KERNEL_SWEEP_W, s, [&] {
    return prec == NMF_FP32 ? launch_sweep_rows(bc, p.KB, KIND_UPDATE, want_obj, p.pq, sw_grid, s, ra)
                            : launch_sweep_rows_lp(prec, bc, p.KB, want_obj, p.pq, sw_grid, s, ra);
  });
  if (e == hipSuccess) e = run_decide_after_w(run, s, sa);
  if (e != hipSuccess) return NMF_ERR_HIP;
  e = run_k(c, quiet, NMF_KERNEL_UPDATE_W, s, [&] { return launch_update_w(p.KB, p.uw_blocks, s, ua); });
  if (e != hipSuccess) return NMF_ERR_HIP;
  if (gram) {  // G2 = chi_2^T W~ (joint) or W_new^T W_new (alternating) for the H-step denominators
    e = joint ? launch_gram(false, s, ua.C2, p.KP, W, ldw, (int)K, p.KP, F, Gpart, G2)
              : launch_gram(false, s, ua.Wn, p.KP, ua.Wn, p.KP, (int)K, p.KP, F, Gpart, G2);
    if (e != hipSuccess) return NMF_ERR_HIP;
  }
  e = run_k(c, quiet, NMF_KERNEL_SWEEP_H, s, [&] {
    return prec == NMF_FP32 ? launch_sweep_cols(bc, p.KB, KIND_UPDATE, dual, p.pq, sh_grid, s, ca)
                            : launch_sweep_cols_lp(prec, bc, p.KB, joint, p.pq, sh_grid, s, ca);
  });
  if (e != hipSuccess) return NMF_ERR_HIP;
  e = run_k(c, quiet, NMF_KERNEL_UPDATE_H, s, [&] { return launch_update_h(p.KB, p.uh_blocks, s, ha); });
  return hip_status(e);
}


// ---------------------------------------------------------------------------
// beta = 1 with a sparse V (kernels in nmf_sparse.hip)
// ---------------------------------------------------------------------------
nmf_status check_sparse(const nmf_sparse_v* V, int64_t K) {
  if (!V || !V->row_ptr || !V->col_ptr) return NMF_ERR_NULL;
  if (V->nnz > 0 && (!V->col_idx || !V->row_val || !V->row_idx || !V->col_val)) return NMF_ERR_NULL;
  if (V->F < 1 || V->N < 1 || V->nnz < 0 || K < 1) return NMF_ERR_SHAPE;
  if (V->F > INT32_MAX || V->N > INT32_MAX || V->nnz > V->F * V->N) return NMF_ERR_SHAPE;
  if (K > 64) return NMF_ERR_UNSUPPORTED;
  return NMF_OK;
}

// Workspace offsets of the sparse step (after the header).
struct SparsePlan {
  size_t ht, wc, wn, numw, numh, prow, pcw, pobj, pcol, total;
  int hb, wcb, rb, cb, K4;
};

SparsePlan sparse_plan(int64_t F, int64_t N, int64_t K) {
  SparsePlan p{};
  p.K4 = (int)((K + 3) & ~int64_t(3));
  sparse_blocks((int)F, (int)N, &p.hb, &p.wcb, &p.rb, &p.cb);
  size_t o = kHeaderBytes;
  auto take = [&](size_t bytes) { size_t r = o; o = align_up(o + bytes); return r; };
  p.ht = take(sizeof(float) * (size_t)N * p.K4);
  p.wc = take(sizeof(float) * (size_t)F * p.K4);
  p.wn = take(sizeof(float) * (size_t)F * p.K4);
  p.numw = take(sizeof(float) * (size_t)F * p.K4);
  p.numh = take(sizeof(float) * (size_t)N * p.K4);
  p.prow = take(sizeof(double) * (size_t)p.hb * p.K4);
  p.pcw = take(sizeof(double) * (size_t)p.wcb * p.K4);
  p.pobj = take(sizeof(double) * (size_t)p.rb);
  p.pcol = take(sizeof(double) * (size_t)p.wcb * 2 * p.K4);
  p.total = o;
  return p;
}

SparseArgs sparse_args(const SparsePlan& p, char* ws, unsigned* flags, const nmf_sparse_v* V, int64_t K,
                       float* W, int64_t ldw, float* H, int64_t ldh) {
  SparseArgs a{};
  a.F = (int)V->F; a.N = (int)V->N; a.K = (int)K; a.nnz = V->nnz;
  a.row_ptr = V->row_ptr; a.col_idx = V->col_idx; a.row_val = V->row_val;
  a.col_ptr = V->col_ptr; a.row_idx = V->row_idx; a.col_val = V->col_val;
  a.Wio = W; a.ldw = ldw; a.Hio = H; a.ldh = ldh;
  a.HT = (float*)(ws + p.ht); a.Wc = (float*)(ws + p.wc); a.Wn = (float*)(ws + p.wn);
  a.numW = (float*)(ws + p.numw); a.numH = (float*)(ws + p.numh);
  a.prow = (double*)(ws + p.prow); a.pcw = (double*)(ws + p.pcw);
  a.pobj = (double*)(ws + p.pobj); a.pcol = (double*)(ws + p.pcol);
  a.flags = flags;
  return a;
}

// The two gradient passes of nmf_beta_grad / nmf_beta_kkt: E = Lambda^(beta-2)
// (Lambda - V) contracted with H^T (row pass) and W^T (column pass), as partial
// sums in the workspace of plan p (and the objective partials with want_obj).
struct GradParts {
  hipError_t e;
  const float* pnumw;
  const float* pnumh;
  double* pobj;
  int sw_grid;
};

GradParts grad_passes(nmf_ctx_s* c, hipStream_t s, const Plan& p, int64_t F, int64_t N, int64_t K, const float* V,
                      int64_t ldv, const float* W, int64_t ldw, const float* H, int64_t ldh, double beta,
                      float kappa, bool want_obj) {
  const int bc = beta_class(beta);
  char* ws = c->ws;
  SweepRowsArgs ra{};
  ra.V = V; ra.ldv = ldv; ra.W = W; ra.ldw = ldw; ra.H = H; ra.ldh = ldh;
  ra.F = (int)F; ra.N = (int)N; ra.K = (int)K;
  ra.bm2 = (float)(beta - 2.0); ra.kappa = kappa; ra.beta = beta;
  ra.n_groups = p.n_groups; ra.tiles_per_group = p.tiles_n;
  ra.pnum = (float*)(ws + p.o_pnum); ra.pobj = (double*)(ws + p.o_pobj);
  ra.vec4 = ((uintptr_t)V % 16 == 0) && (ldv % 4 == 0);
  ra.hvec = ((uintptr_t)H % 16 == 0) && (ldh % 4 == 0);
  ra.vstream = 0;
  GradParts g{hipSuccess, ra.pnum, (float*)(ws + p.o_pnumh), ra.pobj, p.row_blocks * p.n_groups};
  g.e = launch_sweep_rows(bc, p.KB, KIND_GRAD, want_obj, false, g.sw_grid, s, ra);
  if (g.e != hipSuccess) return g;
  float* WT = (float*)(ws + p.o_wt);
  float* Wp = (float*)(ws + p.o_wn);
  if ((g.e = launch_transpose(s, W, ldw, (int)F, (int)K, p.KP, WT, p.ldt, Wp)) != hipSuccess) return g;
  SweepColsArgs ca{};
  ca.V = V; ca.ldv = ldv; ca.WT = WT; ca.ldwt = p.ldt; ca.C1 = Wp; ca.C2 = Wp;
  ca.H = H; ca.ldh = ldh; ca.F = (int)F; ca.N = (int)N; ca.K = (int)K;
  ca.bm2 = (float)(beta - 2.0); ca.kappa = kappa;
  ca.f_groups = p.f_groups; ca.tiles_per_group = p.tiles_f;
  ca.pnum = (float*)(ws + p.o_pnumh);
  g.e = launch_sweep_cols(bc, p.KB, KIND_GRAD, false, false, p.col_blocks * p.f_groups, s, ca);
  return g;
}

}  // namespace

extern "C" {

void nmf_default_opts(nmf_step_opts* o) {
  if (!o) return;
  o->precision = NMF_FP32;
  o->kappa = 0.f;
  o->inner_iters = 1;
  o->normalize = 1;
  o->exponent = NMF_EXPONENT_MM;
  o->gram = 0;
}

const char* nmf_version(void) { return "nmfbeta 0.2 (gfx950)"; }

const char* nmf_status_string(nmf_status s) {
  // a C caller may pass any int: read it as one (an out-of-range enumerator
  // value must not be loaded as the enum type)
  int v = 0;
  std::memcpy(&v, &s, sizeof(v));
  switch (v) {
    case NMF_OK: return "NMF_OK";
    case NMF_ERR_NULL: return "NMF_ERR_NULL: required pointer is NULL";
    case NMF_ERR_SHAPE: return "NMF_ERR_SHAPE: bad size or leading dimension";
    case NMF_ERR_BETA: return "NMF_ERR_BETA: beta or kappa not finite (or kappa < 0)";
    case NMF_ERR_ALIAS: return "NMF_ERR_ALIAS: matrices overlap";
    case NMF_ERR_WORKSPACE: return "NMF_ERR_WORKSPACE: workspace (or batched region) too small, missing, or fixed by a capture";
    case NMF_ERR_HIP: return "NMF_ERR_HIP: HIP runtime error";
    case NMF_ERR_UNSUPPORTED: return "NMF_ERR_UNSUPPORTED: unsupported size or option";
    case NMF_ERR_ARG: return "NMF_ERR_ARG: invalid argument";
    case NMF_ERR_NO_DEVICE: return "NMF_ERR_NO_DEVICE: no usable GPU";
    case NMF_ERR_IO: return "NMF_ERR_IO: the tuning cache file could not be written";
  }
  return "unknown nmf_status";
}

nmf_status nmf_create(nmf_ctx_t* out, int device) {
  if (!out) return NMF_ERR_NULL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return NMF_ERR_NO_DEVICE;
  if (device < 0 || device >= n) return NMF_ERR_NO_DEVICE;
  nmf_ctx_s* c = new (std::nothrow) nmf_ctx_s();
  if (!c) return NMF_ERR_HIP;
  c->device = device;
  for (int b = 0; b < kBatchBuckets; ++b) c->batch_tiles[b] = kBatchTilesDefault;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
    c->num_cus = prop.multiProcessorCount;
  // set-up of the no-allocation step: this device's scratch address, looked up
  // with the device current (the caller's current device is restored)
  int prev = -1;
  (void)hipGetDevice(&prev);
  nmf_status st = hipSetDevice(device) == hipSuccess ? scratch_setup(device, &c->scratch) : NMF_ERR_HIP;
  if (prev >= 0 && prev != device) (void)hipSetDevice(prev);
  if (st != NMF_OK) {
    delete c;
    return st;
  }
  *out = c;
  return NMF_OK;
}

nmf_status nmf_destroy(nmf_ctx_t c) {
  if (!c) return NMF_ERR_NULL;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (auto& v : c->pending)
    for (auto& t : v) { (void)hipEventDestroy(t.start); (void)hipEventDestroy(t.stop); }
  for (auto e : c->event_pool) (void)hipEventDestroy(e);
  if (c->ws) (void)hipFree(c->ws);
  if (c->bmem) (void)hipFree(c->bmem);
  delete c;
  return NMF_OK;
}

nmf_status nmf_reserve(nmf_ctx_t c, int64_t maxF, int64_t maxN, int64_t maxK) {
  if (!c) return NMF_ERR_NULL;
  if (maxF < 1 || maxN < 1 || maxK < 1) return NMF_ERR_SHAPE;
  if (maxK > 128) return NMF_ERR_UNSUPPORTED;
  const size_t need = plan_bound(c, maxF, maxN, maxK);
  return ensure_ws(c, nullptr, need);
}

nmf_status nmf_check_step_args(int64_t F, int64_t N, int64_t K, const float* V, int64_t ldv, const float* W,
                               int64_t ldw, const float* H, int64_t ldh, double beta, int32_t mode,
                               const nmf_step_opts* opts) {
  nmf_status st = check_mats(F, N, K, V, ldv, W, ldw, H, ldh);
  if (st != NMF_OK) return st;
  if (!is_fin(beta)) return NMF_ERR_BETA;
  if (mode != NMF_ALTERNATING && mode != NMF_JOINT) return NMF_ERR_ARG;
  st = check_opts(opts);
  if (st != NMF_OK) return st;
  if (opts && opts->precision != NMF_FP32 && K > 64) return NMF_ERR_UNSUPPORTED;
  // Gram-form denominators: beta = 2, kappa = 0, float32, one sub-iteration, K <= 64
  if (opts && opts->gram &&
      (beta != 2.0 || opts->kappa != 0.f || opts->precision != NMF_FP32 || opts->inner_iters != 1 || K > 64))
    return NMF_ERR_UNSUPPORTED;
  // L > 1 sub-iterations of joint MM: float32 products, P and Q kept between the passes
  if (opts && opts->inner_iters > 1 && mode == NMF_JOINT &&
      (opts->precision != NMF_FP32 || F * N > kPQMaxEntries))
    return NMF_ERR_UNSUPPORTED;
  return NMF_OK;
}

nmf_status nmf_beta_step(nmf_ctx_t c, void* stream, int64_t F, int64_t N, int64_t K, const float* V, int64_t ldv,
                         float* W, int64_t ldw, float* H, int64_t ldh, double beta, int32_t mode,
                         const nmf_step_opts* opts, double* d_objective) {
  return step_impl(c, stream, F, N, K, V, ldv, W, ldw, H, ldh, beta, mode, opts, d_objective, false, nullptr);
}

nmf_status nmf_beta_step_noalloc(nmf_ctx_t c, void* stream, int64_t F, int64_t N, int64_t K, const float* V,
                                 int64_t ldv, float* W, int64_t ldw, float* H, int64_t ldh, double beta,
                                 int32_t mode, const nmf_step_opts* opts, double* d_objective, uint32_t* d_flags) {
  if (!c) return NMF_ERR_NULL;
  // without d_flags the status word is the scratch's first word (written, never read)
  unsigned* flags = d_flags ? (unsigned*)d_flags : (unsigned*)c->scratch;
  return step_impl(c, stream, F, N, K, V, ldv, W, ldw, H, ldh, beta, mode, opts, d_objective, true, flags);
}

nmf_status nmf_beta_objective(nmf_ctx_t c, void* stream, int64_t F, int64_t N, int64_t K, const float* V,
                              int64_t ldv, const float* W, int64_t ldw, const float* H, int64_t ldh, double beta,
                              float kappa, double* d_out) {
  if (!c || !d_out) return NMF_ERR_NULL;
  nmf_status st = check_mats(F, N, K, V, ldv, W, ldw, H, ldh);
  if (st != NMF_OK) return st;
  if (!is_fin(beta) || !std::isfinite(kappa) || kappa < 0.f) return NMF_ERR_BETA;
  hipStream_t s = (hipStream_t)stream;
  const Plan p = make_plan(c, F, N, K);
  if ((st = ensure_ws(c, s, p.total)) != NMF_OK) return st;
  if (hipSetDevice(c->device) != hipSuccess) return NMF_ERR_HIP;
  SweepRowsArgs ra{};
  ra.V = V; ra.ldv = ldv; ra.W = W; ra.ldw = ldw; ra.H = H; ra.ldh = ldh;
  ra.F = (int)F; ra.N = (int)N; ra.K = (int)K;
  ra.bm2 = (float)(beta - 2.0); ra.kappa = kappa; ra.beta = beta;
  ra.n_groups = p.n_groups; ra.tiles_per_group = p.tiles_n;
  ra.pobj = (double*)(c->ws + p.o_pobj);
  ra.vec4 = ((uintptr_t)V % 16 == 0) && (ldv % 4 == 0);
  ra.hvec = ((uintptr_t)H % 16 == 0) && (ldh % 4 == 0);
  ra.vstream = 0;
  const int grid = p.row_blocks * p.n_groups;
  hipError_t e = launch_sweep_rows(beta_class(beta), p.KB, KIND_OBJ, true, false, grid, s, ra);
  if (e != hipSuccess) return NMF_ERR_HIP;
  return hip_status(launch_finalize_objective(s, ra.pobj, grid, d_out, flags_ptr(c)));
}

nmf_status nmf_beta_grad(nmf_ctx_t c, void* stream, int64_t F, int64_t N, int64_t K, const float* V, int64_t ldv,
                         const float* W, int64_t ldw, const float* H, int64_t ldh, double beta, float kappa,
                         double scale, const double* d_scale, float* dW, int64_t lddw, float* dH, int64_t lddh,
                         double* d_objective) {
  if (!c || !dW || !dH) return NMF_ERR_NULL;
  nmf_status st = check_mats(F, N, K, V, ldv, W, ldw, H, ldh);
  if (st != NMF_OK) return st;
  if (lddw < K || lddh < N) return NMF_ERR_SHAPE;
  if (!is_fin(beta) || !is_fin(scale) || !std::isfinite(kappa) || kappa < 0.f) return NMF_ERR_BETA;
  {
    const size_t sv = span_bytes(F, N, ldv), sw = span_bytes(F, K, ldw), sh = span_bytes(K, N, ldh);
    const size_t sdw = span_bytes(F, K, lddw), sdh = span_bytes(K, N, lddh);
    const void* in[3] = {V, W, H};
    const size_t ns[3] = {sv, sw, sh};
    for (int i = 0; i < 3; ++i)
      if (overlaps(in[i], ns[i], dW, sdw) || overlaps(in[i], ns[i], dH, sdh)) return NMF_ERR_ALIAS;
    if (overlaps(dW, sdw, dH, sdh)) return NMF_ERR_ALIAS;
  }
  hipStream_t s = (hipStream_t)stream;
  const Plan p = make_plan(c, F, N, K);
  if ((st = ensure_ws(c, s, p.total)) != NMF_OK) return st;
  if (hipSetDevice(c->device) != hipSuccess) return NMF_ERR_HIP;
  GradParts g = grad_passes(c, s, p, F, N, K, V, ldv, W, ldw, H, ldh, beta, kappa, d_objective != nullptr);
  if (g.e != hipSuccess) return NMF_ERR_HIP;
  hipError_t e;
  const int gw = (int)std::min<int64_t>(1024, std::max<int64_t>(1, cdiv(F * K, kBlock)));
  if ((e = launch_grad_w(p.KB, gw, s, g.pnumw, (int)F, (int)K, p.n_groups, scale, d_scale, dW, lddw)) != hipSuccess)
    return NMF_ERR_HIP;
  if ((e = launch_grad_h(p.KB, (int)cdiv(N, kTile), s, g.pnumh, (int)N, (int)K, p.f_groups, scale, d_scale, dH,
                         lddh)) != hipSuccess)
    return NMF_ERR_HIP;
  if (d_objective) return hip_status(launch_finalize_objective(s, g.pobj, g.sw_grid, d_objective, flags_ptr(c)));
  return NMF_OK;
}

nmf_status nmf_beta_kkt(nmf_ctx_t c, void* stream, int64_t F, int64_t N, int64_t K, const float* V, int64_t ldv,
                        const float* W, int64_t ldw, const float* H, int64_t ldh, double beta, float kappa,
                        double* d_res) {
  if (!c || !d_res) return NMF_ERR_NULL;
  nmf_status st = check_mats(F, N, K, V, ldv, W, ldw, H, ldh);
  if (st != NMF_OK) return st;
  if (!is_fin(beta) || !std::isfinite(kappa) || kappa < 0.f) return NMF_ERR_BETA;
  hipStream_t s = (hipStream_t)stream;
  const Plan p = make_plan(c, F, N, K);
  const size_t part_off = align_up(p.total);
  if ((st = ensure_ws(c, s, part_off + sizeof(double) * (size_t)kkt_parts())) != NMF_OK) return st;
  if (hipSetDevice(c->device) != hipSuccess) return NMF_ERR_HIP;
  GradParts g = grad_passes(c, s, p, F, N, K, V, ldv, W, ldw, H, ldh, beta, kappa, false);
  if (g.e != hipSuccess) return NMF_ERR_HIP;
  return hip_status(launch_kkt(p.KB, s, g.pnumw, p.n_groups, g.pnumh, p.f_groups, W, ldw, H, ldh, (int)F, (int)N,
                               (int)K, (double*)(c->ws + part_off), d_res));
}

nmf_status nmf_beta_run(nmf_ctx_t c, void* stream, int64_t F, int64_t N, int64_t K, const float* V, int64_t ldv,
                        float* W, int64_t ldw, float* H, int64_t ldh, double beta, int32_t mode,
                        const nmf_step_opts* opts, int32_t max_iters, double eps, double* d_trace, int32_t* d_stop) {
  if (!c || !d_trace || !d_stop) return NMF_ERR_NULL;
  if (max_iters < 0 || !std::isfinite(eps)) return NMF_ERR_ARG;
  nmf_status st = nmf_check_step_args(F, N, K, V, ldv, W, ldw, H, ldh, beta, mode, opts);
  if (st != NMF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  // the workspace of the steps (reserved before the first launch, so that the
  // steps below never reallocate it) plus the objective-only pass
  {
    nmf_step_opts o;
    nmf_default_opts(&o);
    if (opts) o = *opts;
    const bool joint = mode == NMF_JOINT;
    const bool pq = joint && F * N <= kPQMaxEntries;
    const Plan p = make_plan(c, F, N, K, sweep_cols_occupancy(beta_class(beta), kblocks_for(K), KIND_UPDATE, joint),
                             0, pq, joint && o.inner_iters > 1);
    if ((st = ensure_ws(c, s, std::max(p.total, make_plan(c, F, N, K).total))) != NMF_OK) return st;
  }
  if (hipSetDevice(c->device) != hipSuccess) return NMF_ERR_HIP;
  RunCtl run{(unsigned*)(c->ws + kHaltOffset), d_trace, 0, eps, d_stop};
  if (launch_run_init(s, run.halt, d_stop) != hipSuccess) return NMF_ERR_HIP;
  for (int t = 0; t < max_iters; ++t) {
    run.t = t;
    st = step_impl(c, stream, F, N, K, V, ldv, W, ldw, H, ldh, beta, mode, opts, nullptr, false, nullptr, &run);
    if (st != NMF_OK) return st;
  }
  // the objective of the last iterate and the rule at t = max_iters
  const Plan p = make_plan(c, F, N, K);
  SweepRowsArgs ra{};
  ra.V = V; ra.ldv = ldv; ra.W = W; ra.ldw = ldw; ra.H = H; ra.ldh = ldh;
  ra.F = (int)F; ra.N = (int)N; ra.K = (int)K;
  ra.bm2 = (float)(beta - 2.0); ra.kappa = opts ? opts->kappa : 0.f; ra.beta = beta;
  ra.n_groups = p.n_groups; ra.tiles_per_group = p.tiles_n;
  ra.pobj = (double*)(c->ws + p.o_pobj);
  ra.vec4 = ((uintptr_t)V % 16 == 0) && (ldv % 4 == 0);
  ra.hvec = ((uintptr_t)H % 16 == 0) && (ldh % 4 == 0);
  ra.vstream = 0;
  ra.halt = run.halt;
  const int grid = p.row_blocks * p.n_groups;
  hipError_t e = launch_sweep_rows(beta_class(beta), p.KB, KIND_OBJ, true, false, grid, s, ra);
  if (e != hipSuccess) return NMF_ERR_HIP;
  return hip_status(launch_run_decide(s, ra.pobj, grid, d_trace, max_iters, eps, run.halt, d_stop, flags_ptr(c)));
}

nmf_status nmf_kl_step_sparse(nmf_ctx_t c, void* stream, const nmf_sparse_v* V, int64_t K, float* W, int64_t ldw,
                              float* H, int64_t ldh, int32_t mode, const nmf_step_opts* opts, double* d_objective) {
  if (!c || !W || !H) return NMF_ERR_NULL;
  nmf_status st = check_sparse(V, K);
  if (st != NMF_OK) return st;
  if (ldw < K || ldh < V->N) return NMF_ERR_SHAPE;
  if (mode != NMF_ALTERNATING && mode != NMF_JOINT) return NMF_ERR_ARG;
  if ((st = check_opts(opts)) != NMF_OK) return st;
  if (opts && (opts->precision != NMF_FP32 || opts->kappa != 0.f || opts->inner_iters != 1))
    return NMF_ERR_UNSUPPORTED;
  {
    const size_t sw = span_bytes(V->F, K, ldw), sh = span_bytes(K, V->N, ldh);
    if (overlaps(W, sw, H, sh)) return NMF_ERR_ALIAS;
    const void* in[4] = {V->row_val, V->col_val, V->col_idx, V->row_idx};
    const size_t ni[4] = {sizeof(float) * (size_t)V->nnz, sizeof(float) * (size_t)V->nnz,
                          sizeof(int32_t) * (size_t)V->nnz, sizeof(int32_t) * (size_t)V->nnz};
    for (int i = 0; i < 4; ++i)
      if (overlaps(in[i], ni[i], W, sw) || overlaps(in[i], ni[i], H, sh)) return NMF_ERR_ALIAS;
  }
  hipStream_t s = (hipStream_t)stream;
  const SparsePlan p = sparse_plan(V->F, V->N, K);
  if ((st = ensure_ws(c, s, p.total)) != NMF_OK) return st;
  if (hipSetDevice(c->device) != hipSuccess) return NMF_ERR_HIP;
  SparseArgs a = sparse_args(p, c->ws, flags_ptr(c), V, K, W, ldw, H, ldh);
  a.normalize = opts ? opts->normalize : 1;
  a.d_obj = d_objective;
  if (!d_objective) a.pobj = nullptr;
  hipError_t e = launch_sparse_prep(s, a);
  if (e != hipSuccess) return NMF_ERR_HIP;
  if (mode == NMF_JOINT) {
    // the column pass needs only W~ and H~: both passes in one launch
    a.Wg = a.Wc;
    e = timed(c, NMF_KERNEL_SPARSE_PASS, s, [&] { return launch_sparse_pass(s, a, true, true); });
    if (e == hipSuccess) e = launch_sparse_update_w(s, a);
  } else {
    e = timed(c, NMF_KERNEL_SPARSE_PASS, s, [&] { return launch_sparse_pass(s, a, true, false); });
    if (e == hipSuccess) e = launch_sparse_update_w(s, a);
    a.Wg = a.Wn;
    if (e == hipSuccess)
      e = timed(c, NMF_KERNEL_SPARSE_COLS, s, [&] { return launch_sparse_pass(s, a, false, true); });
  }
  if (e == hipSuccess) e = launch_sparse_update_h(s, a);
  return hip_status(e);
}

nmf_status nmf_kl_objective_sparse(nmf_ctx_t c, void* stream, const nmf_sparse_v* V, int64_t K, const float* W,
                                   int64_t ldw, const float* H, int64_t ldh, double* d_out) {
  if (!c || !W || !H || !d_out) return NMF_ERR_NULL;
  nmf_status st = check_sparse(V, K);
  if (st != NMF_OK) return st;
  if (ldw < K || ldh < V->N) return NMF_ERR_SHAPE;
  hipStream_t s = (hipStream_t)stream;
  const SparsePlan p = sparse_plan(V->F, V->N, K);
  if ((st = ensure_ws(c, s, p.total)) != NMF_OK) return st;
  if (hipSetDevice(c->device) != hipSuccess) return NMF_ERR_HIP;
  // the preparation kernels only read W and H
  SparseArgs a = sparse_args(p, c->ws, flags_ptr(c), V, K, const_cast<float*>(W), ldw, const_cast<float*>(H), ldh);
  return hip_status(launch_sparse_objective(s, a, d_out));
}

nmf_status nmf_sparse_validate(nmf_ctx_t c, void* stream, const nmf_sparse_v* V) {
  if (!c) return NMF_ERR_NULL;
  nmf_status st = check_sparse(V, 1);
  if (st != NMF_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  if ((st = ensure_ws(c, s, kHeaderBytes)) != NMF_OK) return st;
  if (hipSetDevice(c->device) != hipSuccess) return NMF_ERR_HIP;
  SparseArgs a{};
  a.F = (int)V->F; a.N = (int)V->N; a.nnz = V->nnz;
  a.row_ptr = V->row_ptr; a.col_idx = V->col_idx; a.row_val = V->row_val;
  a.col_ptr = V->col_ptr; a.row_idx = V->row_idx; a.col_val = V->col_val;
  a.flags = flags_ptr(c);
  return hip_status(launch_sparse_validate(s, a));
}

nmf_status nmf_beta_validate(nmf_ctx_t c, void* stream, int64_t F, int64_t N, int64_t K, const float* V,
                             int64_t ldv, const float* W, int64_t ldw, const float* H, int64_t ldh, double beta,
                             float kappa) {
  if (!c) return NMF_ERR_NULL;
  nmf_status st = check_mats(F, N, K, V, ldv, W, ldw, H, ldh);
  if (st != NMF_OK) return st;
  if (!is_fin(beta) || !std::isfinite(kappa) || kappa < 0.f) return NMF_ERR_BETA;
  hipStream_t s = (hipStream_t)stream;
  if ((st = ensure_ws(c, s, kHeaderBytes)) != NMF_OK) return st;
  if (hipSetDevice(c->device) != hipSuccess) return NMF_ERR_HIP;
  const int zero_bad = (beta <= 0.0 && kappa == 0.f) ? 1 : 0;
  return hip_status(launch_validate(s, V, ldv, W, ldw, H, ldh, (int)F, (int)N, (int)K, zero_bad, flags_ptr(c)));
}

nmf_status nmf_get_flags(nmf_ctx_t c, void* stream, uint32_t* flags, int32_t clear) {
  if (!c || !flags) return NMF_ERR_NULL;
  *flags = 0;
  if (!c->ws && !c->bmem) return NMF_OK;
  if (hipSetDevice(c->device) != hipSuccess) return NMF_ERR_HIP;
  hipStream_t s = (hipStream_t)stream;
  // the step workspace's word and the batched region's word
  char* words[2] = {c->ws, c->bmem};
  uint32_t got[2] = {0, 0};
  for (int k = 0; k < 2; ++k)
    if (words[k] && hipMemcpyAsync(&got[k], words[k], sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
      return NMF_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return NMF_ERR_HIP;
  *flags = got[0] | got[1];
  if (clear) {
    const uint32_t z = 0;
    for (int k = 0; k < 2; ++k)
      if (words[k] && hipMemcpyAsync(words[k], &z, sizeof(uint32_t), hipMemcpyHostToDevice, s) != hipSuccess)
        return NMF_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return NMF_ERR_HIP;
  }
  return NMF_OK;
}

nmf_status nmf_profile_enable(nmf_ctx_t c, uint32_t mask) {
  if (!c) return NMF_ERR_NULL;
  c->profile_mask = mask;
  return NMF_OK;
}

nmf_status nmf_profile_read(nmf_ctx_t c, int32_t kernel, double* total_ms, int64_t* launches) {
  if (!c || !total_ms || !launches) return NMF_ERR_NULL;
  if (kernel < 0 || kernel >= NMF_KERNEL_COUNT) return NMF_ERR_ARG;
  nmf_status st = NMF_OK;
  for (auto& t : c->pending[kernel]) {
    float ms = 0.f;
    if (hipEventSynchronize(t.stop) != hipSuccess || hipEventElapsedTime(&ms, t.start, t.stop) != hipSuccess)
      st = NMF_ERR_HIP;
    c->prof_ms[kernel] += ms;
    c->prof_count[kernel] += 1;
    c->event_pool.push_back(t.start);
    c->event_pool.push_back(t.stop);
  }
  c->pending[kernel].clear();
  *total_ms = c->prof_ms[kernel];
  *launches = c->prof_count[kernel];
  c->prof_ms[kernel] = 0.0;
  c->prof_count[kernel] = 0;
  return st;
}

nmf_status nmf_profile_phases(nmf_ctx_t c, void* stream, double* us, int32_t n) {
  if (!c || !us) return NMF_ERR_NULL;
  if (n < 1 || n > 7) return NMF_ERR_ARG;
  if (!c->ws) return NMF_ERR_ARG;
  unsigned long long t[8];
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(t, c->ws + 64, sizeof(t), hipMemcpyDeviceToHost, s) != hipSuccess) return NMF_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return NMF_ERR_HIP;
  for (int i = 0; i < n; ++i) us[i] = (double)(t[i + 1] - t[i]) * 0.01;  // 100 MHz clock
  return NMF_OK;
}

nmf_status nmf_set_path(nmf_ctx_t c, int32_t path) {
  if (!c) return NMF_ERR_NULL;
  if (path != NMF_PATH_AUTO && path != NMF_PATH_STREAM && path != NMF_PATH_FUSED) return NMF_ERR_ARG;
  c->path = path;
  return NMF_OK;
}

nmf_status nmf_set_launch(nmf_ctx_t c, int32_t target_blocks, int32_t min_tiles) {
  if (!c) return NMF_ERR_NULL;
  if (target_blocks < 0 || min_tiles < 0) return NMF_ERR_ARG;
  c->target_blocks = target_blocks;
  c->min_tiles = min_tiles > 0 ? min_tiles : 1;
  return NMF_OK;
}

}  // extern "C"

namespace {

// Validated options of a batch (precision FP32 or BF16, one sub-iteration, no
// Gram form); NMF_OK or the status to return.
nmf_status batch_opts(const nmf_step_opts* opts, nmf_step_opts* o) {
  nmf_status st = check_opts(opts);
  if (st != NMF_OK) return st;
  nmf_default_opts(o);
  if (opts) *o = *opts;
  if (o->precision != NMF_FP32 && o->precision != NMF_BF16) return NMF_ERR_UNSUPPORTED;
  if (o->inner_iters != 1 || o->gram) return NMF_ERR_UNSUPPORTED;
  return NMF_OK;
}

int batch_grid(nmf_ctx_s* c, int prec, bool joint) {
  int& g = c->batch_grid[prec == NMF_BF16][joint];
  if (g <= 0) g = batched_max_blocks(prec, joint, c->num_cus);
  return g;
}

// nmf_batch_create with an explicit tile count per bucket.
nmf_status batch_create(nmf_ctx_s* c, const nmf_problem* pr, int count, int mode, const nmf_step_opts& o,
                        const int* tiles, int workers, int lag, nmf_batch_t* out) {
  *out = nullptr;
  for (int i = 0; i < count; ++i) {
    const nmf_problem& q = pr[i];
    nmf_status st = nmf_check_step_args(q.F, q.N, q.K, q.V, q.ldv, q.W, q.ldw, q.H, q.ldh, q.beta, mode, &o);
    if (st != NMF_OK) return st;
    if (q.K > 64) return NMF_ERR_UNSUPPORTED;
  }
  nmf_status st = check_batch_alias(pr, count);
  if (st != NMF_OK) return st;
  if (hipSetDevice(c->device) != hipSuccess) return NMF_ERR_HIP;
  const bool joint = mode == NMF_JOINT;
  const int max_grid = batch_grid(c, o.precision, joint);
  if (max_grid <= 0) return NMF_ERR_HIP;
  const int grid = workers > 0 ? std::min(workers, max_grid) : max_grid;

  // plans and memory layout
  std::vector<Plan> plans(count);
  std::vector<size_t> base(count);
  size_t off = kHeaderBytes;
  const size_t o_done = off;
  off = align_up(off + sizeof(unsigned) * 4 * (size_t)count);
  const size_t o_desc = off;
  off = align_up(off + sizeof(BatchProblem) * (size_t)count);
  int64_t total = 0;
  for (int i = 0; i < count; ++i) {
    const nmf_problem& q = pr[i];
    plans[i] = make_batch_plan(q.F, q.N, q.K, q.beta, tiles[bucket_of(q.F, q.N, q.K, q.beta)], joint, o.precision);
    total += batch_items(plans[i], q.F, o.precision);
  }
  if (total >= (int64_t)1 << 31) return NMF_ERR_UNSUPPORTED;
  const size_t o_list = off;
  off = align_up(off + sizeof(int2) * (size_t)total);
  for (int i = 0; i < count; ++i) {
    base[i] = off;
    off = align_up(off + plans[i].total);
  }
  nmf_batch_s* b = new (std::nothrow) nmf_batch_s();
  if (!b) return NMF_ERR_HIP;
  b->device = c->device;
  b->count = count;
  b->mode = mode;
  b->prec = o.precision;
  b->grid = grid;
  b->total = total;
  b->bytes = off;
  if (hipMalloc(&b->mem, off) != hipSuccess) {
    delete b;
    return NMF_ERR_HIP;
  }
  char* mem = b->mem;
  unsigned* flags = (unsigned*)mem;

  // descriptors
  std::vector<BatchProblem> desc(count);
  for (int i = 0; i < count; ++i) desc[i] = make_batch_problem(plans[i], mem + base[i], flags, pr[i], joint, o);
  // queue, larger problems first: phase-major (lag 0), or pipelined with phase q
  // of the problem at position j listed at step j + q lag.  Either way every
  // item is listed after all the items it waits for.
  std::vector<int> order(count);
  for (int i = 0; i < count; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int bb) {
    return pr[a].F * pr[a].N * pr[a].K > pr[bb].F * pr[bb].N * pr[bb].K;
  });
  std::vector<int2> list;
  list.reserve((size_t)total);
  auto emit = [&](int i, int ph) {
    for (int it = 0; it < desc[i].items[ph]; ++it) list.push_back(make_int2(i, (ph << 24) | it));
  };
  if (lag == 0) {
    for (int ph = 0; ph < 4; ++ph)
      for (int i : order) emit(i, ph);
  } else {
    for (int64_t step = 0; step < (int64_t)count + 3 * (int64_t)lag; ++step)
      for (int ph = 0; ph < 4; ++ph) {
        const int64_t j = step - (int64_t)ph * lag;
        if (j >= 0 && j < count) emit(order[j], ph);
      }
  }

  hipError_t e = hipMemset(mem, 0, o_desc);
  if (e == hipSuccess) e = hipMemcpy(mem + o_desc, desc.data(), sizeof(BatchProblem) * count, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(mem + o_list, list.data(), sizeof(int2) * list.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(b->mem);
    delete b;
    return NMF_ERR_HIP;
  }
  BatchArgs& a = b->args;
  a.probs = (const BatchProblem*)(mem + o_desc);
  a.list = (const int2*)(mem + o_list);
  a.total = (int)total;
  a.counts = nullptr;
  a.next = (unsigned*)(mem + 8);
  a.exited = (unsigned*)(mem + 12);
  a.done = (unsigned*)(mem + o_done);
  a.nprob = count;
  a.d_obj = nullptr;
  a.flags = flags;
  a.spin_limit = kBatchSpinLimit;
  *out = b;
  return NMF_OK;
}

// ---- tuning cache: one text line per key ----
//   nmf_tune 2 <arch> <compute units> <mode> <precision> <bucket mask, hex> <tiles x NMF_BATCH_BUCKETS> <ms>
struct TuneKey {
  char arch[64];
  int cus, mode, prec;
};

struct TuneEntry {
  uint64_t mask = 0;
  int tiles[kBatchBuckets] = {};
  double ms = 0.0;
};

constexpr int kTuneVersion = 2;

bool parse_tune_line(const char* line, TuneKey* k, TuneEntry* e) {
  int ver = 0, used = 0;
  unsigned long long mask = 0;
  if (sscanf(line, "nmf_tune %d %63s %d %d %d %llx%n", &ver, k->arch, &k->cus, &k->mode, &k->prec, &mask, &used) != 6 ||
      ver != kTuneVersion)
    return false;
  const char* p = line + used;
  for (int b = 0; b < kBatchBuckets; ++b) {
    char* end = nullptr;
    const long t = std::strtol(p, &end, 10);
    if (end == p || t < 1 || t > 4096) return false;
    e->tiles[b] = (int)t;
    p = end;
  }
  char* end = nullptr;
  e->ms = std::strtod(p, &end);
  if (end == p) return false;
  e->mask = (uint64_t)mask & ((kBatchBuckets >= 64) ? ~0ull : ((1ull << kBatchBuckets) - 1));
  return true;
}

bool same_key(const TuneKey& a, const TuneKey& b) {
  return std::strcmp(a.arch, b.arch) == 0 && a.cus == b.cus && a.mode == b.mode && a.prec == b.prec;
}

// Lines of the cache file (none if it does not exist or cannot be read).
std::vector<std::string> read_lines(const char* path) {
  std::vector<std::string> lines;
  FILE* f = std::fopen(path, "r");
  if (!f) return lines;
  char buf[512];
  std::string cur;
  while (std::fgets(buf, sizeof(buf), f)) {
    cur += buf;
    if (!cur.empty() && cur.back() == '\n') {
      cur.pop_back();
      lines.push_back(cur);
      cur.clear();
    }
  }
  if (!cur.empty()) lines.push_back(cur);
  std::fclose(f);
  return lines;
}

bool cache_lookup(const char* path, const TuneKey& key, TuneEntry* out) {
  bool found = false;
  for (const std::string& l : read_lines(path)) {
    TuneKey k;
    TuneEntry e;
    if (parse_tune_line(l.c_str(), &k, &e) && same_key(k, key)) {
      *out = e;  // the last entry of a key wins
      found = true;
    }
  }
  return found;
}

nmf_status cache_store(const char* path, const TuneKey& key, const TuneEntry& e) {
  std::vector<std::string> keep;
  for (const std::string& l : read_lines(path)) {
    TuneKey k;
    TuneEntry old;
    if (!(parse_tune_line(l.c_str(), &k, &old) && same_key(k, key))) keep.push_back(l);
  }
  std::string line = "nmf_tune " + std::to_string(kTuneVersion) + " " + key.arch + " " + std::to_string(key.cus) +
                     " " + std::to_string(key.mode) + " " + std::to_string(key.prec);
  char buf[64];
  std::snprintf(buf, sizeof(buf), " 0x%012llx", (unsigned long long)e.mask);
  line += buf;
  for (int b = 0; b < kBatchBuckets; ++b) line += " " + std::to_string(e.tiles[b]);
  std::snprintf(buf, sizeof(buf), " %.6f", e.ms);
  line += buf;
  keep.push_back(line);
  const std::string tmp = std::string(path) + ".tmp." + std::to_string((long)getpid());
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return NMF_ERR_IO;
  bool ok = true;
  for (const std::string& l : keep) ok = ok && std::fprintf(f, "%s\n", l.c_str()) > 0;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    (void)std::remove(tmp.c_str());
    return NMF_ERR_IO;
  }
  return NMF_OK;
}

nmf_status upload_tiles(nmf_ctx_s* c) {
  if (!c->bmem) return NMF_OK;
  if (hipSetDevice(c->device) != hipSuccess) return NMF_ERR_HIP;
  return hip_status(hipMemcpy(c->bmem + c->bo_tiles, c->batch_tiles, sizeof(int) * kBatchBuckets,
                              hipMemcpyHostToDevice));
}

}  // namespace

extern "C" {

nmf_status nmf_batch_create(nmf_ctx_t c, const nmf_problem* pr, int32_t count, int32_t mode,
                            const nmf_step_opts* opts, const nmf_batch_config* cfg, nmf_batch_t* out) {
  if (!out) return NMF_ERR_NULL;
  *out = nullptr;
  if (!c || !pr) return NMF_ERR_NULL;
  if (count < 1) return NMF_ERR_ARG;
  if (mode != NMF_ALTERNATING && mode != NMF_JOINT) return NMF_ERR_ARG;
  nmf_step_opts o;
  nmf_status st = batch_opts(opts, &o);
  if (st != NMF_OK) return st;
  if (cfg && (cfg->workers < 0 || cfg->tiles_per_item < 0 || cfg->lag < 0)) return NMF_ERR_ARG;
  int tiles[kBatchBuckets];
  for (int b = 0; b < kBatchBuckets; ++b)
    tiles[b] = cfg && cfg->tiles_per_item > 0 ? cfg->tiles_per_item : c->batch_tiles[b];
  return batch_create(c, pr, count, mode, o, tiles, cfg ? cfg->workers : 0, cfg ? cfg->lag : 0, out);
}

nmf_status nmf_batch_step(nmf_batch_t b, void* stream, double* d_objectives) {
  if (!b) return NMF_ERR_NULL;
  if (hipSetDevice(b->device) != hipSuccess) return NMF_ERR_HIP;
  BatchArgs a = b->args;
  a.d_obj = d_objectives;
  return hip_status(launch_batched(b->prec, b->mode == NMF_JOINT, b->grid, (hipStream_t)stream, a));
}

nmf_status nmf_batch_get_flags(nmf_batch_t b, void* stream, uint32_t* flags, int32_t clear) {
  if (!b || !flags) return NMF_ERR_NULL;
  *flags = 0;
  if (hipSetDevice(b->device) != hipSuccess) return NMF_ERR_HIP;
  hipStream_t s = (hipStream_t)stream;
  if (hipMemcpyAsync(flags, b->mem, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess) return NMF_ERR_HIP;
  if (hipStreamSynchronize(s) != hipSuccess) return NMF_ERR_HIP;
  if (clear) {
    const uint32_t z = 0;
    if (hipMemcpyAsync(b->mem, &z, sizeof(uint32_t), hipMemcpyHostToDevice, s) != hipSuccess) return NMF_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return NMF_ERR_HIP;
  }
  return NMF_OK;
}

nmf_status nmf_batch_info(nmf_batch_t b, int64_t* work_items, int32_t* workers, int64_t* device_bytes) {
  if (!b) return NMF_ERR_NULL;
  if (work_items) *work_items = b->total;
  if (workers) *workers = b->grid;
  if (device_bytes) *device_bytes = (int64_t)b->bytes;
  return NMF_OK;
}

nmf_status nmf_batch_destroy(nmf_batch_t b) {
  if (!b) return NMF_ERR_NULL;
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  if (b->mem) (void)hipFree(b->mem);
  delete b;
  return NMF_OK;
}

int32_t nmf_batch_bucket(int64_t F, int64_t N, int64_t K, double beta) {
  if (F < 1 || N < 1 || K < 1 || K > 64 || !std::isfinite(beta)) return -1;
  return bucket_of(F, N, K, beta);
}

nmf_status nmf_set_batch_tiles(nmf_ctx_t c, const int32_t* tiles) {
  if (!c || !tiles) return NMF_ERR_NULL;
  for (int b = 0; b < kBatchBuckets; ++b)
    if (tiles[b] < 1 || tiles[b] > 4096) return NMF_ERR_ARG;
  for (int b = 0; b < kBatchBuckets; ++b) c->batch_tiles[b] = tiles[b];
  return upload_tiles(c);
}

nmf_status nmf_get_batch_tiles(nmf_ctx_t c, int32_t* tiles) {
  if (!c || !tiles) return NMF_ERR_NULL;
  for (int b = 0; b < kBatchBuckets; ++b) tiles[b] = c->batch_tiles[b];
  return NMF_OK;
}

nmf_status nmf_batch_requirements(const nmf_problem* pr, int32_t count, int32_t mode, int32_t precision,
                                  const int32_t* tiles, int64_t* items, int64_t* workspace_bytes) {
  if (!pr || !items || !workspace_bytes) return NMF_ERR_NULL;
  *items = 0;
  *workspace_bytes = 0;
  if (count < 1) return NMF_ERR_ARG;
  if (mode != NMF_ALTERNATING && mode != NMF_JOINT) return NMF_ERR_ARG;
  if (precision != NMF_FP32 && precision != NMF_BF16 && precision != NMF_FP16) return NMF_ERR_ARG;
  if (precision == NMF_FP16) return NMF_ERR_UNSUPPORTED;  // batches run float32 or bfloat16 products
  if (tiles)
    for (int b = 0; b < kBatchBuckets; ++b)
      if (tiles[b] < 1 || tiles[b] > 4096) return NMF_ERR_ARG;
  int64_t n = 0, bytes = 0;
  for (int i = 0; i < count; ++i) {
    const nmf_problem& q = pr[i];
    if (q.F < 1 || q.N < 1 || q.K < 1 || q.F > INT32_MAX || q.N > INT32_MAX) return NMF_ERR_SHAPE;
    if (q.K > 64) return NMF_ERR_UNSUPPORTED;
    if (!std::isfinite(q.beta)) return NMF_ERR_BETA;
    const int b = bucket_of(q.F, q.N, q.K, q.beta);
    const Plan p =
        make_batch_plan(q.F, q.N, q.K, q.beta, tiles ? tiles[b] : kBatchTilesDefault, mode == NMF_JOINT, precision);
    n += batch_items(p, q.F, precision);
    bytes += (int64_t)align_up(p.total);
  }
  *items = n;
  *workspace_bytes = bytes;
  return NMF_OK;
}

nmf_status nmf_reserve_batched(nmf_ctx_t c, int32_t max_problems, int64_t max_items, int64_t workspace_bytes) {
  if (!c) return NMF_ERR_NULL;
  if (max_problems < 1 || max_items < 1 || max_items > INT32_MAX || workspace_bytes < 0) return NMF_ERR_ARG;
  if (c->b_captured) return NMF_ERR_WORKSPACE;
  if (hipSetDevice(c->device) != hipSuccess) return NMF_ERR_HIP;
  // the persistent grids, so that a captured step makes no occupancy query
  for (int prec : {NMF_FP32, NMF_BF16})
    for (bool joint : {false, true})
      if (batch_grid(c, prec, joint) <= 0) return NMF_ERR_HIP;
  const size_t P = (size_t)max_problems;
  size_t off = kHeaderBytes;  // flags @0, queue position @8, exits @12, counts @16
  auto take = [&](size_t bytes) { size_t r = off; off = align_up(off + bytes); return r; };
  const size_t o_tiles = take(sizeof(int) * kBatchBuckets);
  const size_t o_done = take(sizeof(unsigned) * 4 * P);
  const size_t o_desc = take(sizeof(BatchProblem) * P);
  const size_t o_list = take(sizeof(int2) * (size_t)max_items);
  const size_t o_sbytes = take(sizeof(int64_t) * P);
  const size_t o_sitems = take(sizeof(int64_t) * 4 * P);
  const size_t o_soff = take(sizeof(int64_t) * 4 * P);
  const size_t o_sorder = take(sizeof(int) * P);
  const size_t o_work = take((size_t)workspace_bytes);
  uint32_t flags_keep = 0;
  if (c->bmem) {
    if (hipDeviceSynchronize() != hipSuccess) return NMF_ERR_HIP;
    (void)hipMemcpy(&flags_keep, c->bmem, sizeof(uint32_t), hipMemcpyDeviceToHost);
    (void)hipFree(c->bmem);
    c->bmem = nullptr;
    c->bbytes = 0;
  }
  void* p = nullptr;
  if (hipMalloc(&p, off) != hipSuccess) return NMF_ERR_HIP;
  char* m = (char*)p;
  hipError_t e = hipMemset(m, 0, o_desc);  // header, tile table, done counters
  if (e == hipSuccess) e = hipMemcpy(m, &flags_keep, sizeof(uint32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(m + o_tiles, c->batch_tiles, sizeof(int) * kBatchBuckets, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(p);
    return NMF_ERR_HIP;
  }
  c->bmem = m;
  c->bbytes = off;
  c->b_max_problems = max_problems;
  c->b_max_items = max_items;
  c->b_work_bytes = workspace_bytes;
  c->bo_tiles = o_tiles;
  c->bo_done = o_done;
  c->bo_desc = o_desc;
  c->bo_list = o_list;
  c->bo_sbytes = o_sbytes;
  c->bo_sitems = o_sitems;
  c->bo_soff = o_soff;
  c->bo_sorder = o_sorder;
  c->bo_work = o_work;
  return NMF_OK;
}

nmf_status nmf_beta_step_batched(nmf_ctx_t c, void* stream, int32_t count, const nmf_problem* d_problems,
                                 int32_t mode, const nmf_step_opts* opts, double* d_objectives,
                                 const int32_t* d_count) {
  if (!c || !d_problems) return NMF_ERR_NULL;
  if (count < 1) return NMF_ERR_ARG;
  if (mode != NMF_ALTERNATING && mode != NMF_JOINT) return NMF_ERR_ARG;
  nmf_step_opts o;
  nmf_status st = batch_opts(opts, &o);
  if (st != NMF_OK) return st;
  if (!c->bmem || count > c->b_max_problems) return NMF_ERR_WORKSPACE;
  if (hipSetDevice(c->device) != hipSuccess) return NMF_ERR_HIP;
  hipStream_t s = (hipStream_t)stream;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return NMF_ERR_HIP;
  if (cs != hipStreamCaptureStatusNone) c->b_captured = true;
  const bool joint = mode == NMF_JOINT;
  const int grid = batch_grid(c, o.precision, joint);
  if (grid <= 0) return NMF_ERR_HIP;
  char* m = c->bmem;
  BatchPlanArgs pa{};
  pa.problems = d_problems;
  pa.count = count;
  pa.d_count = d_count;
  pa.tiles = (const int*)(m + c->bo_tiles);
  pa.joint = joint;
  pa.opts = o;
  pa.work = m + c->bo_work;
  pa.work_bytes = c->b_work_bytes;
  pa.max_items = c->b_max_items;
  pa.s_bytes = (int64_t*)(m + c->bo_sbytes);
  pa.s_items = (int64_t*)(m + c->bo_sitems);
  pa.s_off = (int64_t*)(m + c->bo_soff);
  pa.s_order = (int*)(m + c->bo_sorder);
  pa.desc = (BatchProblem*)(m + c->bo_desc);
  pa.list = (int2*)(m + c->bo_list);
  pa.done = (unsigned*)(m + c->bo_done);
  pa.next = (unsigned*)(m + 8);
  pa.exited = (unsigned*)(m + 12);
  pa.counts = (int*)(m + 16);
  pa.flags = (unsigned*)m;
  hipError_t e = launch_batch_plan(s, pa);
  if (e != hipSuccess) return NMF_ERR_HIP;
  BatchArgs a{};
  a.probs = pa.desc;
  a.list = pa.list;
  a.total = 0;
  a.counts = pa.counts;
  a.next = pa.next;
  a.exited = pa.exited;
  a.done = pa.done;
  a.nprob = 0;
  a.d_obj = d_objectives;
  a.flags = pa.flags;
  a.spin_limit = kBatchSpinLimit;
  return hip_status(launch_batched(o.precision, joint, grid, s, a));
}

nmf_status nmf_tune(nmf_ctx_t c, void* stream, const nmf_problem* pr, int32_t count, int32_t mode,
                    const nmf_step_opts* opts, int32_t iters, const char* cache_path, int32_t* tiles_out,
                    double* ms_out, int32_t* from_cache) {
  if (!c || !pr || !tiles_out) return NMF_ERR_NULL;
  if (count < 1 || iters < 1) return NMF_ERR_ARG;
  if (mode != NMF_ALTERNATING && mode != NMF_JOINT) return NMF_ERR_ARG;
  nmf_step_opts o;
  nmf_status st = batch_opts(opts, &o);
  if (st != NMF_OK) return st;
  for (int i = 0; i < count; ++i) {
    const nmf_problem& q = pr[i];
    if ((st = nmf_check_step_args(q.F, q.N, q.K, q.V, q.ldv, q.W, q.ldw, q.H, q.ldh, q.beta, mode, &o)) != NMF_OK)
      return st;
    if (q.K > 64) return NMF_ERR_UNSUPPORTED;
  }
  if ((st = check_batch_alias(pr, count)) != NMF_OK) return st;
  if (from_cache) *from_cache = 0;
  if (hipSetDevice(c->device) != hipSuccess) return NMF_ERR_HIP;
  const bool joint = mode == NMF_JOINT;

  TuneKey key{};
  {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) != hipSuccess) return NMF_ERR_HIP;
    size_t n = 0;
    while (n + 1 < sizeof(key.arch) && prop.gcnArchName[n] && prop.gcnArchName[n] != ':' &&
           prop.gcnArchName[n] != ' ')
      ++n;
    std::memcpy(key.arch, prop.gcnArchName, n);
    key.arch[n] = 0;
    if (n == 0) std::strcpy(key.arch, "gpu");
    key.cus = c->num_cus;
    key.mode = mode;
    key.prec = o.precision;
  }
  uint64_t needed = 0;
  for (int i = 0; i < count; ++i) needed |= 1ull << bucket_of(pr[i].F, pr[i].N, pr[i].K, pr[i].beta);
  TuneEntry cached;
  const bool have = cache_path && cache_lookup(cache_path, key, &cached);
  int table[kBatchBuckets];
  for (int b = 0; b < kBatchBuckets; ++b)
    table[b] = have && (cached.mask >> b & 1ull) ? cached.tiles[b] : c->batch_tiles[b];
  if (have && (needed & ~cached.mask) == 0) {
    for (int b = 0; b < kBatchBuckets; ++b) c->batch_tiles[b] = table[b];
    if ((st = upload_tiles(c)) != NMF_OK) return st;
    for (int b = 0; b < kBatchBuckets; ++b) tiles_out[b] = table[b];
    if (ms_out) *ms_out = cached.ms;
    if (from_cache) *from_cache = 1;
    return NMF_OK;
  }

  // save W and H of every problem (packed) to restore them after each timing
  hipStream_t s = (hipStream_t)stream;
  size_t words = 0;
  for (int i = 0; i < count; ++i) words += (size_t)(pr[i].F * pr[i].K + pr[i].K * pr[i].N);
  float* save = nullptr;
  if (hipMalloc(&save, sizeof(float) * std::max<size_t>(words, 1)) != hipSuccess) return NMF_ERR_HIP;
  auto copy_all = [&](bool to_save) -> hipError_t {
    size_t w = 0;
    for (int i = 0; i < count; ++i) {
      const nmf_problem& q = pr[i];
      float* sw = save + w;
      float* sh = sw + q.F * q.K;
      w += (size_t)(q.F * q.K + q.K * q.N);
      hipError_t e;
      if (to_save) {
        e = hipMemcpy2DAsync(sw, q.K * 4, q.W, q.ldw * 4, q.K * 4, q.F, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpy2DAsync(sh, q.N * 4, q.H, q.ldh * 4, q.N * 4, q.K, hipMemcpyDeviceToDevice, s);
      } else {
        e = hipMemcpy2DAsync(q.W, q.ldw * 4, sw, q.K * 4, q.K * 4, q.F, hipMemcpyDeviceToDevice, s);
        if (e == hipSuccess) e = hipMemcpy2DAsync(q.H, q.ldh * 4, sh, q.N * 4, q.N * 4, q.K, hipMemcpyDeviceToDevice, s);
      }
      if (e != hipSuccess) return e;
    }
    return hipStreamSynchronize(s);
  };
  hipEvent_t e0 = nullptr, e1 = nullptr;
  // time per step of the whole set under `t`; +inf if a work item gave up waiting
  auto time_table = [&](const int* t, double* ms) -> nmf_status {
    nmf_batch_t b = nullptr;
    nmf_status r = batch_create(c, pr, count, mode, o, t, 0, 0, &b);
    if (r != NMF_OK) return r;
    float el = 0.f;
    hipError_t e = launch_batched(b->prec, joint, b->grid, s, b->args);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int k = 0; e == hipSuccess && k < iters; ++k) e = launch_batched(b->prec, joint, b->grid, s, b->args);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&el, e0, e1);
    uint32_t fl = 0;
    if (e == hipSuccess && nmf_batch_get_flags(b, stream, &fl, 1) != NMF_OK) e = hipErrorUnknown;
    (void)nmf_batch_destroy(b);
    if (e == hipSuccess) e = copy_all(false);
    if (e != hipSuccess) return NMF_ERR_HIP;
    *ms = (fl & NMF_FLAG_BARRIER) ? HUGE_VAL : (double)el / iters;
    return NMF_OK;
  };
  // how the problems of bucket `b` are split under `t` tiles per item
  auto split_of = [&](int b, int t) {
    std::vector<int> sig;
    for (int i = 0; i < count; ++i) {
      const nmf_problem& q = pr[i];
      if (bucket_of(q.F, q.N, q.K, q.beta) != b) continue;
      const Plan p = make_batch_plan(q.F, q.N, q.K, q.beta, t, joint, o.precision);
      sig.insert(sig.end(), {p.n_groups, p.tiles_n, p.f_groups, p.tiles_f});
    }
    return sig;
  };
  static const int kCandidates[] = {4, 8, 16, 32, 64, 128, 256};
  double best = HUGE_VAL;
  st = NMF_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess || copy_all(true) != hipSuccess)
    st = NMF_ERR_HIP;
  if (st == NMF_OK) st = time_table(table, &best);
  const uint64_t todo = needed & ~(have ? cached.mask : 0ull);
  for (int b = 0; st == NMF_OK && b < kBatchBuckets; ++b) {
    if (!(todo >> b & 1ull)) continue;
    std::vector<std::vector<int>> seen{split_of(b, table[b])};
    for (int cand : kCandidates) {
      std::vector<int> sig = split_of(b, cand);
      if (std::find(seen.begin(), seen.end(), sig) != seen.end()) continue;
      seen.push_back(sig);
      int trial[kBatchBuckets];
      std::memcpy(trial, table, sizeof(trial));
      trial[b] = cand;
      double ms = HUGE_VAL;
      if ((st = time_table(trial, &ms)) != NMF_OK) break;
      if (ms < best) {
        best = ms;
        table[b] = cand;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(save);
  if (st != NMF_OK) return st;
  for (int b = 0; b < kBatchBuckets; ++b) c->batch_tiles[b] = table[b];
  if ((st = upload_tiles(c)) != NMF_OK) return st;
  for (int b = 0; b < kBatchBuckets; ++b) tiles_out[b] = table[b];
  if (ms_out) *ms_out = best;
  if (cache_path) {
    TuneEntry e;
    e.mask = needed | (have ? cached.mask : 0ull);
    std::memcpy(e.tiles, table, sizeof(table));
    e.ms = best;
    if ((st = cache_store(cache_path, key, e)) != NMF_OK) return st;
  }
  return NMF_OK;
}

}  // extern "C"
