// Batched path: many frames of mixed sizes through one persistent tile-queue
// launch per pass, the whole niter loop recorded once per batch shape as a
// HIP graph and replayed; the tile shape is picked by timing the candidates
// on the first call for a batch shape.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "lacosmic.h"
#include "lacosmic_internal.h"

namespace lac {

// Per-frame counters are packed in one device block so a single copy reads
// them all back: for each frame, niter + 1 counters (new pixels per
// iteration, then the unreplaced pixels), then the status word (in an 8-byte
// slot) and kCntPerIter list lengths per iteration (4 bytes each).
static size_t counter_stride(int niter) {
  return (size_t)niter + 2 + ((size_t)kCntPerIter * niter + 1) / 2;
}

// Frames are split into groups of about equal pixel counts; each group's
// passes form their own chain of launches, on its own stream inside the
// recorded graph, so one group's latency-bound passes and launch tails
// overlap another group's work.  The frame table holds the groups one after
// another.
struct BatchPlan {
  // signature (est: some frame estimates its gain, so every iteration
  // launches the gain passes and A1)
  int n = 0, niter = 0, early = 0, est = 0, cfg = 0, mode = kModeQueue;
  std::vector<int64_t> hs, ws;  // in the caller's order
  // frame groups: table entry t holds the caller's frame order[t]; group g is
  // entries [gstart[g], gstart[g + 1]); its tile bases start at goff[g] in
  // tile_base_dev (pass-A tiles, then pass-B tiles, (ng + 1) each)
  int ngroups = 1;
  std::vector<int> order, gstart, goff, total_a, total_b;
  std::vector<int> gain_nbx;  // per group: blocks per frame of the gain passes
  // device buffers
  char* ws_dev = nullptr;           // per-frame workspaces
  FrameDev* frames_dev = nullptr;   // frame table
  int* tile_base_dev = nullptr;
  unsigned int* cursors_dev = nullptr;  // ncur() per group
  unsigned long long* counters_dev = nullptr;
  std::vector<WsLayout> lay;  // per table entry
  std::vector<size_t> ws_off;
  FrameDev* frames_pin = nullptr;   // pinned staging of the frame table
  hipEvent_t table_done = nullptr;  // the last upload of frames_pin finished
  // the last enqueued run of the plan (graph replay or eager replay) finished:
  // it reads the frame table and uses the workspaces, so the next run, on
  // whatever stream, waits for it before it uploads a new table
  hipEvent_t run_done = nullptr;
  hipGraphExec_t exec = nullptr;
  int blocks[kDenseSlots] = {};  // persistent grid of each dense pass
  std::vector<hipStream_t> gstream;  // groups 1.. (group 0 runs on the capture stream)
  std::vector<hipEvent_t> fork, join;
  std::vector<hipEvent_t> a1_done;  // group g's first A1 finished (groups 0 .. G-2)
  // timing events for an eager replay of the plan (lacosmic_batch_pass_ms),
  // per group: marks[g * per + 0] before its first pass, marks[g * per + k + 1]
  // after pass k (per = kPassesPerIter * niter + 1)
  std::vector<hipEvent_t> marks;
  int ncur() const { return 8 * kDenseSlots * niter; }
  ~BatchPlan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    for (hipEvent_t e : marks) (void)hipEventDestroy(e);
    for (hipEvent_t e : fork) (void)hipEventDestroy(e);
    for (hipEvent_t e : join) (void)hipEventDestroy(e);
    for (hipEvent_t e : a1_done) (void)hipEventDestroy(e);
    for (hipStream_t st : gstream) (void)hipStreamDestroy(st);
    if (table_done) (void)hipEventDestroy(table_done);
    if (run_done) (void)hipEventDestroy(run_done);
    if (frames_pin) (void)hipHostFree(frames_pin);
    if (ws_dev) (void)hipFree(ws_dev);
    if (frames_dev) (void)hipFree(frames_dev);
    if (tile_base_dev) (void)hipFree(tile_base_dev);
    if (cursors_dev) (void)hipFree(cursors_dev);
    if (counters_dev) (void)hipFree(counters_dev);
  }
  bool same(int n_, const int64_t* h_, const int64_t* w_, int niter_, int early_, int est_) const {
    if (n_ != n || niter_ != niter || early_ != early || est_ != est) return false;
    for (int i = 0; i < n; ++i)
      if (hs[i] != h_[i] || ws[i] != w_[i]) return false;
    return true;
  }
};

struct BatchCache {
  BatchPlan* plan = nullptr;  // the most recent batch shape
  std::vector<std::pair<std::vector<int64_t>, int>> tuned;  // shape key -> groups << 8 | cfg << 1 | mode
};

void DevCtx::release_extras() {
  if (batch) {
    delete batch->plan;
    delete batch;
    batch = nullptr;
  }
}

static std::vector<int64_t> shape_key(int n, const int64_t* hs, const int64_t* ws, int niter,
                                      int early, int est) {
  std::vector<int64_t> k;
  k.reserve(2 * n + 3);
  k.push_back(niter);
  k.push_back(early);
  k.push_back(est);
  for (int i = 0; i < n; ++i) {
    k.push_back(hs[i]);
    k.push_back(ws[i]);
  }
  return k;
}

// Fill the pinned frame table for this call's buffers and parameters.
static void fill_table(BatchPlan& P, const float* const* imgs, const lacosmic_params* p,
                       uint8_t* const* out_masks, float* const* out_cleans) {
  for (int t = 0; t < P.n; ++t) {
    const int i = P.order[t];
    FrameDev f = make_frame(imgs[i], P.hs[i], P.ws[i], p[i], out_masks[i], out_cleans[i],
                            P.ws_dev + P.ws_off[t], P.lay[t], P.cfg);
    unsigned long long* ctr = P.counters_dev + counter_stride(P.niter) * (size_t)t;
    f.n_new = ctr;
    f.status = reinterpret_cast<int*>(ctr + P.niter + 1);
    f.counts = reinterpret_cast<unsigned int*>(ctr + P.niter + 2);
    P.frames_pin[t] = f;
  }
}

// The whole run of a plan on stream s: one reset kernel for every frame and
// cursor, then each group's chain -- per iteration the passes that iteration
// runs, in kPass* order -- on its own stream (forked from s and joined back).
// The groups' first A1 launches run one after another (group g + 1's waits
// for group g's): A1 fills the chip by itself, and group g's later passes,
// which are latency-bound, then overlap the following groups' A1 instead of
// all starting together after every A1.
// With marks (eager launches only, never inside a capture) the groups run one
// after another on s with timing events before each group's first pass and
// after each of its pass slots.
static hipError_t enqueue_plan(BatchPlan& P, hipStream_t s, bool marks) {
  const int niter = P.niter, G = P.ngroups;
  QueueArgs all{P.frames_dev, P.tile_base_dev, P.tile_base_dev, P.n, P.cursors_dev, 0, 0};
  hipError_t e = launch_queue_init(all, P.ncur() * G, 1, s);
  const bool split = !marks && G > 1;
  if (e == hipSuccess && split) {
    e = hipEventRecord(P.fork[0], s);
    for (int g = 1; g < G && e == hipSuccess; ++g) e = hipStreamWaitEvent(P.gstream[g - 1], P.fork[0], 0);
  }
  const int per = kPassesPerIter * niter + 1;
  for (int g = 0; g < G && e == hipSuccess; ++g) {
    hipStream_t st = split && g > 0 ? P.gstream[g - 1] : s;
    const int ng = P.gstart[g + 1] - P.gstart[g];
    const int* tb = P.tile_base_dev + P.goff[g];
    QueueArgs a{P.frames_dev + P.gstart[g], tb, tb + (ng + 1), ng,
                P.cursors_dev + (size_t)P.ncur() * g, 0, 0};
    if (marks) e = hipEventRecord(P.marks[g * per], s);
    for (int it = 0; it < niter && e == hipSuccess; ++it) {
      for (int pass = 0; pass < kPassesPerIter && e == hipSuccess; ++pass) {
        if (pass_runs(pass, it, niter, P.est != 0)) {
          const int slot = dense_slot(pass);
          a.cursor_slot = it * kDenseSlots + (slot < 0 ? 0 : slot);
          if (pass == kPassGain)
            a.blocks = P.gain_nbx[g];
          else if (slot < 0)
            a.blocks = 0;
          else if (P.mode == kModeGrid)
            a.blocks = pass == kPassA1 ? P.total_a[g] : P.total_b[g];
          else
            a.blocks = P.blocks[slot];
          const bool chain = split && pass == kPassA1 && it == 0;
          if (chain && g > 0) e = hipStreamWaitEvent(st, P.a1_done[g - 1], 0);
          if (e == hipSuccess) e = launch_queue_pass(a, pass, it, P.cfg, P.mode, st);
          if (e == hipSuccess && chain && g + 1 < G) e = hipEventRecord(P.a1_done[g], st);
        }
        if (e == hipSuccess && marks)
          e = hipEventRecord(P.marks[g * per + 1 + kPassesPerIter * it + pass], s);
      }
    }
  }
  if (split)
    for (int g = 1; g < G && e == hipSuccess; ++g) {
      e = hipEventRecord(P.join[g - 1], P.gstream[g - 1]);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, P.join[g - 1], 0);
    }
  return e;
}

// Frame groups: at most `want` (and at most n), each frame to the group with
// the fewest pixels so far, largest frames first; table order is group by
// group, frames of a group in the caller's order.
static void make_groups(BatchPlan& P, int want) {
  const int n = P.n;
  const int G = std::max(1, std::min(want, n));
  std::vector<int> by_size(n);
  for (int i = 0; i < n; ++i) by_size[i] = i;
  std::stable_sort(by_size.begin(), by_size.end(), [&](int a, int b) {
    return P.hs[a] * P.ws[a] > P.hs[b] * P.ws[b];
  });
  std::vector<int64_t> load(G, 0);
  std::vector<int> grp(n, 0);
  for (int i : by_size) {
    const int g = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    grp[i] = g;
    load[g] += P.hs[i] * P.ws[i];
  }
  P.order.clear();
  P.gstart.assign(1, 0);
  for (int g = 0; g < G; ++g) {
    for (int i = 0; i < n; ++i)
      if (grp[i] == g) P.order.push_back(i);
    P.gstart.push_back((int)P.order.size());
  }
  P.ngroups = G;
}

// Group counts the autotuner tries; LACOSMIC_BATCH_GROUPS (1 .. 8) pins one.
constexpr int kGroupChoices[] = {1, 4};
constexpr int kNumGroupChoices = 2;
constexpr int kDefaultGroups = 4;
static int pinned_groups() {
  if (const char* env = std::getenv("LACOSMIC_BATCH_GROUPS")) {
    const int g = std::atoi(env);
    if (g >= 1 && g <= 8) return g;
  }
  return 0;
}

static int build_plan(BatchPlan& P, int n, const int64_t* hs, const int64_t* ws, int niter,
                      int early, int est, int cfg, int mode, int groups, hipStream_t cap) {
  P.n = n;
  P.niter = niter;
  P.early = early;
  P.est = est;
  P.cfg = cfg;
  P.mode = mode;
  P.hs.assign(hs, hs + n);
  P.ws.assign(ws, ws + n);
  make_groups(P, groups);
  const int G = P.ngroups;
  P.lay.resize(n);
  P.ws_off.resize(n);
  size_t total = 0;
  const TileShape ts = tile_shape(cfg);
  std::vector<int> base;  // per group: pass-A tile bases, then pass-B tile bases
  P.goff.clear();
  P.total_a.assign(G, 0);
  P.total_b.assign(G, 0);
  P.gain_nbx.assign(G, 1);
  for (int g = 0; g < G; ++g) {
    const int t0 = P.gstart[g], ng = P.gstart[g + 1] - t0;
    const size_t o = base.size();
    P.goff.push_back((int)o);
    base.resize(o + 2 * (ng + 1), 0);
    for (int k = 0; k < ng; ++k) {
      const int t = t0 + k, i = P.order[t];
      P.lay[t] = ws_layout(hs[i], ws[i]);
      P.ws_off[t] = total;
      total += P.lay[t].total;
      const int64_t tiles = ((ws[i] + ts.tw - 1) / ts.tw) * ((hs[i] + ts.th - 1) / ts.th);
      const int64_t band = (int64_t)kBStrip * kBWaves;
      const int64_t tiles_b =
          ((hs[i] + band - 1) / band) * strip_ncols((int)((ws[i] + 63) / 64));
      if ((int64_t)base[o + k] + tiles > 0x7fffffff ||
          (int64_t)base[o + ng + 1 + k] + tiles_b > 0x7fffffff)
        return LACOSMIC_EINVAL;
      base[o + k + 1] = base[o + k] + (int)tiles;
      base[o + ng + 1 + k + 1] = base[o + ng + 1 + k] + (int)tiles_b;
    }
    P.total_a[g] = base[o + ng];
    P.total_b[g] = base[o + 2 * ng + 1];
    int64_t biggest = 1;
    for (int k = 0; k < ng; ++k) {
      const int i = P.order[t0 + k];
      biggest = std::max<int64_t>(biggest, hs[i] * ws[i]);
    }
    P.gain_nbx[g] = gain_blocks(biggest);
  }
  const int ncur = P.ncur() * G;
  if (hipMalloc(&P.ws_dev, total) != hipSuccess ||
      hipMalloc(&P.frames_dev, sizeof(FrameDev) * n) != hipSuccess ||
      hipMalloc(&P.tile_base_dev, sizeof(int) * base.size()) != hipSuccess ||
      hipMalloc(&P.cursors_dev, sizeof(unsigned int) * ncur) != hipSuccess ||
      hipMalloc(&P.counters_dev, sizeof(unsigned long long) * counter_stride(niter) * n) !=
          hipSuccess ||
      hipHostMalloc(&P.frames_pin, sizeof(FrameDev) * n, hipHostMallocDefault) != hipSuccess)
    return LACOSMIC_ENOMEM;
  if (hipEventCreateWithFlags(&P.table_done, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&P.run_done, hipEventDisableTiming) != hipSuccess)
    return LACOSMIC_EHIP;
  if (hipMemcpy(P.tile_base_dev, base.data(), sizeof(int) * base.size(),
                hipMemcpyHostToDevice) != hipSuccess)
    return LACOSMIC_EHIP;
  for (int pass : {kPassA1, kPassSC, kPassB, kPassOut}) P.blocks[dense_slot(pass)] = queue_blocks(cfg, pass);
  P.marks.resize((size_t)G * (kPassesPerIter * niter + 1), nullptr);
  for (auto& ev : P.marks)
    if (hipEventCreate(&ev) != hipSuccess) return LACOSMIC_EHIP;
  P.gstream.resize(G - 1, nullptr);
  P.fork.resize(1, nullptr);
  P.join.resize(G - 1, nullptr);
  P.a1_done.resize(G - 1, nullptr);
  for (auto& st : P.gstream)
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) return LACOSMIC_EHIP;
  for (auto* v : {&P.fork, &P.join, &P.a1_done})
    for (auto& ev : *v)
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return LACOSMIC_EHIP;

  // Record the whole run once: counter/cursor reset, then the passes of each
  // iteration.  Only kernel nodes: the cursors are cleared by a kernel, never
  // by a memset node.
  hipGraph_t g = nullptr;
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess)
    return LACOSMIC_EHIP;
  const hipError_t e = enqueue_plan(P, cap, false);
  const hipError_t e2 = hipStreamEndCapture(cap, &g);
  if (e != hipSuccess || e2 != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return LACOSMIC_EHIP;
  }
  const hipError_t e3 = hipGraphInstantiate(&P.exec, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  return e3 == hipSuccess ? LACOSMIC_OK : LACOSMIC_EHIP;
}

static int launch_plan(BatchPlan& P, const float* const* imgs, const lacosmic_params* p,
                       uint8_t* const* out_masks, float* const* out_cleans, hipStream_t s) {
  // the previous upload from the staging table must have been consumed, and
  // the previous run (perhaps on another stream) must be over before the new
  // table and the shared workspaces are touched
  if (hipEventSynchronize(P.table_done) != hipSuccess) return LACOSMIC_EHIP;
  fill_table(P, imgs, p, out_masks, out_cleans);
  if (hipStreamWaitEvent(s, P.run_done, 0) != hipSuccess ||
      hipMemcpyAsync(P.frames_dev, P.frames_pin, sizeof(FrameDev) * P.n, hipMemcpyHostToDevice,
                     s) != hipSuccess ||
      hipEventRecord(P.table_done, s) != hipSuccess || hipGraphLaunch(P.exec, s) != hipSuccess ||
      hipEventRecord(P.run_done, s) != hipSuccess)
    return LACOSMIC_EHIP;
  return LACOSMIC_OK;
}

static int batch_status(DevCtx* c, BatchPlan& P, hipStream_t s) {
  const size_t bytes = sizeof(unsigned long long) * counter_stride(P.niter) * P.n;
  if (bytes > kPinnedBytes) {
    // large batches: read the status words one by one
    int bad = 0;
    for (int i = 0; i < P.n; ++i) {
      int st = 0;
      if (hipMemcpyAsync(&st, P.counters_dev + counter_stride(P.niter) * i + P.niter + 1,
                         sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
          hipStreamSynchronize(s) != hipSuccess)
        return LACOSMIC_EHIP;
      bad |= st & 1;
    }
    return bad ? LACOSMIC_ENONFINITE : LACOSMIC_OK;
  }
  if (hipMemcpyAsync(c->pinned, P.counters_dev, bytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return LACOSMIC_EHIP;
  const unsigned long long* ctr = static_cast<const unsigned long long*>(c->pinned);
  for (int i = 0; i < P.n; ++i) {
    int st = 0;
    std::memcpy(&st, ctr + counter_stride(P.niter) * i + P.niter + 1, sizeof(int));
    if (st & 1) return LACOSMIC_ENONFINITE;
  }
  return LACOSMIC_OK;
}

// Candidate tile shapes, launch forms (persistent queue, one block per tile)
// and frame-group counts timed on the caller's batch (each run also produces
// valid outputs); the fastest plan is kept.  LACOSMIC_AUTOTUNE=0 skips the
// timing and uses the single-frame path's tile shape with the persistent
// queue; LACOSMIC_BATCH_PLAN="cfg,mode[,groups]" skips it and uses that plan;
// LACOSMIC_BATCH_GROUPS pins the group count.
static int autotune(DevCtx* c, int n, const float* const* imgs, const int64_t* hs,
                    const int64_t* ws, const lacosmic_params* p, uint8_t* const* out_masks,
                    float* const* out_cleans, int niter, int early, int est, hipStream_t s,
                    BatchPlan** best) {
  *best = nullptr;
  const char* env = std::getenv("LACOSMIC_AUTOTUNE");
  bool tune = !(env && env[0] == '0');
  // LACOSMIC_BATCH_PLAN="cfg,mode[,groups]" pins the plan (profiling runs)
  int pin_cfg = -1, pin_mode = -1, pin_groups = pinned_groups();
  if (const char* pin = std::getenv("LACOSMIC_BATCH_PLAN")) {
    int g = 0;
    const int got = std::sscanf(pin, "%d,%d,%d", &pin_cfg, &pin_mode, &g);
    if (got >= 2 && pin_cfg >= 0 && pin_cfg < kNumTileCfgs &&
        (pin_mode == kModeQueue || pin_mode == kModeGrid) && (got == 2 || (g >= 1 && g <= 8))) {
      tune = false;
      if (got == 3) pin_groups = g;
    } else {
      pin_cfg = pin_mode = -1;
    }
  }
  std::vector<int> group_choices;
  if (pin_groups > 0)
    group_choices.push_back(pin_groups);
  else if (!tune)
    group_choices.push_back(kDefaultGroups);
  else
    group_choices.assign(kGroupChoices, kGroupChoices + kNumGroupChoices);
  std::vector<int> tried;  // group counts after capping at n, per cfg/mode
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
    return LACOSMIC_EHIP;
  float best_ms = 1e30f;
  int rc = LACOSMIC_OK;
  const int ncand = 2 * kNumTileCfgs * (int)group_choices.size();
  for (int cand = 0; cand < ncand && rc == LACOSMIC_OK; ++cand) {
    const int cfg = (cand >> 1) % kNumTileCfgs, mode = cand & 1;
    const int groups = std::min(n, group_choices[cand / (2 * kNumTileCfgs)]);
    if (!tune && pin_cfg >= 0 && (cfg != pin_cfg || mode != pin_mode)) continue;
    if (!tune && pin_cfg < 0 && (cfg != c->cfg || mode != kModeQueue)) continue;
    const int key = (groups << 8) | (cfg << 1) | mode;
    if (std::find(tried.begin(), tried.end(), key) != tried.end()) continue;
    tried.push_back(key);
    BatchPlan* P = new BatchPlan();
    rc = build_plan(*P, n, hs, ws, niter, early, est, cfg, mode, groups, c->stream);
    // rep 0 warms up; the plan's time is the best of the next three runs (an
    // untimed plan counts as 0 and is kept)
    float ms = tune ? 1e29f : 0.0f;
    for (int rep = 0; rep < (tune ? 4 : 0) && rc == LACOSMIC_OK; ++rep) {
      float t = 0.0f;
      if (hipEventRecord(t0, s) != hipSuccess) rc = LACOSMIC_EHIP;
      if (!rc) rc = launch_plan(*P, imgs, p, out_masks, out_cleans, s);
      if (!rc && (hipEventRecord(t1, s) != hipSuccess || hipEventSynchronize(t1) != hipSuccess ||
                  hipEventElapsedTime(&t, t0, t1) != hipSuccess))
        rc = LACOSMIC_EHIP;
      if (!rc && rep > 0 && t < ms) ms = t;
    }
    if (rc == LACOSMIC_OK && ms < best_ms) {
      best_ms = ms;
      if (*best) {
        (void)hipStreamSynchronize(s);
        delete *best;
      }
      *best = P;
    } else {
      (void)hipStreamSynchronize(s);
      delete P;
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (rc && *best) {
    delete *best;
    *best = nullptr;
  }
  return rc;
}

}  // namespace lac

using namespace lac;

extern "C" int lacosmic_run_batch(int32_t n, const float* const* imgs, const int64_t* hs,
                                  const int64_t* ws, const lacosmic_params* p,
                                  uint8_t* const* out_masks, float* const* out_cleans,
                                  void* hip_stream) {
  return guarded([&]() -> int {
    if (n < 0) return LACOSMIC_EINVAL;
    if (n == 0) return LACOSMIC_OK;
    if (!imgs || !hs || !ws || !p || !out_masks || !out_cleans) return LACOSMIC_EINVAL;
    // the iteration count and early stop are the batch's; the input type and
    // a missing gain are per frame
    constexpr uint32_t kShared = LACOSMIC_F_EARLY_STOP | LACOSMIC_F_FULL_SP;
    int est = 0;
    for (int i = 0; i < n; ++i) {
      int rc = check_params(hs[i], ws[i], &p[i]);
      if (rc) return rc;
      if (p[i].niter != p[0].niter || (p[i].flags & kShared) != (p[0].flags & kShared))
        return LACOSMIC_EINVAL;
      rc = check_buffers(imgs[i], hs[i], ws[i], out_masks[i], out_cleans[i], input_bytes(p[i]));
      if (rc) return rc;
      if (p[i].flags & LACOSMIC_F_ESTIMATE_GAIN) est = 1;
    }
    // outputs of one frame must not overlap any buffer of another
    for (int i = 0; i < n; ++i) {
      const size_t ni = (size_t)hs[i] * (size_t)ws[i];
      const uintptr_t oc = (uintptr_t)out_cleans[i], om = (uintptr_t)out_masks[i];
      for (int j = 0; j < n; ++j) {
        if (j == i) continue;
        const size_t nj = (size_t)hs[j] * (size_t)ws[j];
        const uintptr_t ranges[3][2] = {{(uintptr_t)imgs[j], (size_t)input_bytes(p[j]) * nj},
                                        {(uintptr_t)out_cleans[j], 4 * nj},
                                        {(uintptr_t)out_masks[j], nj}};
        for (auto& r : ranges) {
          if ((oc < r[0] + r[1] && r[0] < oc + 4 * ni) || (om < r[0] + r[1] && r[0] < om + ni))
            return LACOSMIC_EALIAS;
        }
      }
    }
    const int niter = p[0].niter;
    const int early = (p[0].flags & LACOSMIC_F_EARLY_STOP) ? 1 : 0;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LACOSMIC_EHIP;
    DevCtx* c = ctx_for(dev);
    if (!c) return LACOSMIC_EHIP;
    std::lock_guard<std::mutex> lk(c->mu);
    hipStream_t s = hip_stream ? static_cast<hipStream_t>(hip_stream) : c->stream_after_null();
    if (!s) return LACOSMIC_EHIP;
    if (!c->batch) c->batch = new BatchCache();
    BatchCache* B = c->batch;

    if (!B->plan || !B->plan->same(n, hs, ws, niter, early, est)) {
      const std::vector<int64_t> key = shape_key(n, hs, ws, niter, early, est);
      int cfg = -1;
      for (auto& kv : B->tuned)
        if (kv.first == key) cfg = kv.second;
      if (B->plan) {
        // its graph may still run on another stream
        if (hipDeviceSynchronize() != hipSuccess) return LACOSMIC_EHIP;
        delete B->plan;
        B->plan = nullptr;
      }
      BatchPlan* P = nullptr;
      if (cfg < 0) {
        const int rc =
            autotune(c, n, imgs, hs, ws, p, out_masks, out_cleans, niter, early, est, s, &P);
        if (rc) return rc;
        B->tuned.emplace_back(key, (P->ngroups << 8) | (P->cfg << 1) | P->mode);
      } else {
        P = new BatchPlan();
        const int rc = build_plan(*P, n, hs, ws, niter, early, est, (cfg >> 1) & 127, cfg & 1,
                                  cfg >> 8, c->stream);
        if (rc) {
          delete P;
          return rc;
        }
      }
      B->plan = P;
    }
    int rc = launch_plan(*B->plan, imgs, p, out_masks, out_cleans, s);
    if (rc) return rc;
    if (!hip_stream) return batch_status(c, *B->plan, s);
    return LACOSMIC_OK;
  });
}

// Durations (ms) of the passes of the most recent batch plan on the current
// device, kPassesPerIter per iteration in launch order: the plan's kernels
// replayed once, eagerly, over the buffers of the last call, with events
// between them.  Returns the number of values written, or a negative status.
extern "C" int lacosmic_batch_pass_ms(float* ms, int32_t n, void* hip_stream) {
  return guarded([&]() -> int {
    if (!ms || n < 0) return LACOSMIC_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LACOSMIC_EHIP;
    DevCtx* c = ctx_for(dev);
    if (!c) return LACOSMIC_EHIP;
    std::lock_guard<std::mutex> lk(c->mu);
    if (!c->batch || !c->batch->plan) return 0;
    BatchPlan& P = *c->batch->plan;
    hipStream_t s = hip_stream ? static_cast<hipStream_t>(hip_stream) : c->stream_after_null();
    if (!s || hipStreamWaitEvent(s, P.run_done, 0) != hipSuccess ||
        enqueue_plan(P, s, true) != hipSuccess || hipEventRecord(P.run_done, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return LACOSMIC_EHIP;
    // each pass slot summed over the groups (which the replay runs in turn)
    const int per = kPassesPerIter * P.niter + 1;
    const int k = std::min<int>(n, per - 1);
    for (int i = 0; i < k; ++i) {
      ms[i] = 0.0f;
      for (int g = 0; g < P.ngroups; ++g) {
        float t = 0.0f;
        if (hipEventElapsedTime(&t, P.marks[g * per + i], P.marks[g * per + i + 1]) != hipSuccess)
          return LACOSMIC_EHIP;
        ms[i] += t;
      }
    }
    return k;
  });
}

// Tile shape the batched path chose for the most recent batch shape on the
// current device (-1 if none yet).
extern "C" int lacosmic_batch_tile_shape(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  DevCtx* c = ctx_for(dev);
  if (!c) return -1;
  std::lock_guard<std::mutex> lk(c->mu);
  return (c->batch && c->batch->plan) ? c->batch->plan->cfg : -1;
}

// Frame groups of the most recent batch plan on the current device (-1 if
// none yet).
extern "C" int lacosmic_batch_groups(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  DevCtx* c = ctx_for(dev);
  if (!c) return -1;
  std::lock_guard<std::mutex> lk(c->mu);
  return (c->batch && c->batch->plan) ? c->batch->plan->ngroups : -1;
}

// Launch form the batched path chose for the most recent batch shape on the
// current device: 0 = persistent tile queue, 1 = one block per tile; -1 if
// none yet.
extern "C" int lacosmic_batch_launch_mode(void) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  DevCtx* c = ctx_for(dev);
  if (!c) return -1;
  std::lock_guard<std::mutex> lk(c->mu);
  return (c->batch && c->batch->plan) ? c->batch->plan->mode : -1;
}
