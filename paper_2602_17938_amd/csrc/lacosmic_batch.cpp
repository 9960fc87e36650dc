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
// them all back: for each frame, niter counters, then the status word (in an
// 8-byte slot) and kCntPerIter list lengths per iteration (4 bytes each).
static size_t counter_stride(int niter) {
  return (size_t)niter + 1 + ((size_t)kCntPerIter * niter + 1) / 2;
}

struct BatchPlan {
  // signature
  int n = 0, niter = 0, early = 0, cfg = 0, mode = kModeQueue;
  int total_a = 0, total_b = 0;  // tiles of all frames for passes A and B
  std::vector<int64_t> hs, ws;
  // device buffers
  char* ws_dev = nullptr;           // per-frame workspaces
  FrameDev* frames_dev = nullptr;   // frame table
  int* tile_base_dev = nullptr;     // pass-A tiles, then pass-B tiles (2 x (n + 1))
  unsigned int* cursors_dev = nullptr;
  unsigned long long* counters_dev = nullptr;
  std::vector<WsLayout> lay;
  std::vector<size_t> ws_off;
  FrameDev* frames_pin = nullptr;   // pinned staging of the frame table
  hipEvent_t table_done = nullptr;  // the last upload of frames_pin finished
  hipGraphExec_t exec = nullptr;
  int blocks[kDenseSlots] = {};  // persistent grid of each dense pass
  // timing events for an eager replay of the plan (lacosmic_batch_pass_ms):
  // marks[0] before the first pass, marks[k + 1] after pass k
  std::vector<hipEvent_t> marks;
  ~BatchPlan() {
    if (exec) (void)hipGraphExecDestroy(exec);
    for (hipEvent_t e : marks) (void)hipEventDestroy(e);
    if (table_done) (void)hipEventDestroy(table_done);
    if (frames_pin) (void)hipHostFree(frames_pin);
    if (ws_dev) (void)hipFree(ws_dev);
    if (frames_dev) (void)hipFree(frames_dev);
    if (tile_base_dev) (void)hipFree(tile_base_dev);
    if (cursors_dev) (void)hipFree(cursors_dev);
    if (counters_dev) (void)hipFree(counters_dev);
  }
  bool same(int n_, const int64_t* h_, const int64_t* w_, int niter_, int early_) const {
    if (n_ != n || niter_ != niter || early_ != early) return false;
    for (int i = 0; i < n; ++i)
      if (hs[i] != h_[i] || ws[i] != w_[i]) return false;
    return true;
  }
};

struct BatchCache {
  BatchPlan* plan = nullptr;  // the most recent batch shape
  std::vector<std::pair<std::vector<int64_t>, int>> tuned;  // shape key -> cfg * 2 + mode
};

void DevCtx::release_extras() {
  if (batch) {
    delete batch->plan;
    delete batch;
    batch = nullptr;
  }
}

static std::vector<int64_t> shape_key(int n, const int64_t* hs, const int64_t* ws, int niter,
                                      int early) {
  std::vector<int64_t> k;
  k.reserve(2 * n + 2);
  k.push_back(niter);
  k.push_back(early);
  for (int i = 0; i < n; ++i) {
    k.push_back(hs[i]);
    k.push_back(ws[i]);
  }
  return k;
}

// Fill the pinned frame table for this call's buffers and parameters.
static void fill_table(BatchPlan& P, const float* const* imgs, const lacosmic_params* p,
                       uint8_t* const* out_masks, float* const* out_cleans) {
  for (int i = 0; i < P.n; ++i) {
    FrameDev f = make_frame(imgs[i], P.hs[i], P.ws[i], p[i], out_masks[i], out_cleans[i],
                            P.ws_dev + P.ws_off[i], P.lay[i], P.cfg, kBStripMulti);
    unsigned long long* ctr = P.counters_dev + counter_stride(P.niter) * (size_t)i;
    f.n_new = ctr;
    f.status = reinterpret_cast<int*>(ctr + P.niter);
    f.counts = reinterpret_cast<unsigned int*>(ctr + P.niter + 1);
    P.frames_pin[i] = f;
  }
}

// The whole run of a plan on stream s: reset kernel, then per iteration the
// passes that iteration runs, in kPass* order.  With marks, a timing event is
// recorded before the first pass and after each pass slot (eager launches
// only, never inside a capture).
static hipError_t enqueue_plan(BatchPlan& P, hipStream_t s, bool marks) {
  const int n = P.n, niter = P.niter;
  QueueArgs a{P.frames_dev, P.tile_base_dev, P.tile_base_dev + (n + 1), n, P.cursors_dev, 0, 0};
  hipError_t e = launch_queue_init(a, 8 * kDenseSlots * niter, 1, s);
  if (e == hipSuccess && marks) e = hipEventRecord(P.marks[0], s);
  for (int it = 0; it < niter && e == hipSuccess; ++it) {
    for (int pass = 0; pass < kPassesPerIter && e == hipSuccess; ++pass) {
      if (pass_runs(pass, it, niter)) {
        const int slot = dense_slot(pass);
        a.cursor_slot = it * kDenseSlots + (slot < 0 ? 0 : slot);
        if (slot < 0)
          a.blocks = 0;
        else if (P.mode == kModeGrid)
          a.blocks = pass == kPassA1 ? P.total_a : P.total_b;
        else
          a.blocks = P.blocks[slot];
        e = launch_queue_pass(a, pass, it, P.cfg, P.mode, s);
      }
      if (e == hipSuccess && marks)
        e = hipEventRecord(P.marks[1 + kPassesPerIter * it + pass], s);
    }
  }
  return e;
}

static int build_plan(BatchPlan& P, int n, const int64_t* hs, const int64_t* ws, int niter,
                      int early, int cfg, int mode, hipStream_t cap) {
  P.n = n;
  P.niter = niter;
  P.early = early;
  P.cfg = cfg;
  P.mode = mode;
  P.hs.assign(hs, hs + n);
  P.ws.assign(ws, ws + n);
  P.lay.resize(n);
  P.ws_off.resize(n);
  size_t total = 0;
  std::vector<int> base(2 * (n + 1), 0);
  const TileShape ts = tile_shape(cfg);
  for (int i = 0; i < n; ++i) {
    P.lay[i] = ws_layout(hs[i], ws[i]);
    P.ws_off[i] = total;
    total += P.lay[i].total;
    const int64_t tiles = ((ws[i] + ts.tw - 1) / ts.tw) * ((hs[i] + ts.th - 1) / ts.th);
    const int64_t band = (int64_t)kBStripMulti * kBWaves;
    const int64_t tiles_b =
        ((hs[i] + band - 1) / band) * ((((ws[i] + 63) / 64) + kBWords - 1) / kBWords);
    if ((int64_t)base[i] + tiles > 0x7fffffff ||
        (int64_t)base[n + 1 + i] + tiles_b > 0x7fffffff)
      return LACOSMIC_EINVAL;
    base[i + 1] = base[i] + (int)tiles;
    base[n + 1 + i + 1] = base[n + 1 + i] + (int)tiles_b;
  }
  P.total_a = base[n];
  P.total_b = base[2 * n + 1];
  const int ncur = 8 * kDenseSlots * niter;
  if (hipMalloc(&P.ws_dev, total) != hipSuccess ||
      hipMalloc(&P.frames_dev, sizeof(FrameDev) * n) != hipSuccess ||
      hipMalloc(&P.tile_base_dev, sizeof(int) * 2 * (n + 1)) != hipSuccess ||
      hipMalloc(&P.cursors_dev, sizeof(unsigned int) * ncur) != hipSuccess ||
      hipMalloc(&P.counters_dev, sizeof(unsigned long long) * counter_stride(niter) * n) !=
          hipSuccess ||
      hipHostMalloc(&P.frames_pin, sizeof(FrameDev) * n, hipHostMallocDefault) != hipSuccess)
    return LACOSMIC_ENOMEM;
  if (hipEventCreateWithFlags(&P.table_done, hipEventDisableTiming) != hipSuccess)
    return LACOSMIC_EHIP;
  if (hipMemcpy(P.tile_base_dev, base.data(), sizeof(int) * 2 * (n + 1),
                hipMemcpyHostToDevice) != hipSuccess)
    return LACOSMIC_EHIP;
  for (int pass : {kPassA1, kPassSC, kPassB, kPassOut}) P.blocks[dense_slot(pass)] = queue_blocks(cfg, pass);
  P.marks.resize(kPassesPerIter * niter + 1, nullptr);
  for (auto& ev : P.marks)
    if (hipEventCreate(&ev) != hipSuccess) return LACOSMIC_EHIP;

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
  // the previous upload from the staging table must have been consumed
  if (hipEventSynchronize(P.table_done) != hipSuccess) return LACOSMIC_EHIP;
  fill_table(P, imgs, p, out_masks, out_cleans);
  if (hipMemcpyAsync(P.frames_dev, P.frames_pin, sizeof(FrameDev) * P.n, hipMemcpyHostToDevice,
                     s) != hipSuccess ||
      hipEventRecord(P.table_done, s) != hipSuccess || hipGraphLaunch(P.exec, s) != hipSuccess)
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
      if (hipMemcpyAsync(&st, P.counters_dev + counter_stride(P.niter) * i + P.niter,
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
    std::memcpy(&st, ctr + counter_stride(P.niter) * i + P.niter, sizeof(int));
    if (st & 1) return LACOSMIC_ENONFINITE;
  }
  return LACOSMIC_OK;
}

// Candidate tile shapes and launch forms (persistent queue, one block per
// tile) timed on the caller's batch (each run also produces valid outputs);
// the fastest plan is kept.  LACOSMIC_AUTOTUNE=0 skips the timing and uses
// the single-frame path's tile shape with the persistent queue;
// LACOSMIC_BATCH_PLAN="cfg,mode" skips it and uses that plan.
static int autotune(DevCtx* c, int n, const float* const* imgs, const int64_t* hs,
                    const int64_t* ws, const lacosmic_params* p, uint8_t* const* out_masks,
                    float* const* out_cleans, int niter, int early, hipStream_t s,
                    BatchPlan** best) {
  *best = nullptr;
  const char* env = std::getenv("LACOSMIC_AUTOTUNE");
  bool tune = !(env && env[0] == '0');
  // LACOSMIC_BATCH_PLAN="cfg,mode" pins the plan (profiling runs)
  int pin_cfg = -1, pin_mode = -1;
  if (const char* pin = std::getenv("LACOSMIC_BATCH_PLAN")) {
    if (std::sscanf(pin, "%d,%d", &pin_cfg, &pin_mode) == 2 && pin_cfg >= 0 &&
        pin_cfg < kNumTileCfgs && (pin_mode == kModeQueue || pin_mode == kModeGrid))
      tune = false;
    else
      pin_cfg = pin_mode = -1;
  }
  hipEvent_t t0 = nullptr, t1 = nullptr;
  if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess)
    return LACOSMIC_EHIP;
  float best_ms = 1e30f;
  int rc = LACOSMIC_OK;
  for (int cand = 0; cand < 2 * kNumTileCfgs && rc == LACOSMIC_OK; ++cand) {
    const int cfg = cand >> 1, mode = cand & 1;
    if (!tune && pin_cfg >= 0 && (cfg != pin_cfg || mode != pin_mode)) continue;
    if (!tune && pin_cfg < 0 && (cfg != c->cfg || mode != kModeQueue)) continue;
    BatchPlan* P = new BatchPlan();
    rc = build_plan(*P, n, hs, ws, niter, early, cfg, mode, c->stream);
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
  if (n < 0) return LACOSMIC_EINVAL;
  if (n == 0) return LACOSMIC_OK;
  if (!imgs || !hs || !ws || !p || !out_masks || !out_cleans) return LACOSMIC_EINVAL;
  for (int i = 0; i < n; ++i) {
    int rc = check_params(hs[i], ws[i], &p[i]);
    if (rc) return rc;
    if (p[i].niter != p[0].niter || p[i].flags != p[0].flags) return LACOSMIC_EINVAL;
    rc = check_buffers(imgs[i], hs[i], ws[i], out_masks[i], out_cleans[i]);
    if (rc) return rc;
  }
  // outputs of one frame must not overlap any buffer of another
  for (int i = 0; i < n; ++i) {
    const size_t ni = (size_t)hs[i] * (size_t)ws[i];
    const uintptr_t oc = (uintptr_t)out_cleans[i], om = (uintptr_t)out_masks[i];
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      const size_t nj = (size_t)hs[j] * (size_t)ws[j];
      const uintptr_t ranges[3][2] = {{(uintptr_t)imgs[j], 4 * nj},
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
  hipStream_t s = hip_stream ? static_cast<hipStream_t>(hip_stream) : c->stream;
  if (!c->batch) c->batch = new BatchCache();
  BatchCache* B = c->batch;

  if (!B->plan || !B->plan->same(n, hs, ws, niter, early)) {
    const std::vector<int64_t> key = shape_key(n, hs, ws, niter, early);
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
      const int rc = autotune(c, n, imgs, hs, ws, p, out_masks, out_cleans, niter, early, s, &P);
      if (rc) return rc;
      B->tuned.emplace_back(key, P->cfg * 2 + P->mode);
    } else {
      P = new BatchPlan();
      const int rc = build_plan(*P, n, hs, ws, niter, early, cfg >> 1, cfg & 1, c->stream);
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
}

// Durations (ms) of the passes of the most recent batch plan on the current
// device, in launch order (A1, A2, S1, B, S2 for each iteration): the plan's
// kernels are replayed once, eagerly, on hip_stream (NULL = the library
// stream) over the buffers of the last call, with events between them.
// Returns the number of values written, or a negative status.
extern "C" int lacosmic_batch_pass_ms(float* ms, int32_t n, void* hip_stream) {
  if (!ms || n < 0) return LACOSMIC_EINVAL;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return LACOSMIC_EHIP;
  DevCtx* c = ctx_for(dev);
  if (!c) return LACOSMIC_EHIP;
  std::lock_guard<std::mutex> lk(c->mu);
  if (!c->batch || !c->batch->plan) return 0;
  BatchPlan& P = *c->batch->plan;
  hipStream_t s = hip_stream ? static_cast<hipStream_t>(hip_stream) : c->stream;
  if (enqueue_plan(P, s, true) != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
    return LACOSMIC_EHIP;
  const int k = std::min<int>(n, (int)P.marks.size() - 1);
  for (int i = 0; i < k; ++i)
    if (hipEventElapsedTime(&ms[i], P.marks[i], P.marks[i + 1]) != hipSuccess)
      return LACOSMIC_EHIP;
  return k;
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
