// Host runtime internals shared by the library's translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <mutex>
#include <new>

#include "lacosmic.h"
#include "lacosmic_device.h"
#include "lacosmic_launch.h"

namespace lac {

constexpr int kMaxIter = 1024;
constexpr int64_t kMaxDim = int64_t(1) << 24;
constexpr int64_t kMaxPixels = 2147483647;  // pixel indices are 32-bit
constexpr size_t kPinnedBytes = 64 * 1024;
constexpr uint32_t kKnownFlags = LACOSMIC_F_EARLY_STOP | LACOSMIC_F_FULL_SP |
                                 LACOSMIC_F_INPUT_U16 | LACOSMIC_F_ESTIMATE_GAIN |
                                 LACOSMIC_F_SEPMED;

struct WsLayout {
  size_t rec, counters, status, counts, gw, coef, stamps, nstamps, list, conf, splane, sp, g1, g2,
      b1, cb, m0, m1, dirty, rs, r4, wpr, total;
};

size_t align256(size_t v);

// Runs the body of a C entry point so that no C++ exception crosses the C ABI:
// an allocation failure reads LACOSMIC_ENOMEM, anything else LACOSMIC_EHIP.
template <typename F>
int guarded(F&& body) noexcept {
  try {
    return body();
  } catch (const std::bad_alloc&) {
    return LACOSMIC_ENOMEM;
  } catch (...) {
    return LACOSMIC_EHIP;
  }
}
WsLayout ws_layout(int64_t h, int64_t w);
int check_params(int64_t h, int64_t w, const lacosmic_params* p);
// in_bytes: bytes per input pixel (4, or 2 for uint16 input)
int check_buffers(const float* img, int64_t h, int64_t w, const uint8_t* out_mask,
                  const float* out_clean, int in_bytes = 4);
inline int input_bytes(const lacosmic_params& p) {
  return (p.flags & LACOSMIC_F_INPUT_U16) ? 2 : 4;
}
void set_tiles(FrameDev& f, int cfg);
FrameDev make_frame(const float* img, int64_t h, int64_t w, const lacosmic_params& p,
                    uint8_t* out_mask, float* out_clean, char* ws, const WsLayout& L, int cfg);

struct BatchCache;

// Frames of at most this many pixels run one fused launch per iteration on
// the single-frame path (LACOSMIC_FUSED_MAX_PX overrides; 0 turns it off);
// frames with the full-S' flag never do.
constexpr int64_t kFusedMaxPx = int64_t(1) << 19;  // measured crossover between 512^2 and 1024^2
int64_t fused_max_px();
// Whether a single-frame run of this frame takes the fused launches.
inline bool use_fused(int64_t h, int64_t w, const lacosmic_params& p) {
  return !(p.flags & LACOSMIC_F_FULL_SP) && h * w <= fused_max_px();
}

// A recorded single-frame run (counter reset and every iteration's launches)
// for one workspace address, frame shape, tile shape, iteration count and
// full-S' choice: the kernels read the frame record from the workspace, so
// the graph serves any input, outputs and parameters of that key.
struct FrameGraph {
  const void* ws = nullptr;
  int64_t h = 0, w = 0;
  int cfg = 0, niter = 0, full_sp = 0, est_gain = 0, fused = 0;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;  // the last launch of exec finished
  uint64_t used = 0;          // last use, for eviction
};
constexpr int kMaxFrameGraphs = 8;

// Per-device state, guarded by mu.
struct DevCtx {
  std::mutex mu;
  int dev = 0;
  int cfg = 0;                    // tile shape of the single-frame path
  hipStream_t stream = nullptr;   // library stream (default priority)
  void* ws = nullptr;             // cached single-frame workspace
  size_t ws_bytes = 0;
  hipEvent_t ws_done = nullptr;   // last enqueued use of ws
  hipEvent_t null_done = nullptr; // the legacy null stream's work so far (calls with no stream)
  void* pinned = nullptr;         // pinned staging for counters
  BatchCache* batch = nullptr;    // batched path: buffers and recorded graph
  FrameGraph graphs[kMaxFrameGraphs];  // single-frame path: recorded runs
  uint64_t graph_clock = 0;
  int use_graphs = 0;             // LACOSMIC_FRAME_GRAPH=1: replay recorded graphs instead
  int ensure_ws(size_t need);
  void release_extras();
  void release_graphs();
  // The recorded run for frame f (record at fd) with workspace ws: found, or
  // captured on the library stream and instantiated (evicting the least
  // recently used one).  nullptr on a runtime error.
  FrameGraph* frame_graph(const FrameDev& f, const FrameDev* fd, const void* ws, size_t nstamps,
                          int cfg);
  // The library stream, ordered after the work already enqueued on the
  // legacy null stream (which a caller with no stream of its own -- torch's
  // default stream, for one -- has used to produce the inputs and to free the
  // output buffers' previous contents); nullptr on a runtime error.
  hipStream_t stream_after_null();
};

DevCtx* ctx_for(int dev);
void shutdown_all();
int finish_sync(DevCtx* c, hipStream_t s, const FrameDev& f, lacosmic_stats* st);
// Host bytes finish_with reads back through: niter + 1 counters, the status
// word and 16 noise constants.
constexpr size_t kStatsHostBytes = 8 * (kMaxIter + 1) + 256 + 16 * sizeof(NoiseCoef) + 256;
static_assert(kStatsHostBytes <= kPinnedBytes, "the context's pinned buffer holds the stats");
int finish_with(char* host, hipStream_t s, const FrameDev& f, lacosmic_stats* st);

}  // namespace lac
