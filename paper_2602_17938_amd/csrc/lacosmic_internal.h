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

struct WsLayout {
  size_t counters, status, counts, stamps, nstamps, list, conf, splane, sp, g1, g2, b1, cb, m0, m1,
      dirty, rs, r4, wpr, total;
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
int check_buffers(const float* img, int64_t h, int64_t w, const uint8_t* out_mask,
                  const float* out_clean);
void set_tiles(FrameDev& f, int cfg, int bstrip);
FrameDev make_frame(const float* img, int64_t h, int64_t w, const lacosmic_params& p,
                    uint8_t* out_mask, float* out_clean, char* ws, const WsLayout& L, int cfg,
                    int bstrip);

struct BatchCache;

// Per-device state, guarded by mu.
struct DevCtx {
  std::mutex mu;
  int dev = 0;
  int cfg = 0;                    // tile shape of the single-frame path
  hipStream_t stream = nullptr;   // library stream (default priority)
  void* ws = nullptr;             // cached single-frame workspace
  size_t ws_bytes = 0;
  hipEvent_t ws_done = nullptr;   // last enqueued use of ws
  void* pinned = nullptr;         // pinned staging for counters
  BatchCache* batch = nullptr;    // batched path: buffers and recorded graph
  int ensure_ws(size_t need);
  void release_extras();
};

DevCtx* ctx_for(int dev);
void shutdown_all();
int finish_sync(DevCtx* c, hipStream_t s, const FrameDev& f, lacosmic_stats* st);

}  // namespace lac
