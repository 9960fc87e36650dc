// lacosmic_run_noalloc: the single-frame run for callers that cannot
// allocate (code under HIP graph capture, tight serving loops, harnesses
// that forbid allocation).  The frame's workspace is a static device array
// of kScratchBytes in this file; the call allocates nothing -- no device
// memory, no pinned staging, no library context, no recorded graph -- and
// launches the single-frame kernels eagerly on the caller's stream.
//
// Each device holds its own copy of the array.  Its address is resolved once
// per device, with that device current, on the first call there; host code
// never passes the array's name to a kernel (on the host it is only a
// stand-in), only the resolved address.  Every call on a device shares that
// device's array and leaves its contents behind: the launches clear what must
// start at zero (counters, list lengths, strip stamps, status; the per-
// iteration bit planes are rewritten by the passes that own them), so calls
// in sequence are independent, but calls that overlap on one device race.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>

#include "lacosmic.h"
#include "lacosmic_internal.h"

namespace lac {
namespace {

constexpr size_t kScratchBytes = size_t(128) << 20;
constexpr int kMaxDevices = 64;

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// The address of this device's copy of scratch (resolved on first use, with
// the device current); nullptr on a runtime error.
void* scratch_of(int dev) {
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
    g_scratch[dev] = ptr;
  }
  return g_scratch[dev];
}

}  // namespace
}  // namespace lac

using namespace lac;

extern "C" int lacosmic_run_noalloc(const float* img, int64_t h, int64_t w,
                                    const lacosmic_params* p, uint8_t* out_mask,
                                    float* out_clean, void* hip_stream, lacosmic_stats* st) {
  return guarded([&]() -> int {
    int rc = check_params(h, w, p);
    if (rc) return rc;
    rc = check_buffers(img, h, w, out_mask, out_clean, input_bytes(*p));
    if (rc) return rc;
    const WsLayout L = ws_layout(h, w);
    if (L.total > kScratchBytes) return LACOSMIC_ESCRATCH;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LACOSMIC_EHIP;
    if (dev < 0 || dev >= kMaxDevices) return LACOSMIC_EINVAL;
    char* ws = static_cast<char*>(scratch_of(dev));
    if (!ws) return LACOSMIC_EHIP;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);  // NULL: the legacy null stream
    FrameDev f = make_frame(img, h, w, *p, out_mask, out_clean, ws, L, kDefaultTileCfg);
    f.fused = use_fused(h, w, *p) ? 1 : 0;
    FrameDev* fd = reinterpret_cast<FrameDev*>(ws + L.rec);
    if (launch_put_frame(f, fd, s) != hipSuccess ||
        launch_init(f.n_new, f.niter, f.status, f.counts, f.b1s, (int64_t)L.nstamps, s) !=
            hipSuccess)
      return LACOSMIC_EHIP;
    for (int it = 0; it < f.niter; ++it)
      if (launch_iteration(f, fd, it, kDefaultTileCfg, s) != hipSuccess) return LACOSMIC_EHIP;
    if (hip_stream != nullptr && st == nullptr) return LACOSMIC_OK;
    alignas(256) char host[kStatsHostBytes];  // the read-back lands on this thread's stack
    return finish_with(host, s, f, st);
  });
}
