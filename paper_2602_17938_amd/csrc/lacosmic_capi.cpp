// C ABI of liblacosmic.so: argument checks, per-device context (stream,
// cached workspace, pinned staging), and the single-frame driver.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>

#include "lacosmic.h"
#include "lacosmic_internal.h"

namespace lac {

size_t align256(size_t v) { return (v + 255) & ~size_t(255); }

WsLayout ws_layout(int64_t h, int64_t w) {
  WsLayout L{};
  const size_t n = (size_t)h * (size_t)w;
  const size_t wpr = (size_t)((w + 63) / 64);
  const size_t plane = (size_t)h * wpr * sizeof(uint64_t);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    const size_t o = off;
    off = align256(off + bytes);
    return o;
  };
  L.rec = take(sizeof(FrameDev));  // the frame record the single-frame kernels read
  L.counters = take(sizeof(unsigned long long) * (kMaxIter + 1));  // n_new[niter] + 1
  L.status = take(sizeof(int) * 4);
  L.counts = take(sizeof(unsigned int) * kCntPerIter * kMaxIter);
  L.gw = take(sizeof(GainWork));
  L.coef = take(sizeof(NoiseCoef) * kMaxIter);
  L.nstamps = 2 * (size_t)max_strips(h, w);  // b1s, then bq
  L.stamps = take(sizeof(int) * L.nstamps);
  L.list = take(n * sizeof(int));
  L.conf = take(n * sizeof(int));
  L.splane = take(n * sizeof(float));
  L.sp = take(n * sizeof(float));
  L.g1 = take(plane);
  L.g2 = take(plane);
  L.b1 = take(plane);
  L.cb = take(plane);
  L.m0 = take(plane);
  L.m1 = take(plane);
  L.dirty = take(plane);
  L.rs = take(plane);
  L.r4 = take(plane);
  L.wpr = wpr;
  L.total = off;
  return L;
}

static bool finite_pos(float v) { return std::isfinite(v) && v > 0.0f; }

int64_t fused_max_px() {
  if (const char* env = std::getenv("LACOSMIC_FUSED_MAX_PX")) return std::atoll(env);
  return kFusedMaxPx;
}

int check_params(int64_t h, int64_t w, const lacosmic_params* p) {
  if (!p) return LACOSMIC_EINVAL;
  if (h < 1 || w < 1 || h > kMaxDim || w > kMaxDim || h * w > kMaxPixels) return LACOSMIC_EINVAL;
  if (p->niter < 1 || p->niter > kMaxIter) return LACOSMIC_EINVAL;
  if ((p->flags & ~kKnownFlags) != 0) return LACOSMIC_EINVAL;
  // an estimated gain ignores the gain field, which must still be a finite value >= 0
  const bool est = (p->flags & LACOSMIC_F_ESTIMATE_GAIN) != 0;
  if (est ? !(std::isfinite(p->gain) && p->gain >= 0.0f) : !finite_pos(p->gain))
    return LACOSMIC_EINVAL;
  if (!finite_pos(p->sigclip) || !finite_pos(p->sigfrac)) return LACOSMIC_EINVAL;
  if (!std::isfinite(p->readnoise) || p->readnoise < 0.0f) return LACOSMIC_EINVAL;
  if (!std::isfinite(p->objlim) || p->objlim < 0.0f) return LACOSMIC_EINVAL;
  return LACOSMIC_OK;
}

static bool overlaps(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
  return pa < pb + nb && pb < pa + na;
}

int check_buffers(const float* img, int64_t h, int64_t w, const uint8_t* out_mask,
                  const float* out_clean, int in_bytes) {
  if (!img || !out_mask || !out_clean) return LACOSMIC_EINVAL;
  const size_t n = (size_t)h * (size_t)w;
  const size_t ni = (size_t)in_bytes * n;
  if (overlaps(img, ni, out_clean, 4 * n) || overlaps(img, ni, out_mask, n) ||
      overlaps(out_clean, 4 * n, out_mask, n))
    return LACOSMIC_EALIAS;
  return LACOSMIC_OK;
}

// 1 / g when g is a power of two whose reciprocal is a normal binary32 number
// (then the reciprocal, and x / g = x * (1 / g), are exact); 0 otherwise.
static float exact_reciprocal(float g) {
  int e = 0;
  const float m = std::frexp(g, &e);  // g = m * 2^e, m in [0.5, 1)
  if (!(g > 0.0f) || !std::isfinite(g) || m != 0.5f) return 0.0f;
  const float r = std::ldexp(1.0f, 1 - e);
  return (std::isnormal(r) && r * g == 1.0f) ? r : 0.0f;
}

FrameDev make_frame(const float* img, int64_t h, int64_t w, const lacosmic_params& p,
                    uint8_t* out_mask, float* out_clean, char* ws, const WsLayout& L, int cfg) {
  FrameDev f{};
  const bool u16 = (p.flags & LACOSMIC_F_INPUT_U16) != 0;
  f.img = u16 ? nullptr : img;
  f.img16 = u16 ? reinterpret_cast<const uint16_t*>(img) : nullptr;
  f.clean = out_clean;
  f.splane = reinterpret_cast<float*>(ws + L.splane);
  f.sp = reinterpret_cast<float*>(ws + L.sp);
  f.g1 = reinterpret_cast<uint64_t*>(ws + L.g1);
  f.g2 = reinterpret_cast<uint64_t*>(ws + L.g2);
  f.b1 = reinterpret_cast<uint64_t*>(ws + L.b1);
  f.cb = reinterpret_cast<uint64_t*>(ws + L.cb);
  f.mbits[0] = reinterpret_cast<uint64_t*>(ws + L.m0);
  f.mbits[1] = reinterpret_cast<uint64_t*>(ws + L.m1);
  f.out_mask = out_mask;
  f.n_new = reinterpret_cast<unsigned long long*>(ws + L.counters);
  f.status = reinterpret_cast<int*>(ws + L.status);
  f.counts = reinterpret_cast<unsigned int*>(ws + L.counts);
  f.list = reinterpret_cast<int*>(ws + L.list);
  f.conf = reinterpret_cast<int*>(ws + L.conf);
  f.b1s = reinterpret_cast<int*>(ws + L.stamps);
  f.bq = f.b1s + L.nstamps / 2;
  f.dirty = reinterpret_cast<uint64_t*>(ws + L.dirty);
  f.rs = reinterpret_cast<uint64_t*>(ws + L.rs);
  f.r4 = reinterpret_cast<uint64_t*>(ws + L.r4);
  f.gw = reinterpret_cast<GainWork*>(ws + L.gw);
  f.coef = reinterpret_cast<NoiseCoef*>(ws + L.coef);
  f.h = (int)h;
  f.w = (int)w;
  f.wpr = (int)L.wpr;
  {
    // Division of pixel indices by w as a multiply and a shift (Granlund and
    // Montgomery, 1994): with l = ceil(log2 w) and m = ceil(2^(31+l) / w),
    // 2^(31+l) <= m w < 2^(31+l) + 2^l, so (n m) >> (31 + l) == n / w for
    // every 0 <= n < 2^31, and m < 2^32.
    int l = 0;
    while ((int64_t(1) << l) < w) ++l;
    f.w_shr = 31 + l;
    f.w_mul = (unsigned int)(((uint64_t(1) << (31 + l)) + (uint64_t)w - 1) / (uint64_t)w);
  }
  f.gain = p.gain;
  f.readnoise = p.readnoise;
  f.est_gain = (p.flags & LACOSMIC_F_ESTIMATE_GAIN) ? 1 : 0;
  // Both derived constants are rounded to binary32 once, as products of
  // binary32 values.
  volatile float rn = p.readnoise;
  f.rn2 = rn * rn;
  volatile float sf = p.sigfrac;
  f.lo = sf * p.sigclip;
  f.inv_gain = exact_reciprocal(p.gain);
  {  // the variance at the floor, as the kernels round it: the smallest there is
    volatile float g = p.gain, floor_m = 1e-4f;
    volatile float gm = g * floor_m;
    volatile float vmin = gm + f.rn2;
    f.fast_sqrt = vmin >= 0x1p-96f ? 1 : 0;
  }
  f.sigclip = p.sigclip;
  f.objlim = p.objlim;
  f.niter = p.niter;
  f.early_stop = (p.flags & LACOSMIC_F_EARLY_STOP) ? 1 : 0;
  f.full_sp = (p.flags & LACOSMIC_F_FULL_SP) ? 1 : 0;
  f.sepmed = (p.flags & LACOSMIC_F_SEPMED) ? 1 : 0;
  set_tiles(f, cfg);
  f.it = 0;
  return f;
}

void set_tiles(FrameDev& f, int cfg) {
  const TileShape ts = tile_shape(cfg);
  f.tiles_x = (f.w + ts.tw - 1) / ts.tw;
  f.tiles = f.tiles_x * ((f.h + ts.th - 1) / ts.th);
  const int band = kBStrip * kBWaves;
  f.tiles_b = ((f.h + band - 1) / band) * strip_ncols(f.wpr);
}

// ------------------------------------------------------------ device context
static std::mutex g_mu;
static std::map<int, DevCtx*> g_ctx;

DevCtx* ctx_for(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_ctx.find(dev);
  if (it != g_ctx.end()) return it->second;
  // never throws: any failure releases what was created and returns null
  DevCtx* c = new (std::nothrow) DevCtx();
  if (!c) return nullptr;
  c->dev = dev;
  if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) == hipSuccess &&
      hipEventCreateWithFlags(&c->ws_done, hipEventDisableTiming) == hipSuccess &&
      hipEventCreateWithFlags(&c->null_done, hipEventDisableTiming) == hipSuccess &&
      hipHostMalloc(&c->pinned, kPinnedBytes, hipHostMallocDefault) == hipSuccess) {
    const char* cfg = std::getenv("LACOSMIC_TILE_CFG");
    c->cfg = cfg ? std::atoi(cfg) : kDefaultTileCfg;
    if (c->cfg < 0 || c->cfg >= kNumTileCfgs) c->cfg = kDefaultTileCfg;
    const char* gr = std::getenv("LACOSMIC_FRAME_GRAPH");
    c->use_graphs = (gr && gr[0] == '1') ? 1 : 0;
    try {
      g_ctx[dev] = c;
      return c;
    } catch (...) {
    }
  }
  if (c->pinned) (void)hipHostFree(c->pinned);
  if (c->null_done) (void)hipEventDestroy(c->null_done);
  if (c->ws_done) (void)hipEventDestroy(c->ws_done);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
  return nullptr;
}

hipStream_t DevCtx::stream_after_null() {
  if (hipEventRecord(null_done, nullptr) != hipSuccess ||
      hipStreamWaitEvent(stream, null_done, 0) != hipSuccess)
    return nullptr;
  return stream;
}

void DevCtx::release_graphs() {
  for (FrameGraph& g : graphs) {
    if (g.done) (void)hipEventSynchronize(g.done);
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.done) (void)hipEventDestroy(g.done);
    g = FrameGraph{};
  }
}

FrameGraph* DevCtx::frame_graph(const FrameDev& f, const FrameDev* fd, const void* wsp,
                                size_t nstamps, int tcfg) {
  FrameGraph* victim = &graphs[0];
  for (FrameGraph& g : graphs) {
    if (g.exec && g.ws == wsp && g.h == f.h && g.w == f.w && g.cfg == tcfg &&
        g.niter == f.niter && g.full_sp == f.full_sp && g.est_gain == f.est_gain &&
        g.fused == f.fused) {
      g.used = ++graph_clock;
      return &g;
    }
    if (!g.exec || (victim->exec && g.used < victim->used)) victim = &g;
  }
  if (victim->exec) {  // evict: wait for its last launch, then release it
    if (hipEventSynchronize(victim->done) != hipSuccess) return nullptr;
    (void)hipGraphExecDestroy(victim->exec);
    victim->exec = nullptr;
  }
  if (!victim->done && hipEventCreateWithFlags(&victim->done, hipEventDisableTiming) != hipSuccess) {
    victim->done = nullptr;
    return nullptr;
  }
  // record the counter reset and every iteration's launches (kernel nodes only)
  prime_launch_config();
  hipGraph_t graph = nullptr;
  if (hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal) != hipSuccess) return nullptr;
  hipError_t e = launch_init(f.n_new, f.niter, f.status, f.counts, f.b1s, (int64_t)nstamps, stream);
  for (int it = 0; it < f.niter && e == hipSuccess; ++it) e = launch_iteration(f, fd, it, tcfg, stream);
  const hipError_t e2 = hipStreamEndCapture(stream, &graph);
  if (e != hipSuccess || e2 != hipSuccess || !graph) {
    if (graph) (void)hipGraphDestroy(graph);
    return nullptr;
  }
  hipGraphExec_t exec = nullptr;
  const hipError_t e3 = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e3 != hipSuccess) return nullptr;
  victim->exec = exec;
  victim->ws = wsp;
  victim->h = f.h;
  victim->w = f.w;
  victim->cfg = tcfg;
  victim->niter = f.niter;
  victim->full_sp = f.full_sp;
  victim->est_gain = f.est_gain;
  victim->fused = f.fused;
  victim->used = ++graph_clock;
  return victim;
}

int DevCtx::ensure_ws(size_t need) {
  if (ws && ws_bytes >= need) return LACOSMIC_OK;
  if (ws) {
    if (hipEventSynchronize(ws_done) != hipSuccess) return LACOSMIC_EHIP;
    (void)hipFree(ws);
    ws = nullptr;
    ws_bytes = 0;
  }
  if (hipMalloc(&ws, need) != hipSuccess) {
    ws = nullptr;
    return LACOSMIC_ENOMEM;
  }
  ws_bytes = need;
  return LACOSMIC_OK;
}

void shutdown_all() {
  std::lock_guard<std::mutex> lk(g_mu);
  for (auto& kv : g_ctx) {
    DevCtx* c = kv.second;
    int prev = 0;
    (void)hipGetDevice(&prev);
    (void)hipSetDevice(c->dev);
    {
      std::lock_guard<std::mutex> lk2(c->mu);
      (void)hipStreamSynchronize(c->stream);
      c->release_extras();
      c->release_graphs();
      if (c->ws) (void)hipFree(c->ws);
      if (c->pinned) (void)hipHostFree(c->pinned);
      (void)hipEventDestroy(c->ws_done);
      (void)hipEventDestroy(c->null_done);
      (void)hipStreamDestroy(c->stream);
    }
    (void)hipSetDevice(prev);
    delete c;
  }
  g_ctx.clear();
}

// Read back counters and status after the stream's work through the host
// buffer pin (kStatsHostBytes); fill stats.
int finish_with(char* pin, hipStream_t s, const FrameDev& f, lacosmic_stats* st) {
  // the per-iteration counts and the unreplaced-pixel count after them, the
  // status word, and the noise constants of the first 16 estimated gains
  const size_t nbytes = sizeof(unsigned long long) * ((size_t)f.niter + 1);
  const int ncoef = f.niter < 16 ? f.niter : 16;
  const size_t coef_at = align256(nbytes + sizeof(int));
  if (hipMemcpyAsync(pin, f.n_new, nbytes, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(pin + nbytes, f.status, sizeof(int), hipMemcpyDeviceToHost, s) !=
          hipSuccess ||
      (f.est_gain && hipMemcpyAsync(pin + coef_at, f.coef, sizeof(NoiseCoef) * ncoef,
                                    hipMemcpyDeviceToHost, s) != hipSuccess) ||
      hipStreamSynchronize(s) != hipSuccess)
    return LACOSMIC_EHIP;
  const unsigned long long* nn = reinterpret_cast<const unsigned long long*>(pin);
  int status = 0;
  std::memcpy(&status, pin + nbytes, sizeof(int));
  if (st) {
    std::memset(st, 0, sizeof(*st));
    int run = f.niter;
    int64_t total = 0;
    for (int k = 0; k < f.niter; ++k) {
      total += (int64_t)nn[k];
      if (k < 16) st->n_new[k] = (int64_t)nn[k];
      if (f.early_stop && nn[k] == 0) {
        run = k + 1;
        break;
      }
    }
    st->iters_run = run;
    st->n_flagged = total;
    st->n_unreplaced = (int64_t)nn[f.niter];
    for (int k = 0; k < ncoef; ++k) {
      if (f.est_gain) {
        NoiseCoef nc;
        std::memcpy(&nc, pin + coef_at + sizeof(NoiseCoef) * k, sizeof(nc));
        st->gain[k] = k < run ? nc.gain : 0.0f;
        st->gain_estimated[k] = k < run ? (int8_t)(nc.valid ? 1 : -1) : (int8_t)0;
      } else {
        st->gain[k] = f.gain;
      }
    }
  }
  return (status & 1) ? LACOSMIC_ENONFINITE : LACOSMIC_OK;
}

int finish_sync(DevCtx* c, hipStream_t s, const FrameDev& f, lacosmic_stats* st) {
  return finish_with(static_cast<char*>(c->pinned), s, f, st);
}

}  // namespace lac

using namespace lac;

extern "C" {

size_t lacosmic_workspace_bytes(int64_t h, int64_t w) {
  if (h < 1 || w < 1 || h > kMaxDim || w > kMaxDim || h * w > kMaxPixels) return 0;
  return ws_layout(h, w).total;
}

int lacosmic_workspace_layout(int64_t h, int64_t w, lacosmic_ws_layout* out) {
  if (!out || h < 1 || w < 1 || h > kMaxDim || w > kMaxDim || h * w > kMaxPixels)
    return LACOSMIC_EINVAL;
  const WsLayout L = ws_layout(h, w);
  out->s_offset = L.splane;
  out->sp_offset = L.sp;
  out->cand_offset = L.b1;
  out->mask_bits_offset = L.m0;
  out->row_words = L.wpr;
  out->total_bytes = L.total;
  return LACOSMIC_OK;
}

int lacosmic_run_ex(const float* img, int64_t h, int64_t w, const lacosmic_params* p,
                    uint8_t* out_mask, float* out_clean, void* workspace, void* hip_stream,
                    lacosmic_stats* st) {
  return guarded([&]() -> int {
    int rc = check_params(h, w, p);
    if (rc) return rc;
    rc = check_buffers(img, h, w, out_mask, out_clean, input_bytes(*p));
    if (rc) return rc;
    const WsLayout L = ws_layout(h, w);
    if (workspace && ((uintptr_t)workspace & 255u)) return LACOSMIC_EINVAL;

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LACOSMIC_EHIP;
    DevCtx* c = ctx_for(dev);
    if (!c) return LACOSMIC_EHIP;
    std::lock_guard<std::mutex> lk(c->mu);
    hipStream_t s = hip_stream ? static_cast<hipStream_t>(hip_stream) : c->stream_after_null();
    if (!s) return LACOSMIC_EHIP;
    char* ws = static_cast<char*>(workspace);
    if (!ws) {
      rc = c->ensure_ws(L.total);
      if (rc) return rc;
      if (hipStreamWaitEvent(s, c->ws_done, 0) != hipSuccess) return LACOSMIC_EHIP;
      ws = static_cast<char*>(c->ws);
    }
    FrameDev f = make_frame(img, h, w, *p, out_mask, out_clean, ws, L, c->cfg);
    f.fused = use_fused(h, w, *p) ? 1 : 0;
    FrameDev* fd = reinterpret_cast<FrameDev*>(ws + L.rec);
    if (launch_put_frame(f, fd, s) != hipSuccess) return LACOSMIC_EHIP;
    if (c->use_graphs) {  // the recorded run for this workspace and shape
      FrameGraph* g = c->frame_graph(f, fd, ws, L.nstamps, c->cfg);
      if (!g || hipGraphLaunch(g->exec, s) != hipSuccess || hipEventRecord(g->done, s) != hipSuccess)
        return LACOSMIC_EHIP;
    } else {
      if (launch_init(f.n_new, f.niter, f.status, f.counts, f.b1s, (int64_t)L.nstamps, s) !=
          hipSuccess)
        return LACOSMIC_EHIP;
      for (int it = 0; it < f.niter; ++it)
        if (launch_iteration(f, fd, it, c->cfg, s) != hipSuccess) return LACOSMIC_EHIP;
    }
    if (!workspace && hipEventRecord(c->ws_done, s) != hipSuccess) return LACOSMIC_EHIP;
    if (hip_stream == nullptr || st != nullptr) return finish_sync(c, s, f, st);
    return LACOSMIC_OK;
  });
}

int lacosmic_run(const float* img, int64_t h, int64_t w, float gain, float readnoise,
                 float sigclip, float sigfrac, float objlim, int32_t niter, uint8_t* out_mask,
                 float* out_clean) {
  lacosmic_params p;
  p.gain = gain;
  p.readnoise = readnoise;
  p.sigclip = sigclip;
  p.sigfrac = sigfrac;
  p.objlim = objlim;
  p.niter = niter;
  p.flags = LACOSMIC_F_EARLY_STOP;
  lacosmic_stats st;
  return lacosmic_run_ex(img, h, w, &p, out_mask, out_clean, nullptr, nullptr, &st);
}

const char* lacosmic_strerror(int status) {
  switch (status) {
    case LACOSMIC_OK: return "ok";
    case LACOSMIC_EINVAL: return "invalid argument";
    case LACOSMIC_ENOMEM: return "out of memory";
    case LACOSMIC_EHIP: return "HIP runtime error";
    case LACOSMIC_ENONFINITE: return "input image holds NaN or Inf";
    case LACOSMIC_EALIAS: return "output buffer overlaps another buffer";
    case LACOSMIC_EBUDGET: return "frame can never fit the HBM budget";
    case LACOSMIC_ESCRATCH: return "frame needs more than the static scratch buffer";
    default: return "unknown status";
  }
}

int lacosmic_check_sqrt(uint32_t lo_bits, uint32_t hi_bits, uint64_t* mismatches) {
  if (!mismatches || lo_bits > hi_bits) return LACOSMIC_EINVAL;
  const float lo = [&] { float v; std::memcpy(&v, &lo_bits, 4); return v; }();
  const float hi = [&] { float v; std::memcpy(&v, &hi_bits, 4); return v; }();
  if (!(lo >= 0x1p-96f) || !(hi <= INFINITY) || (hi_bits >> 31)) return LACOSMIC_EINVAL;
  unsigned long long* d = nullptr;
  if (hipMalloc(&d, sizeof(*d)) != hipSuccess) return LACOSMIC_EHIP;
  unsigned long long n = 0;
  hipError_t e = hipMemset(d, 0, sizeof(*d));
  if (e == hipSuccess) e = launch_check_sqrt(lo_bits, hi_bits, d, nullptr);
  if (e == hipSuccess) e = hipMemcpy(&n, d, sizeof(n), hipMemcpyDeviceToHost);
  (void)hipFree(d);
  if (e != hipSuccess) return LACOSMIC_EHIP;
  *mismatches = n;
  return LACOSMIC_OK;
}

int lacosmic_set_tile_shape(int32_t cfg) {
  return guarded([&]() -> int {
    if (cfg < 0 || cfg >= kNumTileCfgs) return LACOSMIC_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LACOSMIC_EHIP;
    DevCtx* c = ctx_for(dev);
    if (!c) return LACOSMIC_EHIP;
    std::lock_guard<std::mutex> lk(c->mu);
    c->cfg = cfg;
    return LACOSMIC_OK;
  });
}

int lacosmic_set_frame_graphs(int32_t on) {
  return guarded([&]() -> int {
    if (on != 0 && on != 1) return LACOSMIC_EINVAL;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return LACOSMIC_EHIP;
    DevCtx* c = ctx_for(dev);
    if (!c) return LACOSMIC_EHIP;
    std::lock_guard<std::mutex> lk(c->mu);
    c->use_graphs = on;
    return LACOSMIC_OK;
  });
}

int lacosmic_get_tile_shape(int32_t cfg, int32_t* th, int32_t* tw) {
  if (cfg < 0 || cfg >= kNumTileCfgs || !th || !tw) return LACOSMIC_EINVAL;
  const TileShape ts = tile_shape(cfg);
  *th = ts.th;
  *tw = ts.tw;
  return LACOSMIC_OK;
}

void lacosmic_shutdown(void) { shutdown_all(); }

}  // extern "C"
