// Continuous-batching server.
//
// A worker thread owns a device arena of hbm_budget bytes and loops over
// steps.  Each step (1) admits queued frames, first come first served, while
// a slot is free and the frame's device state fits in the arena; (2) advances
// every admitted frame whose input has landed by exactly one iteration, all
// of them in one launch per pass, one block per tile (frames at different
// iterations share the launches; each frame's iteration index travels in its
// table entry); (3) hands the frames that finished their last iteration to
// the output copy.  Two more threads copy inputs in and results out on
// streams of their own, so copies overlap the steps.  Step tables are
// double-buffered so the host builds step k+1 while step k runs.  Host inputs
// and results are staged in a pinned host pool (first fit, like the device
// arena), so the copies are direct DMA; when the pool is full a request
// stages in pageable host memory instead.  A device input is not staged: the
// input copy reads it in place (device to device) when the frame is admitted.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include "lacosmic.h"
#include "lacosmic_internal.h"

namespace lac {

static double now_ns() {
  return (double)std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

// Host copy of a frame's input or results: copies of 32 MB and more are
// split over 8 threads (one host thread copies at a fraction of the memory
// bandwidth, and these copies run on the caller's thread in submit / poll).
static void host_copy(void* dst, const void* src, size_t bytes) {
  constexpr size_t kSplit = size_t(32) << 20;
  constexpr int kThreads = 8;
  if (bytes < kSplit) {
    std::memcpy(dst, src, bytes);
    return;
  }
  const size_t chunk = ((bytes + kThreads - 1) / kThreads + 4095) & ~size_t(4095);
  std::vector<std::thread> th;
  size_t done = chunk;  // chunk 0 is this thread's; chunks up to `done` are handed out
  try {
    th.reserve(kThreads - 1);
    for (int k = 1; k < kThreads && done < bytes; ++k) {
      const size_t a = done, len = std::min(chunk, bytes - a);
      th.emplace_back([=] {
        std::memcpy(static_cast<char*>(dst) + a, static_cast<const char*>(src) + a, len);
      });
      done += len;
    }
  } catch (...) {  // no thread to spare: this thread copies the rest
  }
  std::memcpy(dst, src, std::min(chunk, bytes));
  if (done < bytes)
    std::memcpy(static_cast<char*>(dst) + done, static_cast<const char*>(src) + done, bytes - done);
  for (auto& t : th) t.join();
}

// First-fit allocator over one device arena (offsets only; host side).
class Arena {
 public:
  explicit Arena(size_t size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = align256(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = align256(bytes);
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;  // offset -> size
};

struct Request {
  uint64_t ticket = 0;
  int64_t h = 0, w = 0;
  lacosmic_params p{};
  int is_u16 = 0;
  std::vector<uint8_t> img;   // host copy of the input (when the pinned pool is full)
  const void* dev_src = nullptr;  // the caller's device input, read at admission
  std::vector<uint8_t> mask;  // results (host, when the pinned pool is full)
  std::vector<float> clean;
  uint8_t* in_pin = nullptr;   // input staged in the pinned pool (in_bytes at in_off)
  size_t in_off = 0, in_bytes = 0;
  uint8_t* out_pin = nullptr;  // results in the pinned pool: clean, then the mask
  size_t out_off = 0, out_bytes = 0;
  double t_submit = 0, t_done = 0;
  int state = 0;  // 0 queued, 1 admitted, 2 done, <0 error
  // device state while admitted
  size_t off = 0, bytes = 0;
  WsLayout lay{};
  int it = 0;
  bool ready = false;
};

static size_t frame_bytes(int64_t h, int64_t w, WsLayout* lay) {
  const size_t n = (size_t)h * (size_t)w;
  *lay = ws_layout(h, w);
  // input (float), clean (float), mask bytes, workspace
  return align256(4 * n) + align256(4 * n) + align256(n) + lay->total;
}

}  // namespace lac

using namespace lac;

struct lacosmic_server {
  int dev = 0;
  uint64_t budget = 0;
  int max_frames = 0;
  char* arena_dev = nullptr;
  std::unique_ptr<Arena> arena;
  uint8_t* host_pool = nullptr;  // pinned staging of inputs and results
  std::unique_ptr<Arena> host_arena;
  hipStream_t s_comp = nullptr, s_in = nullptr, s_out = nullptr;
  FrameDev* table_dev[2] = {nullptr, nullptr};
  int* base_dev[2] = {nullptr, nullptr};  // pass-A tile prefix, then pass-B
  unsigned int* cursors_dev = nullptr;
  FrameDev* table_pin[2] = {nullptr, nullptr};
  int* base_pin[2] = {nullptr, nullptr};
  hipEvent_t step_done[2] = {nullptr, nullptr};
  int blocks[kDenseSlots] = {};  // persistent grid of each dense pass
  int cfg = 0;
  int mode = kModeGrid;  // launch form of the steps

  std::mutex mu;
  std::condition_variable cv;       // wakes the step loop
  std::condition_variable cv_io;    // wakes the copy threads
  std::condition_variable cv_done;  // wakes drain()
  std::deque<Request*> queue;       // submitted, not admitted
  std::deque<Request*> in_q;        // admitted, input copy pending
  std::deque<Request*> out_q;       // finished, output copy pending
  std::map<uint64_t, Request*> reqs;
  std::vector<Request*> active;     // admitted, iterations left
  uint64_t next_ticket = 1;
  uint64_t pending = 0;             // submitted and not yet done
  bool stop = false, stop_io = false;
  int error = 0;
  std::thread worker, copy_in, copy_out;

  void run();
  void run_copy_in();
  void run_copy_out();
  void fail_locked(int rc);
};

static char* ws_of(char* base, const Request* r) {
  const size_t n = (size_t)r->h * (size_t)r->w;
  return base + 2 * align256(4 * n) + align256(n);
}

void lacosmic_server::fail_locked(int rc) {
  if (!error) error = rc;
  cv_done.notify_all();
  cv.notify_all();
}

// Input copies: the host image to the frame's arena block (uint16 frames are
// staged in the S' plane and widened exactly), then the counters reset.
void lacosmic_server::run_copy_in() {
  (void)hipSetDevice(dev);
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_io.wait(lk, [&] { return stop_io || !in_q.empty(); });
      if (in_q.empty()) return;
      r = in_q.front();
      in_q.pop_front();
    }
    const size_t n = (size_t)r->h * (size_t)r->w;
    char* base = arena_dev + r->off;
    char* ws = ws_of(base, r);
    float* img = reinterpret_cast<float*>(base);
    hipError_t e;
    const void* src = r->dev_src  ? r->dev_src
                      : r->in_pin ? static_cast<const void*>(r->in_pin)
                                  : static_cast<const void*>(r->img.data());
    const hipMemcpyKind kind = r->dev_src ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    if (r->is_u16 && r->dev_src) {  // widened straight from the caller's buffer
      e = launch_u16_to_f32(static_cast<const uint16_t*>(src), img, (int64_t)n, s_in);
    } else if (r->is_u16) {
      uint16_t* stage = reinterpret_cast<uint16_t*>(ws + r->lay.sp);
      e = hipMemcpyAsync(stage, src, 2 * n, kind, s_in);
      if (e == hipSuccess) e = launch_u16_to_f32(stage, img, (int64_t)n, s_in);
    } else {
      e = hipMemcpyAsync(img, src, 4 * n, kind, s_in);
    }
    if (e == hipSuccess)
      e = launch_init(reinterpret_cast<unsigned long long*>(ws + r->lay.counters), r->p.niter,
                      reinterpret_cast<int*>(ws + r->lay.status),
                      reinterpret_cast<unsigned int*>(ws + r->lay.counts),
                      reinterpret_cast<int*>(ws + r->lay.stamps), (int64_t)r->lay.nstamps, s_in);
    if (e == hipSuccess) e = hipStreamSynchronize(s_in);
    std::lock_guard<std::mutex> lk(mu);
    if (e != hipSuccess) {
      fail_locked(LACOSMIC_EHIP);
    } else {
      if (r->in_pin) host_arena->release(r->in_off, r->in_bytes);
      r->in_pin = nullptr;
      r->dev_src = nullptr;
      std::vector<uint8_t>().swap(r->img);
      r->ready = true;
      cv.notify_all();
    }
  }
}

// Output copies of finished frames, then the arena block is released.
void lacosmic_server::run_copy_out() {
  (void)hipSetDevice(dev);
  for (;;) {
    Request* r = nullptr;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_io.wait(lk, [&] { return stop_io || !out_q.empty(); });
      if (out_q.empty()) return;
      r = out_q.front();
      out_q.pop_front();
    }
    const size_t n = (size_t)r->h * (size_t)r->w;
    char* base = arena_dev + r->off;
    const float* clean = reinterpret_cast<const float*>(base + align256(4 * n));
    const uint8_t* mask = reinterpret_cast<const uint8_t*>(base + 2 * align256(4 * n));
    const int* st_dev = reinterpret_cast<const int*>(ws_of(base, r) + r->lay.status);
    {
      std::lock_guard<std::mutex> lk(mu);
      r->out_bytes = align256(4 * n) + n;
      if (host_arena && host_arena->alloc(r->out_bytes, &r->out_off))
        r->out_pin = host_pool + r->out_off;
    }
    float* clean_host;
    uint8_t* mask_host;
    if (r->out_pin) {
      clean_host = reinterpret_cast<float*>(r->out_pin);
      mask_host = r->out_pin + align256(4 * n);
    } else {
      r->mask.resize(n);
      r->clean.resize(n);
      clean_host = r->clean.data();
      mask_host = r->mask.data();
    }
    int status = 0;
    hipError_t e = hipMemcpyAsync(clean_host, clean, 4 * n, hipMemcpyDeviceToHost, s_out);
    if (e == hipSuccess) e = hipMemcpyAsync(mask_host, mask, n, hipMemcpyDeviceToHost, s_out);
    if (e == hipSuccess)
      e = hipMemcpyAsync(&status, st_dev, sizeof(int), hipMemcpyDeviceToHost, s_out);
    if (e == hipSuccess) e = hipStreamSynchronize(s_out);
    const double t = now_ns();
    std::lock_guard<std::mutex> lk(mu);
    arena->release(r->off, r->bytes);
    r->t_done = t;
    r->state = (e != hipSuccess) ? LACOSMIC_EHIP : (status & 1) ? LACOSMIC_ENONFINITE : 2;
    --pending;
    cv_done.notify_all();
    cv.notify_all();  // arena space for the queue
  }
}

void lacosmic_server::run() {
  (void)hipSetDevice(dev);
  int slot = 0;
  std::vector<Request*> finishing[2];  // frames whose last iteration runs in that slot's step
  bool inflight[2] = {false, false};
  auto retire = [&](int k) {  // step k is complete: hand its finished frames out
    (void)hipEventSynchronize(step_done[k]);
    inflight[k] = false;
    std::lock_guard<std::mutex> lk(mu);
    for (Request* r : finishing[k]) out_q.push_back(r);
    finishing[k].clear();
    cv_io.notify_all();
  };
  for (;;) {
    std::vector<Request*> step;
    {
      std::unique_lock<std::mutex> lk(mu);
      if (error) return;
      // admit first come, first served, while a slot and arena space are free
      while (!queue.empty() && (int)active.size() < max_frames) {
        Request* r = queue.front();
        size_t off = 0;
        if (!arena->alloc(r->bytes, &off)) break;
        queue.pop_front();
        r->off = off;
        r->state = 1;
        r->it = 0;
        r->ready = false;
        active.push_back(r);
        in_q.push_back(r);
        cv_io.notify_all();
      }
      for (Request* r : active)
        if (r->ready && r->it < r->p.niter) step.push_back(r);
      if (step.empty() && !inflight[0] && !inflight[1]) {
        if (stop && queue.empty() && active.empty()) return;
        cv.wait_for(lk, std::chrono::milliseconds(20));
        continue;
      }
    }
    if (step.empty()) {  // nothing new to launch: complete the older step
      retire(inflight[slot] ? slot : slot ^ 1);
      continue;
    }
    if (inflight[slot]) retire(slot);  // its table buffer is about to be reused

    const TileShape ts = tile_shape(cfg);
    const int nf = (int)step.size();
    int total = 0, total_b = 0;
    bool first = false, later = false, final = false;  // frames at iteration 0 / later / last
    bool est = false;                                   // frames estimating their gain
    int64_t biggest = 1;
    for (size_t i = 0; i < step.size(); ++i) {
      Request* r = step[i];
      (r->it == 0 ? first : later) = true;
      final = final || r->it == r->p.niter - 1;
      est = est || (r->p.flags & LACOSMIC_F_ESTIMATE_GAIN) != 0;
      biggest = std::max<int64_t>(biggest, r->h * r->w);
      const size_t n = (size_t)r->h * (size_t)r->w;
      char* base = arena_dev + r->off;
      FrameDev f = make_frame(reinterpret_cast<const float*>(base), r->h, r->w, r->p,
                              reinterpret_cast<uint8_t*>(base + 2 * align256(4 * n)),
                              reinterpret_cast<float*>(base + align256(4 * n)), ws_of(base, r),
                              r->lay, cfg);
      f.it = r->it;
      table_pin[slot][i] = f;
      base_pin[slot][i] = total;
      base_pin[slot][nf + 1 + i] = total_b;
      total += (int)(((r->w + ts.tw - 1) / ts.tw) * ((r->h + ts.th - 1) / ts.th));
      total_b += f.tiles_b;
    }
    base_pin[slot][nf] = total;
    base_pin[slot][2 * nf + 1] = total_b;
    hipError_t e = hipMemcpyAsync(table_dev[slot], table_pin[slot], sizeof(FrameDev) * nf,
                                  hipMemcpyHostToDevice, s_comp);
    if (e == hipSuccess)
      e = hipMemcpyAsync(base_dev[slot], base_pin[slot], sizeof(int) * 2 * (nf + 1),
                         hipMemcpyHostToDevice, s_comp);
    QueueArgs a{table_dev[slot], base_dev[slot], base_dev[slot] + (nf + 1), nf,
                cursors_dev + 8 * kDenseSlots * slot, 0, 0};
    if (e == hipSuccess) e = launch_queue_init(a, 8 * kDenseSlots, 0, s_comp);
    for (int pass = 0; pass < kPassesPerIter && e == hipSuccess; ++pass) {
      // a pass runs when some frame of the step needs it (the kernels skip
      // the frames it does not apply to)
      bool needed = true;
      switch (pass) {
        case kPassGain: needed = est; break;
        case kPassUS: needed = later; break;
        case kPassA1: needed = first || est; break;
        case kPassOut: needed = final; break;
        default: break;
      }
      if (!needed) continue;
      const int ds = dense_slot(pass);
      a.cursor_slot = ds < 0 ? 0 : ds;
      if (pass == kPassGain)
        a.blocks = gain_blocks(biggest);
      else if (ds < 0)
        a.blocks = 0;
      else if (mode == kModeGrid)
        a.blocks = pass == kPassA1 ? total : total_b;
      else
        a.blocks = blocks[ds];
      e = launch_queue_pass(a, pass, -1, cfg, mode, s_comp);
    }
    if (e == hipSuccess) e = hipEventRecord(step_done[slot], s_comp);
    std::lock_guard<std::mutex> lk(mu);
    if (e != hipSuccess) {
      fail_locked(LACOSMIC_EHIP);
      return;
    }
    inflight[slot] = true;
    for (Request* r : step) {
      if (++r->it == r->p.niter) {
        finishing[slot].push_back(r);
        active.erase(std::find(active.begin(), active.end(), r));
      }
    }
    slot ^= 1;
  }
}

extern "C" {

int lacosmic_server_create(uint64_t hbm_budget_bytes, int32_t max_frames, lacosmic_server** out) {
  return guarded([&]() -> int {
    if (!out || hbm_budget_bytes < 4096 || max_frames < 1 || max_frames > 4096)
      return LACOSMIC_EINVAL;
    *out = nullptr;
    std::unique_ptr<lacosmic_server> s(new lacosmic_server());
    if (hipGetDevice(&s->dev) != hipSuccess) return LACOSMIC_EHIP;
    s->budget = hbm_budget_bytes;
    s->max_frames = max_frames;
    if (hipMalloc(&s->arena_dev, hbm_budget_bytes) != hipSuccess) {
      s->arena_dev = nullptr;
      return LACOSMIC_ENOMEM;
    }
    s->arena.reset(new Arena(hbm_budget_bytes));
    {  // pinned staging: a quarter of the budget, 256 MiB .. 8 GiB
       // (LACOSMIC_SERVER_PINNED_MB overrides; 0 disables it)
      size_t pool = std::min<size_t>(std::max<size_t>(hbm_budget_bytes / 4, size_t(256) << 20),
                                     size_t(8) << 30);
      if (const char* env = std::getenv("LACOSMIC_SERVER_PINNED_MB"))
        pool = (size_t)std::strtoull(env, nullptr, 10) << 20;
      void* hp = nullptr;
      if (pool && hipHostMalloc(&hp, pool, hipHostMallocDefault) == hipSuccess) {
        s->host_pool = static_cast<uint8_t*>(hp);
        s->host_arena.reset(new Arena(pool));
      }
    }
    bool ok = hipStreamCreateWithFlags(&s->s_comp, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&s->s_in, hipStreamNonBlocking) == hipSuccess &&
              hipStreamCreateWithFlags(&s->s_out, hipStreamNonBlocking) == hipSuccess &&
              hipMalloc(&s->cursors_dev, sizeof(unsigned int) * 2 * 8 * kDenseSlots) == hipSuccess;
    for (int k = 0; k < 2 && ok; ++k) {
      ok = hipMalloc(&s->table_dev[k], sizeof(FrameDev) * max_frames) == hipSuccess &&
           hipMalloc(&s->base_dev[k], sizeof(int) * 2 * (max_frames + 1)) == hipSuccess &&
           hipHostMalloc(&s->table_pin[k], sizeof(FrameDev) * max_frames, hipHostMallocDefault) ==
               hipSuccess &&
           hipHostMalloc(&s->base_pin[k], sizeof(int) * 2 * (max_frames + 1), hipHostMallocDefault) ==
               hipSuccess &&
           hipEventCreateWithFlags(&s->step_done[k], hipEventDisableTiming) == hipSuccess;
    }
    if (!ok) {
      lacosmic_server_destroy(s.release());
      return LACOSMIC_ENOMEM;
    }
    int dev = s->dev;
    DevCtx* c = ctx_for(dev);
    s->cfg = c ? c->cfg : 1;
    for (int pass : {kPassA1, kPassSC, kPassB, kPassOut}) s->blocks[dense_slot(pass)] = queue_blocks(s->cfg, pass);
    lacosmic_server* raw = s.release();
    // a thread that fails records the error (drain and poll report it) and
    // stops; a thread that cannot be started undoes the whole server
    auto body = [raw](void (lacosmic_server::*fn)()) {
      try {
        (raw->*fn)();
      } catch (...) {
        std::lock_guard<std::mutex> lk(raw->mu);
        raw->fail_locked(LACOSMIC_ENOMEM);
      }
    };
    try {
      raw->worker = std::thread(body, &lacosmic_server::run);
      raw->copy_in = std::thread(body, &lacosmic_server::run_copy_in);
      raw->copy_out = std::thread(body, &lacosmic_server::run_copy_out);
    } catch (...) {
      lacosmic_server_destroy(raw);
      return LACOSMIC_EHIP;
    }
    *out = raw;
    return LACOSMIC_OK;
  });
}

int lacosmic_server_submit(lacosmic_server* s, const void* img, int is_u16, int64_t h, int64_t w,
                           const lacosmic_params* p, uint64_t* ticket) {
  return guarded([&]() -> int {
    if (!s || !img || !ticket) return LACOSMIC_EINVAL;
    const int rc = check_params(h, w, p);
    if (rc) return rc;
    if (p->flags & LACOSMIC_F_INPUT_U16) return LACOSMIC_EINVAL;  // is_u16 says it here
    std::unique_ptr<Request> r(new Request());
    r->h = h;
    r->w = w;
    r->p = *p;
    r->is_u16 = is_u16 ? 1 : 0;
    r->bytes = frame_bytes(h, w, &r->lay);
    if (r->bytes > s->budget) return LACOSMIC_EBUDGET;
    const size_t n = (size_t)h * (size_t)w;
    const size_t in_bytes = (is_u16 ? 2 : 4) * n;
    r->t_submit = now_ns();
    {  // device memory is read in place at admission; anything else is host memory
      hipPointerAttribute_t attr{};
      if (hipPointerGetAttributes(&attr, img) == hipSuccess) {
        if (attr.type == hipMemoryTypeDevice) {
          if (attr.device != s->dev) return LACOSMIC_EINVAL;
          r->dev_src = img;
        }
      } else {
        (void)hipGetLastError();  // pageable host memory: not an error of this thread's next call
      }
    }
    if (!r->dev_src) {
      {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->error) return s->error;
        r->in_bytes = in_bytes;
        if (s->host_arena && s->host_arena->alloc(in_bytes, &r->in_off))
          r->in_pin = s->host_pool + r->in_off;
      }
      if (r->in_pin) {
        host_copy(r->in_pin, img, in_bytes);
      } else {
        r->img.resize(in_bytes);
        host_copy(r->img.data(), img, in_bytes);
      }
    }
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->error) {
      if (r->in_pin) s->host_arena->release(r->in_off, r->in_bytes);
      return s->error;
    }
    r->ticket = s->next_ticket++;
    *ticket = r->ticket;
    s->reqs[r->ticket] = r.get();
    s->queue.push_back(r.release());
    ++s->pending;
    s->cv.notify_all();
    return LACOSMIC_OK;
  });
}

int lacosmic_server_poll(lacosmic_server* s, uint64_t ticket, uint8_t* out_mask, float* out_clean,
                         double* t_submit_ns, double* t_done_ns) {
  if (!s) return LACOSMIC_EINVAL;
  Request* r = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(ticket);
    if (it == s->reqs.end()) return LACOSMIC_EINVAL;
    r = it->second;
    // still queued or running: pending, unless the server has failed (its
    // worker stopped, so the frame will never finish)
    if (r->state == 0 || r->state == 1) return s->error ? s->error : 0;
    s->reqs.erase(it);
  }
  const int state = r->state;
  if (t_submit_ns) *t_submit_ns = r->t_submit;
  if (t_done_ns) *t_done_ns = r->t_done;
  const size_t n = (size_t)r->h * (size_t)r->w;
  if (state == 2) {
    const float* clean_host =
        r->out_pin ? reinterpret_cast<const float*>(r->out_pin) : r->clean.data();
    const uint8_t* mask_host = r->out_pin ? r->out_pin + align256(4 * n) : r->mask.data();
    if (out_mask) host_copy(out_mask, mask_host, n);
    if (out_clean) host_copy(out_clean, clean_host, n * sizeof(float));
  }
  if (r->out_pin) {
    std::lock_guard<std::mutex> lk(s->mu);
    s->host_arena->release(r->out_off, r->out_bytes);
  }
  delete r;
  return state == 2 ? 1 : state;
}

int lacosmic_server_drain(lacosmic_server* s) {
  if (!s) return LACOSMIC_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->pending == 0 || s->error != 0; });
  return s->error;
}

int lacosmic_server_destroy(lacosmic_server* s) {
  if (!s) return LACOSMIC_EINVAL;
  if (s->worker.joinable()) {  // every submitted frame finishes first
    {
      std::lock_guard<std::mutex> lk(s->mu);
      s->stop = true;
      s->cv.notify_all();
    }
    s->worker.join();
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop_io = true;
    s->cv_io.notify_all();
  }
  if (s->copy_in.joinable()) s->copy_in.join();
  if (s->copy_out.joinable()) s->copy_out.join();
  if (s->s_comp) (void)hipStreamSynchronize(s->s_comp);
  if (s->s_in) (void)hipStreamSynchronize(s->s_in);
  if (s->s_out) (void)hipStreamSynchronize(s->s_out);
  for (auto& kv : s->reqs) delete kv.second;
  for (int k = 0; k < 2; ++k) {
    if (s->table_dev[k]) (void)hipFree(s->table_dev[k]);
    if (s->base_dev[k]) (void)hipFree(s->base_dev[k]);
    if (s->table_pin[k]) (void)hipHostFree(s->table_pin[k]);
    if (s->base_pin[k]) (void)hipHostFree(s->base_pin[k]);
    if (s->step_done[k]) (void)hipEventDestroy(s->step_done[k]);
  }
  if (s->cursors_dev) (void)hipFree(s->cursors_dev);
  if (s->arena_dev) (void)hipFree(s->arena_dev);
  if (s->host_pool) (void)hipHostFree(s->host_pool);
  if (s->s_comp) (void)hipStreamDestroy(s->s_comp);
  if (s->s_in) (void)hipStreamDestroy(s->s_in);
  if (s->s_out) (void)hipStreamDestroy(s->s_out);
  delete s;
  return LACOSMIC_OK;
}

}  // extern "C"
