// Kernels and launchers: the single-frame launch (one block per tile) and
// the persistent tile-queue launch used by the batched and serving paths.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "lacosmic_gain.h"
#include "lacosmic_launch.h"
#include "lacosmic_small.h"
#include "lacosmic_tiles.h"

namespace lac {

// Logical tile of a block: consecutive tiles go to the same XCD (blocks are
// dispatched round-robin over the 8 XCDs), so neighbouring tiles share their
// halo rows in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, rem = n & 7;
  const int x = b & 7, j = b >> 3;
  return x * q + (x < rem ? x : rem) + j;
}

static_assert(B_WORDS == kStripWords && B_WAVES == kBWaves, "pass-B tiles differ between host and device");

// Dense passes on tile t of frame f: A1 (PASS 0, iteration 0) and A2
// (PASS 1, full-S' frames) on TH x 64 tiles; B (PASS 2), SC (PASS 3) and OUT
// (PASS 5) on pass-B tile t (4 strips of kBStrip rows by one strip column,
// one per wave).
template <int TH, int NT, int PASS>
__device__ __forceinline__ void run_tile(const FrameDev& f, int it, int t, void* smem) {
  if (PASS == 2 || PASS == 3 || PASS == 5) {
    const int ncol = strip_ncols(f.wpr);
    const int band = t / ncol, col = t - band * ncol;
    // wave-uniform (the wave index read through the first lane): the strip's
    // row arithmetic stays scalar
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int y0 = (band * B_WAVES + wv) * kBStrip;
    if (wv < B_WAVES && y0 < f.h) {
      if (PASS == 2)
        strip_b(f, it, y0, col * B_WORDS);
      else if (PASS == 3)
        strip_sc(f, it, y0, col * B_WORDS);
      else
        strip_out(f, it, y0, col * B_WORDS);
    }
    return;
  }
  if (stopped(f, it)) return;
  if ((PASS == 0 && it != 0 && !f.est_gain) || (PASS == 1 && !f.full_sp)) return;
  const int ty = t / f.tiles_x, tx = t - ty * f.tiles_x;
  const int y0 = ty * TH, x0 = tx * TW;
  if (PASS == 0)
    tile_a1<TH, NT>(f, it, y0, x0, tx, *static_cast<SmemA1<TH>*>(smem));
  else
    tile_a2<TH, NT>(f, y0, x0, *static_cast<SmemA2<TH>*>(smem));
}

struct SmemNone {
  int unused;
};
template <int TH, int PASS>
struct SmemOf;
template <int TH>
struct SmemOf<TH, 0> { using T = SmemA1<TH>; };
template <int TH>
struct SmemOf<TH, 1> { using T = SmemA2<TH>; };
template <int TH>
struct SmemOf<TH, 2> { using T = SmemNone; };
template <int TH>
struct SmemOf<TH, 3> { using T = SmemNone; };
template <int TH>
struct SmemOf<TH, 5> { using T = SmemNone; };



// ------------------------------------------------------------ single frame
// The frame's record lives in device memory (written by k_put_frame before
// the launches), so a recorded sequence of these launches serves any buffers
// and parameters of the same shape.  Its fields are wave-uniform: scalar loads.
template <int TH, int NT, int PASS>
__global__ __launch_bounds__(NT) void k_frame(const FrameDev* __restrict__ fp, int it) {
  __shared__ typename SmemOf<TH, PASS>::T s;
  const FrameDev f = *fp;
  run_tile<TH, NT, PASS>(f, it, xcd_remap(blockIdx.x, gridDim.x), &s);
}

// A sparse pass (sparse_frame) of one frame.
template <int WHICH>
__global__ __launch_bounds__(256) void k_sparse_frame(const FrameDev* __restrict__ fp, int it) {
  __shared__ WaveQueue wq[(WHICH == 0 || WHICH == 2) ? 4 : 1];
  const FrameDev f = *fp;
  sparse_frame<WHICH, true>(f, it, (long long)blockIdx.x * blockDim.x + threadIdx.x,
                      (long long)gridDim.x * blockDim.x,
                      &wq[(WHICH == 0 || WHICH == 2) ? (threadIdx.x >> 6) : 0]);
}

// One whole iteration of a small frame, one block per 32 x 32 output tile
// (consecutive tiles on one XCD: their regions overlap).
__global__ __launch_bounds__(kFusedThreads) void k_fused(const FrameDev* __restrict__ fp, int it) {
  __shared__ SmemFused s;
  const FrameDev f = *fp;
  tile_fused<kFusedThreads>(f, it, xcd_remap(blockIdx.x, gridDim.x), s);
}

// Stores a frame record (a kernel argument) in device memory.
__global__ void k_put_frame(FrameDev f, FrameDev* dst) {
  static_assert(sizeof(FrameDev) % 4 == 0, "the record is copied in 32-bit words");
  constexpr int kWords = (int)(sizeof(FrameDev) / 4);
  const uint32_t* src = reinterpret_cast<const uint32_t*>(&f);
  for (int i = threadIdx.x; i < kWords; i += blockDim.x) reinterpret_cast<uint32_t*>(dst)[i] = src[i];
}

// Zero one frame's per-iteration counters (and the unreplaced-pixel count
// after them), list lengths and status.
__global__ void k_init(unsigned long long* n_new, int niter, int* status, unsigned int* counts,
                       int* stamps, int64_t nstamps) {
  for (int i = threadIdx.x; i <= niter; i += blockDim.x) n_new[i] = 0ull;
  for (int i = threadIdx.x; i < kCntPerIter * niter; i += blockDim.x) counts[i] = 0u;
  for (int64_t i = threadIdx.x; i < nstamps; i += blockDim.x) stamps[i] = 0;
  if (threadIdx.x == 0) *status = 0;
}

// ------------------------------------------------------------ tile queue
// Tiles of all frames are numbered frame by frame; tile_base[k] is the first
// tile of frame k (tile_base[nframes] = total).  A block stages tile_base in
// LDS (up to kLdsFrames frames) so finding a tile's frame is a short search
// in LDS.
constexpr int kLdsFrames = 512;

template <typename P>
__device__ __forceinline__ int frame_of_t(P base, int nframes, int t) {
  int lo = 0, hi = nframes - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (base[mid] <= t) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Tile bases of a multi-frame launch: staged in LDS when they fit (sb), read
// from global memory otherwise.
struct Bases {
  const int* sb;     // LDS copy, or nullptr
  const int* gbase;  // the global array
  __device__ int operator[](int i) const { return sb ? sb[i] : gbase[i]; }
};

__device__ __forceinline__ Bases stage_bases(const int* tile_base, int nframes, int* sb) {
  if (nframes > kLdsFrames) return Bases{nullptr, tile_base};
  for (int i = threadIdx.x; i <= nframes; i += blockDim.x) sb[i] = ldg(tile_base, i);
  __syncthreads();
  return Bases{sb, tile_base};
}

__device__ __forceinline__ int frame_of(const Bases& b, int nframes, int t) {
  if (b.sb) {
    typedef const __attribute__((address_space(3))) int* lptr;
    return frame_of_t((lptr)b.sb, nframes, t);
  }
  return frame_of_t(b.gbase, nframes, t);
}

// Persistent launch: the queue is split into 8 contiguous ranges, one per
// XCD; a block takes tiles from its own XCD's range and, once that is empty,
// from the others in turn.  Thread 0 requests the next tile while the block
// works on the current one.  Every block exits when all 8 ranges are empty.
template <int TH, int NT, int PASS>
__global__ __launch_bounds__(NT) void k_queue(const FrameDev* __restrict__ frames, const int* tile_base,
                                              int nframes, int it, unsigned int* cursors) {
  // tile_base: TH x 64 tiles for PASS 0/1, pass-B tiles for PASS 2/3
  __shared__ typename SmemOf<TH, PASS>::T s;
  __shared__ int sb[kLdsFrames + 1];
  __shared__ int s_next;
  const Bases base = stage_bases(tile_base, nframes, sb);
  const int total = base[nframes];
  const int q = total >> 3, rem = total & 7;
  const int home = blockIdx.x & 7;
  int k = 0;  // ranges tried so far (thread 0)
  // next tile from the queue, moving on to the next XCD's range when empty
  auto grab = [&]() -> int {
    while (k < 8) {
      const int x = (home + k) & 7;
      const unsigned int j = atom_add(cursors + x, 1u);
      const unsigned int count = (unsigned int)(q + (x < rem ? 1 : 0));
      if (j < count) return x * q + (x < rem ? x : rem) + (int)j;
      ++k;
    }
    return -1;
  };
  if (threadIdx.x == 0) s_next = grab();
  __syncthreads();
  for (;;) {
    const int t = s_next;
    __syncthreads();
    if (t < 0) break;
    // request the following tile now; its index is only needed after this one
    unsigned int j_next = 0;
    int x_next = -1;
    if (threadIdx.x == 0 && k < 8) {
      x_next = (home + k) & 7;
      j_next = atom_add(cursors + x_next, 1u);
    }
    // block-uniform frame index: its record is read with scalar loads, into a
    // copy (a reference would be re-read after every store that might alias it)
    const int fi = __builtin_amdgcn_readfirstlane(frame_of(base, nframes, t));
    const FrameDev f = frames[fi];
    const int tl = __builtin_amdgcn_readfirstlane(t - base[fi]);  // tile index in the frame
    run_tile<TH, NT, PASS>(f, it >= 0 ? it : f.it, tl, &s);
    if (threadIdx.x == 0) {
      int nxt = -1;
      if (x_next >= 0) {
        const unsigned int count = (unsigned int)(q + (x_next < rem ? 1 : 0));
        if (j_next < count)
          nxt = x_next * q + (x_next < rem ? x_next : rem) + (int)j_next;
        else {
          ++k;
          nxt = grab();
        }
      }
      s_next = nxt;
    }
    __syncthreads();
  }
}

// Grid launch over the tiles of all frames: one block per tile, consecutive
// tiles on the same XCD.
template <int TH, int NT, int PASS>
__global__ __launch_bounds__(NT) void k_grid(const FrameDev* __restrict__ frames, const int* tile_base,
                                             int nframes, int it) {
  __shared__ typename SmemOf<TH, PASS>::T s;
  __shared__ int sb[kLdsFrames + 1];
  // A1 is bound by vector issue and shares the CUs with the other frame
  // groups' latency-bound passes: its waves take issue slots first
  if constexpr (PASS == 0) __builtin_amdgcn_s_setprio(3);
  const Bases base = stage_bases(tile_base, nframes, sb);
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  // block-uniform frame index: its record is read with scalar loads, into a
  // copy (a reference would be re-read after every store that might alias it)
  const int fi = __builtin_amdgcn_readfirstlane(frame_of(base, nframes, t));
  const FrameDev f = frames[fi];
  const int tl = __builtin_amdgcn_readfirstlane(t - base[fi]);  // tile index in the frame
  run_tile<TH, NT, PASS>(f, it >= 0 ? it : f.it, tl, &s);
}

// A sparse pass over every frame of a multi-frame launch.  The frames' item
// ranges, each padded to a multiple of 64, are one concatenated index space
// (prefix sums staged in LDS), so the items spread over the whole grid
// whatever their distribution over frames, and the 64 items of a wave always
// belong to one frame: the frame lookup is wave-uniform and its record is
// read with scalar loads.
template <int WHICH>
__global__ __launch_bounds__(256) void k_sparse_queue(const FrameDev* __restrict__ frames,
                                                      int nframes, int it) {
  __shared__ long long pre[kLdsFrames + 1];
  __shared__ long long len[kLdsFrames];
  const long long gtid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long gstride = (long long)gridDim.x * blockDim.x;
  if (nframes > kLdsFrames) {  // rare: frame by frame
    for (int fi = 0; fi < nframes; ++fi) {
      const FrameDev f = frames[fi];
      sparse_frame<WHICH, false>(f, it >= 0 ? it : f.it, gtid, gstride, nullptr);
    }
    return;
  }
  const int lane = threadIdx.x & 63;
  if (threadIdx.x < 64) {  // the first wave: lane l reads frames l, l + 64, ...
    long long carry = 0;
    for (int f0 = 0; f0 < nframes; f0 += 64) {
      const int fi = f0 + lane;
      long long n = 0;
      if (fi < nframes) {
        const FrameDev& f = frames[fi];
        n = sparse_len<WHICH>(f, it >= 0 ? it : f.it);
        len[fi] = n;
      }
      const long long padded = (n + 63) & ~63ll;  // whole waves per frame
      long long incl = padded;
#pragma unroll
      for (int off = 1; off < 64; off <<= 1) {
        const long long y = __shfl_up(incl, off);
        if (lane >= off) incl += y;
      }
      if (fi < nframes) pre[fi] = carry + incl - padded;
      carry += __shfl(incl, 63);
    }
    if (lane == 0) pre[nframes] = carry;
  }
  __syncthreads();
  const long long total = pre[nframes];
  // second stages (S1, SG) run at once here: a wave's consecutive chunks
  // belong to different frames too often for the per-wave queue to fill
  for (long long g0 = gtid - lane; g0 < total; g0 += gstride) {  // g0: the wave's chunk
    int lo = 0, hi = nframes - 1;  // last frame whose range starts at or before g0
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pre[mid] <= g0) lo = mid; else hi = mid - 1;
    }
    lo = __builtin_amdgcn_readfirstlane(lo);
    const FrameDev f = frames[lo];  // a copy: not re-read after each store
    const int fit = it >= 0 ? it : f.it;
    const long long g = g0 - pre[lo] + lane;
    const bool active = g < len[lo];
    if constexpr (WHICH == 3) {  // US: whole waves (update_s_quad combines over lanes)
      const int qq = active ? ldg(f.conf, g) : 0;
      const int qy = row_of(f, qq);
      update_s_quad(f, noise_coef(f, fit), qy, qq - qy * f.w, active);
    } else if (active) {
      int ky = 0, kx = 0;
      float val = 0.0f;
      const int key = sparse_item<WHICH>(f, fit, g, ky, kx, val);
      if (key >= 0) sparse_second<WHICH>(f, fit, key, ky, kx, val);
    }
  }
}

// Zero per-frame counters, list lengths and status (first launch of a batch)
// and the queue cursors of every pass of the run.
__global__ void k_batch_init(const FrameDev* frames, int nframes, unsigned int* cursors,
                             int ncursors, int zero_counters) {
  const int fi = blockIdx.x;
  if (fi < nframes && zero_counters) {
    const FrameDev& f = frames[fi];
    for (int i = threadIdx.x; i <= f.niter; i += blockDim.x) f.n_new[i] = 0ull;
    for (int i = threadIdx.x; i < kCntPerIter * f.niter; i += blockDim.x) f.counts[i] = 0u;
    const int nst = ((f.h + kBStrip - 1) / kBStrip) * strip_ncols(f.wpr);
    for (int i = threadIdx.x; i < nst; i += blockDim.x) {
      f.b1s[i] = 0;
      f.bq[i] = 0;
    }
    if (threadIdx.x == 0) *f.status = 0;
  }
  if (fi == 0)
    for (int i = threadIdx.x; i < ncursors; i += blockDim.x) cursors[i] = 0u;
}

// ------------------------------------------------------------ gain estimate
// Launched over frame tables (one frame: its record) with blockIdx.y the
// frame; frames with a supplied gain, or stopped early, do nothing.
__global__ void k_gain_reset(const FrameDev* __restrict__ frames, int it) {
  const FrameDev& f = frames[blockIdx.x];
  const int fit = it >= 0 ? it : f.it;
  if (!f.est_gain || stopped(f, fit)) return;
  gain_reset(f);
}

template <int P>
__global__ __launch_bounds__(kGainThreads) void k_gain(const FrameDev* __restrict__ frames, int it) {
  __shared__ GainShared sh;
  const FrameDev& f = frames[blockIdx.y];
  const int fit = it >= 0 ? it : f.it;
  if (!f.est_gain || stopped(f, fit)) return;
  gain_pass<P>(f, fit, blockIdx.x, gridDim.x, sh);
}

// uint16 ADU to float32: every uint16 value is exact in binary32.
__global__ void k_u16_to_f32(const uint16_t* in, float* out, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

// ------------------------------------------------------------ launchers
int gain_blocks(int64_t pixels) {
  const int64_t want = (pixels + 16 * kGainThreads - 1) / (16 * kGainThreads);
  return (int)std::min<int64_t>(1024, std::max<int64_t>(1, want));
}

hipError_t launch_gain(const FrameDev* frames, int nframes, int it, int nbx, hipStream_t st) {
  if (nframes <= 0) return hipSuccess;
  k_gain_reset<<<nframes, 256, 0, st>>>(frames, it);
  const dim3 grid((unsigned)nbx, (unsigned)nframes);
  for (int r = 0; r < kGainRounds; ++r) {
    k_gain<0><<<grid, kGainThreads, 0, st>>>(frames, it);
    k_gain<1><<<grid, kGainThreads, 0, st>>>(frames, it);
    k_gain<2><<<grid, kGainThreads, 0, st>>>(frames, it);
  }
  k_gain<0><<<grid, kGainThreads, 0, st>>>(frames, it);  // the sums after the last round
  return hipGetLastError();
}

// Grid of the sparse passes: enough waves per SIMD to hide their gathers.
static int sparse_blocks() {
  static int blocks = 0;
  if (!blocks) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus < 1)
      cus = 256;
    blocks = 8 * cus;
  }
  return blocks;
}

// Grid of the multi-frame S1: the blocks that fit on the chip at once.  Its
// test holds 185 registers (two blocks per CU); launched with the grid above,
// three quarters of the blocks only queued behind the resident ones and each
// round of them ended on its slowest block (1.75 against 1.52 ms per batch
// step).  The passes stride over their items, so any grid covers them.
static int s1_batch_blocks() {
  static const int blocks = [] {
    int per_cu = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_sparse_queue<0>, 256, 0) !=
            hipSuccess ||
        per_cu < 1)
      return sparse_blocks();
    return std::min(sparse_blocks(), sparse_blocks() / 8 * per_cu);
  }();
  return blocks;
}

template <int WHICH>
static void sparse_launch(const FrameDev* fd, int it, unsigned ns, hipStream_t st) {
  k_sparse_frame<WHICH><<<ns, 256, 0, st>>>(fd, it);
}

// One iteration: grid sizes from the host copy f, the kernels read the
// device copy fd.
template <int TH, int NT>
static hipError_t frame_iter_t(const FrameDev& f, const FrameDev* fd, int it, hipStream_t st) {
  const unsigned nb = (unsigned)f.tiles;
  // one frame's lists are short: one block per 16k pixels, at most the
  // multi-frame grid
  const int64_t px = (int64_t)f.h * f.w;
  const unsigned ns = (unsigned)std::min<int64_t>(sparse_blocks(),
                                                  std::max<int64_t>(16, px >> 14));
  constexpr int NB = 64 * B_WAVES;
  if (f.fused) {  // the whole iteration in one launch (after the gain estimate, if any)
    if (f.est_gain) {
      const hipError_t e = launch_gain(fd, 1, it, gain_blocks(px), st);
      if (e != hipSuccess) return e;
    }
    const unsigned nt = (unsigned)(((f.h + FT - 1) / FT) * ((f.w + FT - 1) / FT));
    k_fused<<<nt, kFusedThreads, 0, st>>>(fd, it);
    return hipGetLastError();
  }
  if (f.est_gain) {  // this iteration's gain, then S everywhere
    const hipError_t e = launch_gain(fd, 1, it, gain_blocks(px), st);
    if (e != hipSuccess) return e;
    k_frame<TH, NT, 0><<<nb, NT, 0, st>>>(fd, it);
  } else if (it == 0) {
    k_frame<TH, NT, 0><<<nb, NT, 0, st>>>(fd, it);
  } else {
    sparse_launch<3>(fd, it, ns, st);
  }
  k_frame<8, NB, 3><<<(unsigned)f.tiles_b, NB, 0, st>>>(fd, it);
  if (f.full_sp) k_frame<TH, NT, 1><<<nb, NT, 0, st>>>(fd, it);
  sparse_launch<0>(fd, it, ns, st);
  sparse_launch<2>(fd, it, ns, st);
  k_frame<8, NB, 2><<<(unsigned)f.tiles_b, NB, 0, st>>>(fd, it);
  sparse_launch<1>(fd, it, ns, st);
  if (it == f.niter - 1) k_frame<8, NB, 5><<<(unsigned)f.tiles_b, NB, 0, st>>>(fd, it);
  return hipGetLastError();
}

template <int TH, int NT>
static hipError_t queue_pass_t(const QueueArgs& a, int pass, int it, int mode, hipStream_t st) {
  constexpr int NB = 64 * B_WAVES;
  if (a.blocks <= 0) return hipSuccess;
  if (mode == kModeGrid) {
    switch (pass) {
      case kPassA1: k_grid<TH, NT, 0><<<a.blocks, NT, 0, st>>>(a.frames, a.tile_base, a.nframes, it); break;
      case kPassSC: k_grid<8, NB, 3><<<a.blocks, NB, 0, st>>>(a.frames, a.tile_base_b, a.nframes, it); break;
      case kPassOut: k_grid<8, NB, 5><<<a.blocks, NB, 0, st>>>(a.frames, a.tile_base_b, a.nframes, it); break;
      default: k_grid<8, NB, 2><<<a.blocks, NB, 0, st>>>(a.frames, a.tile_base_b, a.nframes, it); break;
    }
    return hipGetLastError();
  }
  unsigned int* cur = a.cursors + 8 * a.cursor_slot;
  switch (pass) {
    case kPassA1: k_queue<TH, NT, 0><<<a.blocks, NT, 0, st>>>(a.frames, a.tile_base, a.nframes, it, cur); break;
    case kPassSC: k_queue<8, NB, 3><<<a.blocks, NB, 0, st>>>(a.frames, a.tile_base_b, a.nframes, it, cur); break;
    case kPassOut: k_queue<8, NB, 5><<<a.blocks, NB, 0, st>>>(a.frames, a.tile_base_b, a.nframes, it, cur); break;
    default:
      k_queue<8, NB, 2><<<a.blocks, NB, 0, st>>>(a.frames, a.tile_base_b, a.nframes, it, cur);
      break;
  }
  return hipGetLastError();
}

template <int TH, int NT>
static int queue_blocks_t(int pass) {
  int per_cu = 0;
  hipError_t e;
  switch (pass) {
    case kPassA1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_queue<TH, NT, 0>, NT, 0); break;
    case kPassSC:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_queue<8, 64 * B_WAVES, 3>,
                                                       64 * B_WAVES, 0);
      break;
    case kPassOut:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_queue<8, 64 * B_WAVES, 5>,
                                                       64 * B_WAVES, 0);
      break;

    default:
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_queue<8, 64 * B_WAVES, 2>,
                                                       64 * B_WAVES, 0);
      break;
  }
  if (e != hipSuccess || per_cu < 1) per_cu = 1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus < 1)
    cus = 256;
  return per_cu * cus;
}

TileShape tile_shape(int cfg) {
  switch (cfg) {
    case 1: return TileShape{32, 64};
    case 2: return TileShape{8, 64};
    default: return TileShape{16, 64};
  }
}

hipError_t launch_init(unsigned long long* n_new, int niter, int* status, unsigned int* counts,
                       int* stamps, int64_t nstamps, hipStream_t st) {
  k_init<<<1, 256, 0, st>>>(n_new, niter, status, counts, stamps, nstamps);
  return hipGetLastError();
}

hipError_t launch_iteration(const FrameDev& f, const FrameDev* fd, int it, int cfg,
                            hipStream_t st) {
  (void)sparse_blocks();  // the device query runs once, before any capture
  switch (cfg) {
    case 1: return frame_iter_t<32, 256>(f, fd, it, st);
    case 2: return frame_iter_t<8, 128>(f, fd, it, st);
    default: return frame_iter_t<16, 256>(f, fd, it, st);
  }
}

hipError_t launch_put_frame(const FrameDev& f, FrameDev* dst, hipStream_t st) {
  k_put_frame<<<1, 64, 0, st>>>(f, dst);
  return hipGetLastError();
}

void prime_launch_config() { (void)s1_batch_blocks(); }

hipError_t launch_queue_init(const QueueArgs& a, int ncursors, int zero_counters,
                             hipStream_t st) {
  k_batch_init<<<a.nframes > 0 ? a.nframes : 1, 256, 0, st>>>(a.frames, a.nframes, a.cursors,
                                                                ncursors, zero_counters);
  return hipGetLastError();
}

hipError_t launch_queue_pass(const QueueArgs& a, int pass, int it, int cfg, int mode,
                             hipStream_t st) {
  const unsigned ns = (unsigned)sparse_blocks();
  switch (pass) {
    case kPassGain: return launch_gain(a.frames, a.nframes, it, a.blocks, st);
    case kPassUS: k_sparse_queue<3><<<ns, 256, 0, st>>>(a.frames, a.nframes, it); return hipGetLastError();
    case kPassS1:
      k_sparse_queue<0><<<(unsigned)s1_batch_blocks(), 256, 0, st>>>(a.frames, a.nframes, it);
      return hipGetLastError();
    case kPassSG: k_sparse_queue<2><<<ns, 256, 0, st>>>(a.frames, a.nframes, it); return hipGetLastError();
    case kPassS2: k_sparse_queue<1><<<ns, 256, 0, st>>>(a.frames, a.nframes, it); return hipGetLastError();
    default: break;
  }
  switch (cfg) {
    case 1: return queue_pass_t<32, 256>(a, pass, it, mode, st);
    case 2: return queue_pass_t<8, 128>(a, pass, it, mode, st);
    default: return queue_pass_t<16, 256>(a, pass, it, mode, st);
  }
}

// Counts the binary32 inputs with bit patterns in [lo, hi] where sqrt_rn_fast
// and the compiler's correctly rounded sqrtf differ in any bit.
__global__ void k_check_sqrt(uint32_t lo, uint32_t hi, unsigned long long* bad) {
  unsigned long long n = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t b = (uint64_t)lo + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; b <= hi;
       b += stride) {
    const float x = __uint_as_float((uint32_t)b);
    n += __float_as_uint(sqrt_rn_fast(x)) != __float_as_uint(sqrtf(x)) ? 1ull : 0ull;
  }
  for (int off = 32; off > 0; off >>= 1) n += __shfl_down(n, off);
  if ((threadIdx.x & 63) == 0 && n) atomicAdd(bad, n);
}

hipError_t launch_check_sqrt(uint32_t lo, uint32_t hi, unsigned long long* bad, hipStream_t st) {
  k_check_sqrt<<<4096, 256, 0, st>>>(lo, hi, bad);
  return hipGetLastError();
}

hipError_t launch_u16_to_f32(const uint16_t* in, float* out, int64_t n, hipStream_t st) {
  const int64_t want = (n + 255) / 256;
  const unsigned blocks = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
  k_u16_to_f32<<<blocks, 256, 0, st>>>(in, out, n);
  return hipGetLastError();
}

int queue_blocks(int cfg, int pass) {  // pass: a dense pass (dense_slot(pass) >= 0)
  (void)s1_batch_blocks();  // query the device here, never inside a graph capture
  switch (cfg) {
    case 1: return queue_blocks_t<32, 256>(pass);
    case 2: return queue_blocks_t<8, 128>(pass);
    default: return queue_blocks_t<16, 256>(pass);
  }
}

}  // namespace lac
