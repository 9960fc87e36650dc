// Host-side launch entry points of the kernels (internal to the library).
#pragma once
#include <hip/hip_runtime.h>

#include "lacosmic_device.h"

namespace lac {

struct TileShape {
  int th, tw;
};

// Tile shapes compiled into the library; cfg indexes them.
constexpr int kNumTileCfgs = 3;
constexpr int kDefaultTileCfg = 1;  // 32 x 64: fastest single-frame shape measured on MI355X
// Pass B works on tiles of kBWaves strips of kBStrip rows by one strip
// column (strip_ncols); one wave streams down each strip.
constexpr int kBWaves = 4;
// Pass-B strips of an h x w frame (the size of each per-strip stamp array in
// the workspace).
inline int64_t max_strips(int64_t h, int64_t w) {
  return ((h + kBStrip - 1) / kBStrip) * strip_ncols((int)((w + 63) / 64));
}
TileShape tile_shape(int cfg);

// Passes of one iteration in launch order.  GAIN runs only for frames
// without a supplied gain, A1 in iteration 0 (and in every iteration of
// those frames), US in iterations >= 1, OUT in the last; A1, SC, B and OUT
// are dense (tile) passes, GAIN a chain of launches over every pixel, the
// others sparse (grid-stride over per-frame item lists).
constexpr int kPassGain = 0; // gain estimate of the iteration (no gain supplied)
constexpr int kPassUS = 1;   // S update near the pixels the previous iteration rewrote
constexpr int kPassA1 = 2;   // S and the candidate plane at every pixel
constexpr int kPassSC = 3;   // candidate list, per-iteration bit planes cleared
constexpr int kPassS1 = 4;   // S', G1, G2 and the objlim test at the candidates
constexpr int kPassSG = 5;   // G2 around the confirmed candidates
constexpr int kPassB = 6;    // growth, mask, recompute list
constexpr int kPassS2 = 7;   // replacement
constexpr int kPassOut = 8;  // mask bytes (last iteration)
constexpr int kPassesPerIter = 9;
// The dense passes each take 8 queue cursors per launch: slot of a pass.
constexpr int kDenseSlots = 4;
inline int dense_slot(int pass) {
  switch (pass) {
    case kPassA1: return 0;
    case kPassSC: return 1;
    case kPassB: return 2;
    case kPassOut: return 3;
    default: return -1;
  }
}
// Whether a launch of the pass is needed for frames at iteration it of
// niter (est: some frame estimates its gain); frames that share a launch at
// different iterations skip what does not apply to them.
inline bool pass_runs(int pass, int it, int niter, bool est = false) {
  switch (pass) {
    case kPassGain: return est;
    case kPassUS: return it > 0;
    case kPassA1: return it == 0 || est;
    case kPassOut: return it == niter - 1;
    default: return true;
  }
}

// Zero one frame's niter + 1 counters (per-iteration new pixels, then the
// unreplaced pixels), list lengths, status word and nstamps strip stamps.
hipError_t launch_init(unsigned long long* n_new, int niter, int* status, unsigned int* counts,
                       int* stamps, int64_t nstamps,
                       hipStream_t st);

// One iteration of one frame (A2 too with the full-S' flag), one block per
// tile for the dense passes and a grid-stride launch for the sparse ones.  f
// is the host copy of the frame record (grid sizes), fd the device copy the
// kernels read (launch_put_frame stores it).
hipError_t launch_iteration(const FrameDev& f, const FrameDev* fd, int it, int cfg,
                            hipStream_t st);
// Stores the frame record f at dst (device memory), in stream order.
hipError_t launch_put_frame(const FrameDev& f, FrameDev* dst, hipStream_t st);
// Queries the device properties the launchers use (once per process), so that
// no such query runs during a graph capture.
void prime_launch_config();

// Launch forms over many frames: a persistent grid pulling tiles from a
// queue, or one block per tile.
constexpr int kModeQueue = 0;
constexpr int kModeGrid = 1;

// Tile-queue / grid launches over many frames.  frames / tile_base /
// cursors are device arrays; tile_base has nframes + 1 entries (prefix sums
// of the frames' tile counts for the launch's tile shape).  Each pass launch
// uses its own 8 cursors (one per XCD range): cursors + 8 * cursor_slot.
struct QueueArgs {
  const FrameDev* frames;      // (kPassGain: blocks = gain blocks per frame)
  const int* tile_base;    // TH x 64 tiles (A1)
  const int* tile_base_b;  // pass-B tiles (SC, B, OUT)
  int nframes;
  unsigned int* cursors;
  int cursor_slot;
  int blocks;  // persistent grid size (queue mode) or the pass's tile count (grid mode)
};

// Zero the cursors [0, ncursors) and, if zero_counters, every frame's
// counters and status.
hipError_t launch_queue_init(const QueueArgs& a, int ncursors, int zero_counters,
                             hipStream_t st);
// pass: one of kPass*.  it >= 0: every frame runs iteration it; it < 0:
// each frame runs its own FrameDev::it (a pass that does not apply to a
// frame's iteration does nothing for it).
hipError_t launch_queue_pass(const QueueArgs& a, int pass, int it, int cfg, int mode,
                             hipStream_t st);
// Gain estimate of iteration it (it < 0: each frame's own FrameDev::it) for
// the frames of a table (one frame: its record) that estimate their gain:
// a reset, then up to 5 sigma-clipping rounds of three passes and the final
// sums, each launch nbx x nframes blocks; the result lands in each frame's
// per-iteration noise constants.
hipError_t launch_gain(const FrameDev* frames, int nframes, int it, int nbx, hipStream_t st);
// Blocks per frame of the gain passes for a frame of the given pixel count.
int gain_blocks(int64_t pixels);
// Exact uint16 -> float32 widening of n values.
hipError_t launch_u16_to_f32(const uint16_t* in, float* out, int64_t n, hipStream_t st);
hipError_t launch_check_sqrt(uint32_t lo, uint32_t hi, unsigned long long* bad, hipStream_t st);
// Grid size that keeps every CU full for the given dense pass (occupancy x
// CUs).
int queue_blocks(int cfg, int pass);

}  // namespace lac
