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
// Pass B works on tiles of kBWaves strips of FrameDev::bstrip rows by kBWords
// 64-pixel words; one wave streams down each strip.  Short strips give a
// single frame enough waves; long ones waste less on the 2-row halos.
constexpr int kBWords = 62;
constexpr int kBWaves = 4;
constexpr int kBStripSingle = 16;  // single-frame path
constexpr int kBStripMulti = 64;   // batched and serving paths
TileShape tile_shape(int cfg);

// Zero one frame's per-iteration counters and its status word.
hipError_t launch_init(unsigned long long* n_new, int niter, int* status, hipStream_t st);

// One iteration (A1, A2, S1, B, S2) of one frame, one block per tile for the
// dense passes and a grid-stride launch over the lists for the sparse ones.
hipError_t launch_iteration(const FrameDev& f, int it, int cfg, hipStream_t st);

// Launch forms over many frames: a persistent grid pulling tiles from a
// queue, or one block per tile.
constexpr int kModeQueue = 0;
constexpr int kModeGrid = 1;

// Tile-queue / grid launches over many frames.  frames / tile_base /
// cursors are device arrays; tile_base has nframes + 1 entries (prefix sums
// of the frames' tile counts for the launch's tile shape).  Each pass launch
// uses its own 8 cursors (one per XCD range): cursors + 8 * cursor_slot.
struct QueueArgs {
  const FrameDev* frames;
  const int* tile_base;    // pass-A tiles (A1, A2)
  const int* tile_base_b;  // pass-B tiles
  int nframes;
  unsigned int* cursors;
  int cursor_slot;
  int blocks;  // persistent grid size (queue mode) or the pass's tile count (grid mode)
};

// Zero the cursors [0, ncursors) and, if zero_counters, every frame's
// counters and status.
hipError_t launch_queue_init(const QueueArgs& a, int ncursors, int zero_counters,
                             hipStream_t st);
// pass: 0 = A1, 1 = A2, 2 = B (tile queue), 3 = S1, 4 = S2 (grid-stride over
// every frame's list).  Order within an iteration: 0, 1, 3, 2, 4.
// it >= 0: every frame runs iteration it; it < 0: each frame runs its own
// FrameDev::it.
hipError_t launch_queue_pass(const QueueArgs& a, int pass, int it, int cfg, int mode,
                             hipStream_t st);
// Exact uint16 -> float32 widening of n values.
hipError_t launch_u16_to_f32(const uint16_t* in, float* out, int64_t n, hipStream_t st);
// Grid size that keeps every CU full for the given pass (occupancy x CUs).
int queue_blocks(int cfg, int pass);

}  // namespace lac
