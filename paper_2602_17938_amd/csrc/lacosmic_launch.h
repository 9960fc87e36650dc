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
TileShape tile_shape(int cfg);

// Zero the per-iteration counters and the status word.
hipError_t launch_init(unsigned long long* n_new, int niter, int* status, hipStream_t st);

// One iteration (pass A then pass B) of one frame, one block per tile.
hipError_t launch_iteration(const FrameDev& f, int it, int cfg, hipStream_t st);

}  // namespace lac
