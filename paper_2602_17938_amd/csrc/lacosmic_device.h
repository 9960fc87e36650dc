// Device-side data structures shared by the kernels and the host runtime.
#pragma once
#include <stdint.h>

namespace lac {

// One frame's device state for one run.  The plain path passes it by value;
// the batched and serving paths keep an array of them in device memory.
struct FrameDev {
  const float* img;            // input, ADU, h*w (read in iteration 0 only)
  float* clean;                // current image C; iteration 0 writes all of it
  float* sp;                   // S' plane of the latest iteration, h*w
  uint8_t* cand;               // candidate map of steps 4-5, h*w (0/1)
  uint8_t* mbuf[2];            // cumulative mask ping-pong, h*w each
  uint8_t* out_mask;           // final cumulative mask, h*w (0/1)
  unsigned long long* n_new;   // new mask pixels per iteration [niter]
  int* status;                 // bit 0: non-finite input seen
  int h, w;
  float gain, rn2, sigclip, lo, objlim;  // rn2 = readnoise^2, lo = sigfrac*sigclip (binary32)
  int niter;
  int early_stop;
  int tiles_x;                 // tiles per row for the launch's tile shape
  int tiles;                   // tiles per frame
  int it;                      // serving only: the iteration this step runs
  int pad_;
};

}  // namespace lac
