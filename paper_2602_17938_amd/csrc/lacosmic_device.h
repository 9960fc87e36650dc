// Device-side data structures shared by the kernels and the host runtime.
#pragma once
#include <stdint.h>

namespace lac {

// One frame's device state for one run.  The single-frame path passes it by
// value; the batched and serving paths keep an array of them in device
// memory.  Bit planes hold one bit per pixel: bit i of word j of row y is
// pixel (y, 64 j + i); rows are wpr words long; bits past the frame's last
// column are zero.
struct FrameDev {
  const float* img;            // input, ADU, h*w (read in iteration 0 only)
  float* clean;                // current image C; iteration 0 writes all of it
  float* splane;               // S of the current iteration, h*w
  float* sp;                   // S' of the current iteration, h*w
  uint64_t* g1;                // S' > sigclip
  uint64_t* g2;                // S' > sigfrac * sigclip
  uint64_t* b1;                // candidates of steps 4-5
  uint64_t* mbits[2];          // cumulative mask, ping-pong
  uint8_t* out_mask;           // final cumulative mask, h*w bytes (0/1)
  unsigned long long* n_new;   // new mask pixels per iteration [niter]
  int* status;                 // bit 0: non-finite input seen
  unsigned int* counts;        // [0]: candidates listed, [1]: flagged pixels listed
  int* list;                   // pixel indices (y*w + x) for the sparse passes, h*w
  int h, w, wpr;
  float gain, rn2, sigclip, lo, objlim;  // rn2 = readnoise^2, lo = sigfrac*sigclip (binary32)
  float tmin;                  // min(sigclip, lo): S' is needed only where S > tmin
  int niter;
  int early_stop;
  int full_sp;                 // compute and keep S' at every pixel
  int tiles_x;                 // tiles per row for the launch's tile shape
  int tiles;                   // tiles per frame
  int tiles_b;                 // pass-B tiles per frame (bands x word columns)
  int bstrip;                  // pass-B rows per wave
  int it;                      // serving only: the iteration this step runs
};

}  // namespace lac
