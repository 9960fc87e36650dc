// Device-side data structures shared by the kernels and the host runtime.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lac {

// Pass-B strip columns of a frame whose rows hold wpr 64-pixel words.  A row
// of at most 64 words is one column, lane l of a wave holding word l (the
// frame's edges supply the zero neighbours).  Wider rows split into columns
// of 62 words; lanes 0 and 63 then hold the neighbouring columns' edge words.
constexpr int kStripWords = 62;
// Rows of a pass-B strip (one wave each): the pass streams kBStrip + 16 rows
// (an 8-row halo each side) as one fully unrolled sequence.  16 rows measured
// fastest on MI355X: enough waves for a frame, halos recomputed twice over.
constexpr int kBStrip = 16;
static_assert(kBStrip % 4 == 0 && kBStrip >= 8,
              "strips start at even rows (pass B lists 2x2 blocks per strip) and a "
              "strip's 8-row halo lies in its neighbour strips");
__host__ __device__ inline int strip_ncols(int wpr) {
  return wpr <= 64 ? 1 : (wpr + kStripWords - 1) / kStripWords;
}

// Per-iteration list lengths: counts[kCntPerIter * it + k].
constexpr int kCntCand = 0;   // candidates (S > sigclip), listed by pass SC
constexpr int kCntDirty = 1;  // mask pixels to (re)compute, listed by pass B
constexpr int kCntConf = 2;   // confirmed candidates (B1 bits), listed by SC and S1
constexpr int kCntRecomp = 3; // 2x2 blocks whose S the next iteration recomputes, listed by pass B
constexpr int kCntPerIter = 4;

// Noise-model constants of one iteration (from a supplied gain, or from the
// gain estimated for that iteration).
struct NoiseCoef {
  float gain;
  float inv_gain;  // 1 / gain when gain is a power of two (then exact), else 0
  int fast_sqrt;   // the noise variance is never below 2^-96 (sqrt_rn_fast applies)
  int valid;       // estimated gains: 0 when there was no estimate (gain 1 used)
};

// State of one frame's gain estimate (sigma clipping and exact sums), reset
// at the start of each iteration; see lacosmic_gain.h.
struct GainWork {
  unsigned int hist[4096];          // histogram of the current selection pass
  unsigned long long acc[5][256];   // exact-sum accumulators by exponent
  uint32_t klo, khi;                // kept values: keys in [klo, khi]
  uint32_t prefix, rank;            // median search: key digits found, rank left
  int round;                        // clipping rounds applied
  int done;                         // this iteration's estimate is final
  unsigned int blocks_done;         // blocks of the current pass that finished
  int pad;
  long long n_prev, n_cur;          // kept values before / in the current round
  double mean, var;                 // of the current round's kept values
};

// One frame's device state for one run.  The single-frame path passes it by
// value; the batched and serving paths keep an array of them in device
// memory.  Bit planes hold one bit per pixel: bit i of word j of row y is
// pixel (y, 64 j + i); rows are wpr words long; bits past the frame's last
// column are zero.
struct FrameDev {
  const float* img;            // input, ADU, h*w (read in iteration 0 only)
  const uint16_t* img16;       // the input as uint16 ADU instead (then img is unused), or null
  float* clean;                // current image C; iteration 0 writes all of it
  float* splane;               // S, h*w: all of it in iteration 0, then kept up to date
  float* sp;                   // S' at the candidates (every pixel with full_sp), h*w
  uint64_t* g1;                // S' > sigclip (exact at the candidates)
  uint64_t* g2;                // S' > sigfrac * sigclip (exact where growth can reach)
  uint64_t* b1;                // candidates passing steps 4-5
                               // (the three kept across iterations outside R4)
  uint64_t* cb;                // candidates S > sigclip, kept up to date with S
  uint64_t* mbits[2];          // cumulative mask, ping-pong
  uint64_t* dirty;             // mask pixels whose replacement is recomputed this iteration
  uint64_t* rs;                // pixels within 2 of a dirty one: S changes only there
  uint64_t* r4;                // pixels within 4 of a dirty one: S' and the objlim inputs
                               // change only there
  uint8_t* out_mask;           // final cumulative mask, h*w bytes (0/1)
  unsigned long long* n_new;   // new mask pixels per iteration [niter], then one more
                               // counter, n_new[niter]: mask pixels whose 5x5 window holds
                               // no un-flagged cell (they keep their value)
  int* status;                 // bit 0: non-finite input seen
  unsigned int* counts;        // list lengths per iteration [kCntPerIter * niter]
  int* list;                   // candidates, then dirty mask pixels (y*w + x), h*w
  int* conf;                   // confirmed candidates, then the next iteration's US blocks, h*w
  // Per pass-B strip (index (y0 / kBStrip) * strip_ncols(wpr) + strip column),
  // iteration stamps it + 1 (0: none): b1s, the strip holds a B1 bit in
  // iteration it; bq, pass B of iteration it found no B1 bit within reach of
  // the strip, so it only carried the mask over and cleared R4 there.
  int* b1s;
  int* bq;
  GainWork* gw;                // gain estimate state (est_gain frames)
  NoiseCoef* coef;             // per-iteration noise constants of est_gain frames [niter]
  int h, w, wpr;
  unsigned int w_mul;          // row of pixel index n < 2^31: n / w == (n * w_mul) >> w_shr
  int w_shr;
  float gain, rn2, sigclip, lo, objlim;  // rn2 = readnoise^2, lo = sigfrac*sigclip (binary32)
  float readnoise;
  float inv_gain;              // 1 / gain when gain is a power of two (then exact), else 0
  int fast_sqrt;               // the noise variance is never below 2^-96 (sqrt_rn_fast applies)
  int niter;
  int early_stop;
  int full_sp;                 // compute and keep S' at every pixel
  int est_gain;                // no gain supplied: estimated at each iteration, and every
                               // iteration runs the dense passes (S changes everywhere)
  int fused;                   // single frame: one fused launch per iteration (small frames)
  int sepmed;                  // detection medians separable (row medians, then column medians)
  int tiles_x;                 // tiles per row for the launch's tile shape
  int tiles;                   // tiles per frame
  int tiles_b;                 // pass-B tiles per frame (bands x word columns)
  int it;                      // serving only: the iteration this step runs
};

}  // namespace lac
