// Tile-level device code of the L.A.Cosmic iteration for gfx950 (MI355X).
//
// Dense passes work on tiles of TH x 64 output pixels (a tile row is one
// 64-bit word of every bit plane); sparse passes run over per-frame pixel
// lists.  One iteration:
//
//  A1 (iteration 0, steps 1-3a): stages C over the tile plus a 2-pixel ring
//     (clamped) in LDS and computes, per pixel, the Laplacian edge image L,
//     med5(C), the noise model N and S = L / (2N); the 5x5 medians of a 4x2
//     block of pixels (2x2 on tiles under 32 rows) share one selection
//     network.  Writes S and the bit
//     plane CB = [S > sigclip] of the candidates (S' <= S, see below).
//  US (iterations >= 1, sparse): S at a pixel reads C within 2 pixels, and C
//     changes only at the pixels the previous iteration's S2 rewrote, so S and
//     CB are recomputed only within 2 pixels of those, the set RS.  Pass B
//     of the previous iteration lists the aligned 2x2 blocks that hold an RS
//     pixel; US computes a block's four S values from one 6x6 patch with the
//     shared 2x2 median network (a block pixel outside RS gets its stored
//     value again).
//  SC (bit-parallel, one wave per strip of row words): lists the candidates
//     for S1 -- every pixel of CB in iteration 0, then only those inside R4 --
//     and clears G1, G2, B1 where S1 and SG recompute them (everywhere in
//     iteration 0, inside R4 later; elsewhere the bits of the previous
//     iteration stand, and its B1 pixels are listed as confirmed).
//  A2 (only with the full-S' flag): S' = S - med5(S) at every pixel.
//  S1 (steps 3b-5, sparse over the candidates): S' = S - med5(S) (clamped on
//     S's own grid); G2 = [S' > sigfrac*sigclip], G1 = [S' > sigclip]; where
//     G1 holds, the fine-structure ratio S' / max((med3 - med7(med3)) / N,
//     0.01) > objlim sets B1 and lists the pixel as confirmed.
//  SG (step 6 input, sparse): the growth reads G2 only next to B2 =
//     dil3(B1) & G1, within 2 of a B1 pixel, so G2 is completed there: in
//     the 5x5 box of each confirmed pixel, where a G1 pixel links the box
//     pixel to it, at sigfrac*sigclip < S <= sigclip.
//  B  (step 6): bit-parallel on 64-bit row words, one wave streaming down a
//     strip of rows of 62 words: B2 = dil3(B1) & G1, B3 = dil3(B2) & G2,
//     M' = M | B3 (ping-pong bit planes), the count of new pixels, the list of
//     mask pixels whose replacement can change -- those within 2 pixels of a
//     new one (every mask pixel in iteration 0) -- the 2x2 blocks holding a
//     pixel of RS (within 2 of those) for the next iteration's US, and the
//     plane R4 of
//     pixels within 2 of RS for the next iteration's S1.
//  S2 (step 7, sparse): each listed pixel takes the lower median of its
//     un-flagged clamped 5x5 neighbours (a sorting network over 25 keys with
//     the flagged ones pushed to the top).  C is updated in place only at
//     flagged pixels and nothing reads a flagged pixel's value, so there is
//     no race on C.
//  OUT (last iteration): the final mask plane expanded to bytes.
//
// Exactness of the sparse forms.  S >= +0 (a clipped Laplacian over a
// positive noise), so med5(S) >= +0 and S' = S - med5(S) <= S after
// rounding: S' > t is impossible where S <= t.  Un-flagged pixels never
// change, so a mask pixel's replacement, a function of the un-flagged values
// in its window, changes only when a pixel of that window joins the mask.
// A value computed from C within radius r of a pixel (S: 2; S' and the
// objlim test: 4) can only change where C changed within r.
//
// Medians run on 32-bit keys whose signed order is the float order, with
// min/max networks (v_min3/v_max3/v_med3_i32): they select exactly.  All
// arithmetic is binary32 in the same expression order as a plain evaluation
// of the method, compiled with -ffp-contract=off and IEEE division / sqrt.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lacosmic_device.h"
#include "lacosmic_mem.h"
#include "median_net.gen.h"

namespace lac {

constexpr int TW = 64;                    // tile width = one bit-plane word
constexpr int KEY_EXCLUDED = 0x7fffffff;  // above every finite or infinite float key

__device__ __forceinline__ int fkey(float f) {
  const int b = __float_as_int(f);
  return b ^ ((b >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float funkey(int k) {
  return __int_as_float(k ^ ((k >> 31) & 0x7fffffff));
}
__device__ __forceinline__ int clampi(int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); }
__device__ __forceinline__ int kmin3(int a, int b, int c) { return kmin(kmin(a, b), c); }
__device__ __forceinline__ int kmax3(int a, int b, int c) { return kmax(kmax(a, b), c); }
__device__ __forceinline__ int kmed3(int a, int b, int c) {
  return kmax(kmin(a, b), kmin(kmax(a, b), c));
}
// Loads the N consecutive floats p[i .. i + N) with as few 4-byte-aligned
// vector loads as fit (dwordx4, then dwordx2, then dword): a lane's window
// row costs one memory instruction per four values instead of one per value.
// Reads nothing outside [i, i + N).
typedef float f4u __attribute__((ext_vector_type(4), aligned(4)));
typedef float f2u __attribute__((ext_vector_type(2), aligned(4)));
template <int N>
__device__ __forceinline__ void ldg_row(const float* p, int64_t i, float* out) {
  typedef const __attribute__((address_space(1))) f4u* g4;
  typedef const __attribute__((address_space(1))) f2u* g2;
  typedef const __attribute__((address_space(1))) float* g1;
  int k = 0;
#pragma unroll
  for (; k + 4 <= N; k += 4) {
    const f4u v = *(g4)(p + i + k);
    out[k] = v.x;
    out[k + 1] = v.y;
    out[k + 2] = v.z;
    out[k + 3] = v.w;
  }
  if constexpr (N % 4 >= 2) {
    const f2u v = *(g2)(p + i + k);
    out[k] = v.x;
    out[k + 1] = v.y;
    k += 2;
  }
  if constexpr (N % 2 == 1) out[k] = *(g1)(p + i + k);
}
// ------------------------------------------------------------------ separable medians
// The separable approximation of a k x k median (LACOSMIC_F_SEPMED, the
// comparison point of astroscrappy's sepmed option): the median of each row
// of the window, then the median of those row medians.  On clamped windows
// the row medians are those of the clamped rows, so this is the two-pass
// filter -- rows, then columns, each clamped on its own grid.
//
// 5x5 of a 2x2 block of windows over a 6x6 patch (row-major): the row
// medians of each patch row for both output columns, then the column
// medians; o = {(0,0), (0,1), (1,0), (1,1)}.
__device__ __forceinline__ void sep25_2x2(const int* v, int* o) {
  int r0[6], r1[6];
#pragma unroll
  for (int a = 0; a < 6; ++a) {
    r0[a] = medline5(v + a * 6);
    r1[a] = medline5(v + a * 6 + 1);
  }
  o[0] = medline5(r0);
  o[1] = medline5(r1);
  o[2] = medline5(r0 + 1);
  o[3] = medline5(r1 + 1);
}
// 5x5 window (25 keys, row-major).
__device__ __forceinline__ int sep25(const int* v) {
  int r[5];
#pragma unroll
  for (int a = 0; a < 5; ++a) r[a] = medline5(v + a * 5);
  return medline5(r);
}
// 3x3 window (9 keys, row-major).
__device__ __forceinline__ int sep9(const int* v) {
  return kmed3(kmed3(v[0], v[1], v[2]), kmed3(v[3], v[4], v[5]), kmed3(v[6], v[7], v[8]));
}
// 7x7 window (49 keys, row-major).
__device__ __forceinline__ int sep49(const int* v) {
  int r[7];
#pragma unroll
  for (int a = 0; a < 7; ++a) r[a] = medline7(v + a * 7);
  return medline7(r);
}
// The detection medians of a frame: classic, or separable with sep (a
// frame-uniform choice).
__device__ __forceinline__ void med25_block(const int* v, int* o, int sep) {
  if (sep)
    sep25_2x2(v, o);
  else
    med25_2x2(v, o);
}
__device__ __forceinline__ int med25_of(const int* v, int sep) { return sep ? sep25(v) : med25(v); }
__device__ __forceinline__ int med49_of(const int* v, int sep) { return sep ? sep49(v) : med49(v); }
__device__ __forceinline__ int med9_of(const int* v, int sep) { return sep ? sep9(v) : med9(v); }

// Row of pixel index n (0 <= n < 2^31) of frame f, n / w, by a multiply and
// a shift with the frame's constants.
__device__ __forceinline__ int row_of(const FrameDev& f, int n) {
  return (int)(((unsigned long long)(unsigned int)n * f.w_mul) >> f.w_shr);
}
__device__ __forceinline__ bool finite_bits(float v) {
  return (__float_as_uint(v) & 0x7f800000u) != 0x7f800000u;
}

__device__ __forceinline__ const float* src_of(const FrameDev& f, int it) {
  return it == 0 ? f.img : f.clean;
}
__device__ __forceinline__ const uint64_t* mprev_of(const FrameDev& f, int it) {
  // selects rather than an index: a run-time index into the record's array
  // would keep the whole record in scratch memory
  return it == 0 ? nullptr : (((it - 1) & 1) ? f.mbits[1] : f.mbits[0]);
}
__device__ __forceinline__ uint64_t* mnext_of(const FrameDev& f, int it) {
  return (it & 1) ? f.mbits[1] : f.mbits[0];
}
// With early stop, iteration it is skipped when iteration it-1 added nothing.
__device__ __forceinline__ bool stopped(const FrameDev& f, int it) {
  return f.early_stop && it > 0 && ldg(f.n_new, it - 1) == 0ull;
}
__device__ __forceinline__ unsigned int* count_of(const FrameDev& f, int it, int k) {
  return f.counts + kCntPerIter * it + k;
}
// Pass-B strip of pixel row y and word column word (see FrameDev::b1s).
__device__ __forceinline__ int strip_cols(const FrameDev& f) { return strip_ncols(f.wpr); }
__device__ __forceinline__ int strip_of(const FrameDev& f, int y, int word) {
  return (y / kBStrip) * strip_cols(f) + (f.wpr <= 64 ? 0 : word / kStripWords);
}
// The word a lane of a strip's wave holds (strip column starting at word0)
// and whether the strip produces it (see strip_ncols).
__device__ __forceinline__ int strip_word(const FrameDev& f, int word0, int lane) {
  return f.wpr <= 64 ? lane : word0 - 1 + lane;
}
__device__ __forceinline__ bool strip_out_lane(const FrameDev& f, int word, int lane) {
  return f.wpr <= 64 ? lane < f.wpr : (lane >= 1 && lane <= kStripWords && word < f.wpr);
}
__device__ __forceinline__ unsigned long long lanes_below() {
  return (1ull << (threadIdx.x & 63)) - 1ull;
}

// Appends idx to the list of the counter it names (lanes with pred set); the
// lanes of a wave that append to one counter share one atomic.  Every active
// lane of the wave calls it.
__device__ __forceinline__ void wave_append(unsigned int* counter, int* list, int idx, bool pred) {
  const int lane = threadIdx.x & 63;
  unsigned long long pending = __ballot(pred);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const unsigned long long mine_ptr = (unsigned long long)counter;
    const unsigned long long lead_ptr = __shfl(mine_ptr, leader);
    const bool same = pred && mine_ptr == lead_ptr;
    const unsigned long long group = __ballot(same);
    unsigned int base = 0;
    if (lane == leader) base = atom_add(counter, (unsigned int)__popcll(group));
    base = __shfl(base, leader);
    if (same) stg(list, base + __popcll(group & lanes_below()), idx);
    pending &= ~group;
  }
}

// Step 1: Laplacian edge image at one pixel from its clamped 4-neighbourhood.
// The 2x replicated pixel has four sub-pixels; each applies the Laplacian
// kernel's taps on the replicated grid (-up, -left, +4 centre, -right, -down,
// summed in that order), is clipped at zero, and the four are averaged.
__device__ __forceinline__ float lap_edge(float c, float u, float d, float l, float r) {
  const float c4 = 4.0f * c;
  float l00 = ((((-u) - l) + c4) - c) - c;
  float l01 = ((((-u) - c) + c4) - r) - c;
  float l10 = ((((-c) - l) + c4) - c) - d;
  float l11 = ((((-c) - c) + c4) - r) - d;
  l00 = (l00 > 0.0f) ? l00 : 0.0f;
  l01 = (l01 > 0.0f) ? l01 : 0.0f;
  l10 = (l10 > 0.0f) ? l10 : 0.0f;
  l11 = (l11 > 0.0f) ? l11 : 0.0f;
  return (((l00 + l01) + l10) + l11) * 0.25f;
}

// Correctly rounded binary32 square root for x in [2^-96, +inf]: the
// hardware estimate s, then s - 1 ulp or s + 1 ulp where the fma residual
// x - s'*s shows the root lies beyond them.  These are the steps of the
// compiler's own sqrtf on this target without its rescaling of arguments
// below 2^-96 and its special case for zero, so on that range the results
// agree bit for bit (lacosmic_check_sqrt compares every such input).
__device__ __forceinline__ float sqrt_rn_fast(float x) {
  const float s = __builtin_amdgcn_sqrtf(x);
  const float sd = __int_as_float(__float_as_int(s) - 1);
  const float su = __int_as_float(__float_as_int(s) + 1);
  const float rd = __builtin_fmaf(-sd, s, x);
  const float ru = __builtin_fmaf(-su, s, x);
  const float r = (0.0f >= rd) ? sd : s;
  return (0.0f < ru) ? su : r;
}

// The noise-model constants of iteration it: those of the supplied gain, or
// those the gain estimate of that iteration stored.  They are frame-uniform;
// reading them through the first lane lets the compiler keep them in scalar
// registers and branch on them as uniform choices (a per-lane copy would turn
// the square root and division choices into divergent branches).
__device__ __forceinline__ NoiseCoef noise_coef(const FrameDev& f, int it) {
  NoiseCoef c;
  if (f.est_gain) {
    const NoiseCoef* cp = f.coef + it;
    c.gain = ldg(&cp->gain, 0);
    c.inv_gain = ldg(&cp->inv_gain, 0);
    c.fast_sqrt = ldg(&cp->fast_sqrt, 0);
    c.valid = ldg(&cp->valid, 0);
  } else {
    c.gain = f.gain;
    c.inv_gain = f.inv_gain;
    c.fast_sqrt = f.fast_sqrt;
    c.valid = 1;
  }
  c.gain = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(c.gain)));
  c.inv_gain = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(c.inv_gain)));
  c.fast_sqrt = __builtin_amdgcn_readfirstlane(c.fast_sqrt);
  c.valid = __builtin_amdgcn_readfirstlane(c.valid);
  return c;
}

// Step 2: noise model from med5(C), floored at 1e-4.  When the gain is a
// power of two its reciprocal is exact, and x / gain and x * (1 / gain) are
// the same correctly rounded value: the division becomes a multiplication
// (inv_gain != 0, a frame-uniform choice).
// The floor is taken on the median's key: keys order as the floats do and
// the floor is positive, so max(key, key(1e-4)) is the key of the floored
// value and, being non-negative, its bits are that float's bits.
// With fast_sqrt (the frame's smallest possible variance, at the floor, is at
// least 2^-96) the square root skips the small-argument path.  Both choices
// are frame-uniform.  FAST: the caller has checked that both are the fast
// ones (fast_sqrt and inv_gain != 0), so no pixel tests them again.
template <bool FAST = false>
__device__ __forceinline__ float noise_from_med(int m5key, const NoiseCoef& nc, float rn2) {
  const float m = __int_as_float(kmax(m5key, 0x38d1b717));  // 0x38d1b717: 1e-4f
  const float var = nc.gain * m + rn2;
  if constexpr (FAST) return sqrt_rn_fast(var) * nc.inv_gain;
  const float sd = nc.fast_sqrt ? sqrt_rn_fast(var) : sqrtf(var);
  return nc.inv_gain != 0.0f ? sd * nc.inv_gain : sd / nc.gain;
}
// Whether a frame's noise model takes both fast forms (a uniform choice).
__device__ __forceinline__ bool noise_fast(const NoiseCoef& nc) {
  return nc.fast_sqrt && nc.inv_gain != 0.0f;
}


// ------------------------------------------------------------------ A1
template <int TH>
struct SmemA1 {
  int ck[TH + 4][TW + 4];    // keys of C over the tile + 2; then the candidates
  float cf[TH + 4][TW + 4];  // C over the tile + 2
  float so[TH][TW];          // S of the tile, staged for a coalesced store
};

// A1 in iteration it: iteration 0 reads the input (float32, or uint16 ADU
// widened exactly) and writes C = its canonical copy; a frame without a
// supplied gain also runs A1 in later iterations (its noise model changes
// everywhere with the estimate), reading C.
template <int TH, int NT>
__device__ __forceinline__ void tile_a1(const FrameDev& f, int it, int y0, int x0, int tx_word, SmemA1<TH>& s) {
  static_assert(TW == 64 && NT % 64 == 0, "a wave covers one tile row");
  constexpr int NW = NT / 64;  // waves per block
  static_assert((TH + 4) % NW == 0 && TH % NW == 0, "rows split evenly over the waves");
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform
  const int h = f.h, w = f.w;
  const float* src = it == 0 ? f.img : f.clean;
  const uint16_t* src16 = it == 0 ? f.img16 : nullptr;
  // Staging, one row per wave at a time: the row base is wave-uniform, lane
  // l loads column x0 - 2 + l and lanes 0..3 also columns x0 + 62 .. 65
  // (clamped).  Every load is issued before the first LDS store.
  constexpr int R = (TH + 4) / NW;
  const int cxa = clampi(x0 - 2 + lane, w - 1), cxb = clampi(x0 + 62 + (lane & 3), w - 1);
  float va[R], vb[R];
  if (src16) {  // frame-uniform
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int ly = wv + k * NW;
      const int64_t row = (int64_t)clampi(y0 - 2 + ly, h - 1) * w;
      va[k] = (float)ldg(src16, row + cxa);
      vb[k] = (float)ldg(src16, row + cxb);
    }
  } else {
#pragma unroll
    for (int k = 0; k < R; ++k) {
      const int ly = wv + k * NW;
      const int64_t row = (int64_t)clampi(y0 - 2 + ly, h - 1) * w;
      va[k] = ldg(src, row + cxa);
      vb[k] = ldg(src, row + cxb);
    }
  }
  int bad = 0;
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int ly = wv + k * NW;
    const float a = va[k] + 0.0f;  // -0 becomes +0
    const float b = vb[k] + 0.0f;  // (every lane checks it: a pixel of the frame)
    bad |= !finite_bits(a) | !finite_bits(b);
    s.cf[ly][lane] = a;
    s.ck[ly][lane] = fkey(a);
    if (lane < 4) {
      s.cf[ly][64 + lane] = b;
      s.ck[ly][64 + lane] = fkey(b);
    }
  }
  if (bad) atom_or(f.status, 1);
  __syncthreads();
  // C starts as the canonical input (rows of the tile, coalesced)
  const bool col_in = x0 + lane < w;
  if (it == 0) {
#pragma unroll
    for (int k = 0; k < TH / NW; ++k) {
      const int ty = wv + k * NW;
      if (y0 + ty < h && col_in) stg(f.clean, (int64_t)(y0 + ty) * w + x0 + lane, s.cf[ty + 2][lane + 2]);
    }
  }
  const NoiseCoef nc = noise_coef(f, it);
  const float rn2 = f.rn2;
  // Each thread takes a block of BY x 2 outputs whose 5x5 medians share one
  // network: 4 x 2 (578 min/max, 72 per output) where the tile has one such
  // block per thread, else 2 x 2 (308, 77 per output).
  constexpr int BY = (TH / 4) * (TW / 2) == NT ? 4 : 2;
  for (int blk = tid; blk < (TH / BY) * (TW / 2); blk += NT) {
    const int by = (blk / (TW / 2)) * BY, bx = (blk % (TW / 2)) * 2;
    int v[(BY + 4) * 6];
#pragma unroll
    for (int a = 0; a < BY + 4; ++a)
#pragma unroll
      for (int b = 0; b < 6; ++b) v[a * 6 + b] = s.ck[by + a][bx + b];
    int m[BY * 2];
    if constexpr (BY == 4) {
      if (f.sepmed) {
        sep25_2x2(v, m);
        sep25_2x2(v + 12, m + 4);
      } else {
        med25_4x2(v, m);
      }
    } else {
      med25_block(v, m, f.sepmed);
    }
    // the noise model's form is chosen once per block, not at every output
    auto outputs = [&](auto fast) {
#pragma unroll
      for (int q = 0; q < BY * 2; ++q) {
        const int ly = by + (q >> 1) + 2, lx = bx + (q & 1) + 2;
        const float L = lap_edge(s.cf[ly][lx], s.cf[ly - 1][lx], s.cf[ly + 1][lx],
                                 s.cf[ly][lx - 1], s.cf[ly][lx + 1]);
        const float N = noise_from_med<decltype(fast)::value>(m[q], nc, rn2);
        s.so[ly - 2][lx - 2] = L / (2.0f * N);
      }
    };
    if (noise_fast(nc))
      outputs(std::true_type{});
    else
      outputs(std::false_type{});
  }
  __syncthreads();
  // S and CB, rows of the tile: the CB word of a row from one ballot
  const float sigclip = f.sigclip;
#pragma unroll
  for (int k = 0; k < TH / NW; ++k) {
    const int ty = wv + k * NW;
    const int gy = y0 + ty;
    const bool in = gy < h && col_in;
    const float S = s.so[ty][lane];
    if (in) stg(f.splane, (int64_t)gy * w + x0 + lane, S);
    const unsigned long long cw = __ballot(in && S > sigclip);
    if (lane == 0 && gy < h) stg(f.cb, (int64_t)gy * f.wpr + tx_word, (uint64_t)cw);
  }
  __syncthreads();  // the block's next tile reuses the LDS
}

// Combines 64-bit bit sets over runs of adjacent lanes that hold the same key
// (a word address; 0 for an inactive lane): afterwards the last lane of each
// run holds the OR of the run's sets and returns true.  A segmented
// Kogge-Stone scan: a lane only takes values from lanes of its own run.
// Every lane of the wave calls it.
__device__ __forceinline__ bool run_or(unsigned long long key, unsigned long long& a,
                                       unsigned long long& b) {
  const int lane = threadIdx.x & 63;
  const unsigned long long kprev = __shfl_up(key, 1);
  const bool head = lane == 0 || kprev != key;
  const unsigned long long heads = __ballot(head);
  const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
  const int start = 63 - __clzll(heads & upto);  // lane 0 is always a head
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned long long ua = __shfl_up(a, off), ub = __shfl_up(b, off);
    if (lane - off >= start) {
      a |= ua;
      b |= ub;
    }
  }
  return lane == 63 || ((heads >> (lane + 1)) & 1ull);
}

// US on the aligned 2x2 block with top-left pixel (qy, qx) (both even): S at
// its pixels inside the frame from C's clamped 6x6 patch (rows qy-2 .. qy+3,
// columns qx-2 .. qx+3), whose 5x5 windows and 4-neighbourhoods are those of
// the four pixels, and their CB bits.  The list puts the blocks of one word
// pair next to each other, so for each of the two CB rows a wave combines
// its lanes' bits (run_or) and one lane per word updates CB.  Every lane of
// the wave calls it; inactive lanes pass active = false.
__device__ __forceinline__ void update_s_quad(const FrameDev& f, const NoiseCoef& nc, int qy,
                                              int qx, bool active) {
  unsigned long long key0 = 0ull, set0 = 0ull, clr0 = 0ull;
  unsigned long long key1 = 0ull, set1 = 0ull, clr1 = 0ull;
  if (active) {
    const int h = f.h, w = f.w;
    const float* C = f.clean;
    int v[36];
    float L[4];
    {
      float c[36];
      if (qy >= 2 && qy + 3 < h && qx >= 2 && qx + 3 < w) {  // no clamping: whole rows
#pragma unroll
        for (int a = 0; a < 6; ++a) ldg_row<6>(C, (int64_t)(qy - 2 + a) * w + (qx - 2), c + a * 6);
      } else {
#pragma unroll
        for (int a = 0; a < 6; ++a) {
          const int64_t row = (int64_t)clampi(qy - 2 + a, h - 1) * w;
#pragma unroll
          for (int b = 0; b < 6; ++b) c[a * 6 + b] = ldg(C, row + clampi(qx - 2 + b, w - 1));
        }
      }
#pragma unroll
      for (int k = 0; k < 36; ++k) c[k] += 0.0f;
      // the Laplacians first, so the float patch dies before the network runs
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int k = ((q >> 1) + 2) * 6 + (q & 1) + 2;  // the pixel's patch index
        L[q] = lap_edge(c[k], c[k - 6], c[k + 6], c[k - 1], c[k + 1]);
      }
#pragma unroll
      for (int k = 0; k < 36; ++k) v[k] = fkey(c[k]);
    }
    int m[4];
    med25_block(v, m, f.sepmed);
    const float sigclip = f.sigclip;
    const int sh = qx & 63;  // qx even: both columns share one word
    auto outputs = [&](auto fast) {  // the noise model's form chosen once
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int y = qy + (q >> 1), x = qx + (q & 1);
        if (y < h && x < w) {
          const float N = noise_from_med<decltype(fast)::value>(m[q], nc, f.rn2);
          const float S = L[q] / (2.0f * N);
          stg(f.splane, (int64_t)y * w + x, S);
          const unsigned long long bit = 1ull << (sh + (q & 1));
          const bool on = S > sigclip;
          if (q < 2) {
            set0 |= on ? bit : 0ull;
            clr0 |= on ? 0ull : bit;
          } else {
            set1 |= on ? bit : 0ull;
            clr1 |= on ? 0ull : bit;
          }
        }
      }
    };
    if (noise_fast(nc))
      outputs(std::true_type{});
    else
      outputs(std::false_type{});
    const int64_t wi = (int64_t)qy * f.wpr + (qx >> 6);
    key0 = (unsigned long long)(f.cb + wi);
    if (qy + 1 < h) key1 = (unsigned long long)(f.cb + wi + f.wpr);
  }
  if (run_or(key0, set0, clr0) && key0) {
    unsigned long long* cw = reinterpret_cast<unsigned long long*>(key0);
    if (set0) atom_or(cw, set0);
    if (clr0) atom_and(cw, ~clr0);
  }
  if (run_or(key1, set1, clr1) && key1) {
    unsigned long long* cw = reinterpret_cast<unsigned long long*>(key1);
    if (set1) atom_or(cw, set1);
    if (clr1) atom_and(cw, ~clr1);
  }
}

// ------------------------------------------------------------------ A2
template <int TH>
struct SmemA2 {
  int sk[TH + 4][TW + 4];  // S over the tile + 2 (S >= +0: its bits are its key)
  float spo[TH][TW];       // S' of the tile
};

// A2 (full-S' flag only): S' = S - med5(S) at every pixel of the tile.
template <int TH, int NT>
__device__ __forceinline__ void tile_a2(const FrameDev& f, int y0, int x0, SmemA2<TH>& s) {
  const int tid = threadIdx.x;
  const int h = f.h, w = f.w;
  constexpr int NE = (TH + 4) * (TW + 4), NS = (NE + NT - 1) / NT;
  int vals[NS];
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int i = min(tid + k * NT, NE - 1);
    const int ly = i / (TW + 4), lx = i - ly * (TW + 4);
    const int cy = clampi(y0 - 2 + ly, h - 1), cx = clampi(x0 - 2 + lx, w - 1);
    vals[k] = __float_as_int(ldg(f.splane, (int64_t)cy * w + cx));
  }
#pragma unroll
  for (int k = 0; k < NS; ++k) {
    const int i = tid + k * NT;
    if (i < NE) {
      const int ly = i / (TW + 4), lx = i - ly * (TW + 4);
      s.sk[ly][lx] = vals[k];
    }
  }
  __syncthreads();
  for (int blk = tid; blk < (TH / 2) * (TW / 2); blk += NT) {
    const int by = (blk / (TW / 2)) * 2, bx = (blk % (TW / 2)) * 2;
    int v[36];
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = 0; b < 6; ++b) v[a * 6 + b] = s.sk[by + a][bx + b];
    int m[4];
    med25_block(v, m, f.sepmed);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ty = by + (q >> 1), tx = bx + (q & 1);
      s.spo[ty][tx] = __int_as_float(s.sk[ty + 2][tx + 2]) - funkey(m[q]);
    }
  }
  __syncthreads();
  for (int i = tid; i < TH * TW; i += NT) {
    const int ty = i / TW, tx = i - ty * TW;
    const int gy = y0 + ty, gx = x0 + tx;
    if (gy < h && gx < w) stg(f.sp, (int64_t)gy * w + gx, s.spo[ty][tx]);
  }
  __syncthreads();
}

// ------------------------------------------------------------------ S1 / SG
// S' = S - med5(S) at one pixel, med5 over S's clamped 5x5 window.  VEC: away
// from the frame edges each window row is read with vector loads (ldg_row).
template <bool VEC = true>
__device__ __forceinline__ float sprime_at(const FrameDev& f, int gy, int gx) {
  const int h = f.h, w = f.w;
  float s[25];
  if (VEC && gy >= 2 && gy + 2 < h && gx >= 2 && gx + 2 < w) {  // no clamping: whole rows
#pragma unroll
    for (int a = 0; a < 5; ++a) ldg_row<5>(f.splane, (int64_t)(gy - 2 + a) * w + (gx - 2), s + a * 5);
  } else {
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const int64_t row = (int64_t)clampi(gy - 2 + a, h - 1) * w;
#pragma unroll
      for (int b = 0; b < 5; ++b) s[a * 5 + b] = ldg((const float*)f.splane, row + clampi(gx - 2 + b, w - 1));
    }
  }
  int v[25];  // S >= +0: its bits are its key
#pragma unroll
  for (int k = 0; k < 25; ++k) v[k] = __float_as_int(s[k]);
  return s[12] - funkey(med25_of(v, f.sepmed));
}

// Step 5 at one candidate pixel (gy, gx): fine structure F = med3 - med7(med3)
// (med7 clamps on med3's own grid), f = F / N floored at 0.01; returns
// whether S' / f exceeds objlim.  Reads C from global memory.  Away from the
// frame edges the 9x9 patch is loaded once; near them every med3 reads its
// own clamped neighbourhood.
__device__ __forceinline__ bool objlim_test(const FrameDev& f, const NoiseCoef& nc,
                                            const float* C, int gy, int gx, float spv) {
  const int h = f.h, w = f.w;
  int v49[49];
  float N;
  if (gy >= 4 && gy < h - 4 && gx >= 4 && gx < w - 4) {
    int p[81];
    {
      float c[81];
#pragma unroll
      for (int a = 0; a < 9; ++a) ldg_row<9>(C, (int64_t)(gy - 4 + a) * w + (gx - 4), c + a * 9);
#pragma unroll
      for (int k = 0; k < 81; ++k) p[k] = fkey(c[k]);
    }
    {  // the noise model first, so its window dies before the med3 field is built
      int v25[25];
#pragma unroll
      for (int a = 0; a < 5; ++a)
#pragma unroll
        for (int b = 0; b < 5; ++b) v25[a * 5 + b] = p[(a + 2) * 9 + (b + 2)];
      N = noise_from_med(med25_of(v25, f.sepmed), nc, f.rn2);
    }
    if (f.sepmed) {  // separable: the row medians of 3, then their column medians
#pragma unroll
      for (int a = 0; a < 7; ++a)
#pragma unroll
        for (int b = 0; b < 7; ++b) {
          const int* q = p + a * 9 + b;
          v49[a * 7 + b] = kmed3(kmed3(q[0], q[1], q[2]), kmed3(q[9], q[10], q[11]),
                                 kmed3(q[18], q[19], q[20]));
        }
    } else {
      // med3 of every 3x3 window of the patch from its three sorted columns:
      // the median of 9 is med3(max of the column minima, med3 of the column
      // medians, min of the column maxima).  Row a of the patch is last used
      // by output row a.
#pragma unroll
      for (int a = 0; a < 7; ++a) {
        int lo[9], md[9], hi[9];
#pragma unroll
        for (int b = 0; b < 9; ++b) {
          const int x0 = p[a * 9 + b], x1 = p[(a + 1) * 9 + b], x2 = p[(a + 2) * 9 + b];
          lo[b] = kmin3(x0, x1, x2);
          md[b] = kmed3(x0, x1, x2);
          hi[b] = kmax3(x0, x1, x2);
        }
#pragma unroll
        for (int b = 0; b < 7; ++b)
          v49[a * 7 + b] = kmed3(kmax3(lo[b], lo[b + 1], lo[b + 2]),
                                 kmed3(md[b], md[b + 1], md[b + 2]),
                                 kmin3(hi[b], hi[b + 1], hi[b + 2]));
      }
    }
  } else {
    int v25[25];
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const int64_t row = (int64_t)clampi(gy - 2 + a, h - 1) * w;
#pragma unroll
      for (int b = 0; b < 5; ++b) v25[a * 5 + b] = fkey(ldg(C, row + clampi(gx - 2 + b, w - 1)));
    }
    N = noise_from_med(med25_of(v25, f.sepmed), nc, f.rn2);
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      const int qy = clampi(gy - 3 + a, h - 1);
#pragma unroll
      for (int b = 0; b < 7; ++b) {
        const int qx = clampi(gx - 3 + b, w - 1);
        int v9[9];
#pragma unroll
        for (int e = 0; e < 3; ++e) {
          const int64_t row = (int64_t)clampi(qy - 1 + e, h - 1) * w;
#pragma unroll
          for (int g = 0; g < 3; ++g) v9[e * 3 + g] = fkey(ldg(C, row + clampi(qx - 1 + g, w - 1)));
        }
        v49[a * 7 + b] = med9_of(v9, f.sepmed);
      }
    }
  }
  const float m3 = funkey(v49[24]);
  const float m7 = funkey(med49_of(v49, f.sepmed));
  const float F = m3 - m7;
  const float fr = F / N;
  const float fn = (fr > 0.01f) ? fr : 0.01f;
  return (spv / fn) > f.objlim;
}


// S1, first stage, at one candidate: S' (kept in the S' plane) and its G1 /
// G2 bits.  Returns whether the objlim test is due (G1 holds).
__device__ __forceinline__ bool s1_sprime(const FrameDev& f, int idx, int gy, int gx,
                                          float& spv) {
  spv = sprime_at(f, gy, gx);
  stg(f.sp, idx, spv);
  const int64_t wi = (int64_t)gy * f.wpr + (gx >> 6);
  const uint64_t bit = 1ull << (gx & 63);
  if (spv > f.lo) atom_or(f.g2 + wi, bit);
  if (!(spv > f.sigclip)) return false;
  atom_or(f.g1 + wi, bit);
  return true;
}

// S1, second stage: the objlim test; a confirmed pixel gets its B1 bit, a
// place in the confirmed list and (after iteration 0) its strip's stamp.
// Every active lane of the wave calls it (wave_append).
__device__ __forceinline__ void s1_objlim(const FrameDev& f, int it, int idx, int gy, int gx,
                                          float spv) {
  const bool conf = objlim_test(f, noise_coef(f, it), f.clean, gy, gx, spv);
  if (conf) atom_or(f.b1 + (int64_t)gy * f.wpr + (gx >> 6), (uint64_t)1 << (gx & 63));
  wave_append(count_of(f, it, kCntConf), f.conf, idx, conf);
  if (conf && it > 0) stg(f.b1s, strip_of(f, gy, gx >> 6), it + 1);  // pass B looks by strip
}

// SG, first stage, at pixel q = p + offset o (o in 0..24 over the 5x5 box of
// a confirmed pixel p): returns q if S' must be evaluated there, else -1.  G2
// is set where sigfrac*sigclip < S <= sigclip and S' > sigfrac*sigclip (S1
// has already decided every pixel with S > sigclip).  The growth reads G2
// only next to a pixel of B2 = dil3(B1) & G1.  Within 1 of p that holds (p
// itself is in B2); on the box's outer ring q is needed for p only through a
// G1 pixel within 1 of both p and q (any other route goes through another
// confirmed pixel, whose own box holds q).
__device__ __forceinline__ int sg_pixel(const FrameDev& f, int p, int o, int& qy, int& qx) {
  const int h = f.h, w = f.w, wpr = f.wpr;
  const int py = row_of(f, p), px = p - py * w;
  const int dy = o / 5 - 2, dx = o % 5 - 2;
  qy = py + dy;
  qx = px + dx;
  if (qy < 0 || qy >= h || qx < 0 || qx >= w) return -1;
  // On the outer ring the G1 pixels within 1 of both p and q lie on one row
  // (|dy| = 2) or one column (|dx| = 2) of p's 3x3: at most three.  Their
  // words are loaded with q's G2 word and S, before any test, so that the
  // item waits for one round of loads (clamped positions; the ones outside
  // the frame or the range do not count).
  const bool ring = dy == 2 || dy == -2 || dx == 2 || dx == -2;
  const int ty0 = max(-1, dy - 1), ty1 = min(1, dy + 1);
  const int tx0 = max(-1, dx - 1), tx1 = min(1, dx + 1);
  const bool along_row = ty0 == ty1;  // else one column (tx0 == tx1)
  uint64_t gw[3];
  int rxk[3];
  bool okk[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const int ty = along_row ? ty0 : ty0 + k, tx = along_row ? tx0 + k : tx0;
    const int ry = py + ty, rx = px + tx;
    okk[k] = ring && (along_row ? tx <= tx1 : ty <= ty1) && ry >= 0 && ry < h && rx >= 0 && rx < w;
    rxk[k] = rx;
    gw[k] = ldg(f.g1, (int64_t)clampi(ry, h - 1) * wpr + (clampi(rx, w - 1) >> 6));
  }
  const uint64_t cur = ldg(f.g2, (int64_t)qy * wpr + (qx >> 6));
  const float S = ldg((const float*)f.splane, (int64_t)qy * w + qx);
  // already set (a stale read only repeats the work), or S outside
  // (sigfrac*sigclip, sigclip]: every test after the loads (no short cut)
  const bool need = (((cur >> (qx & 63)) & 1ull) == 0ull) & (S > f.lo) & !(S > f.sigclip);
  bool via = !ring;
#pragma unroll
  for (int k = 0; k < 3; ++k) via |= okk[k] && ((gw[k] >> (rxk[k] & 63)) & 1ull) != 0ull;
  return need && via ? qy * w + qx : -1;
}

// SG, second stage: G2 at pixel q (from sg_pixel) where S' > sigfrac*sigclip.
// Scalar window loads: the lanes hold nearby pixels (box offsets, or queued
// pixels of nearby boxes), so each load instruction touches few cache lines
// (per-lane row loads measured no faster in this pass).
__device__ __forceinline__ void sg_set(const FrameDev& f, int qy, int qx) {
  if (sprime_at<false>(f, qy, qx) > f.lo)
    atom_or(f.g2 + (int64_t)qy * f.wpr + (qx >> 6), (uint64_t)1 << (qx & 63));
}

// ------------------------------------------------------------------ B
// Pass B: one wave streams down nrows rows of up to 64 consecutive bit-plane
// words (every row is one coalesced access of at most 512 bytes).  On a frame
// whose rows hold at most 64 words lane l holds word l; on wider ones lane l
// holds word word0 - 1 + l and lanes 0 and 63 are a one-word halo, words
// word0 .. word0 + 61 being produced.  Horizontal neighbours' edge bits come
// from lane shuffles; vertical dilations use the last rows held in registers.
constexpr int B_WORDS = 62;                // words produced per wave
constexpr int B_WAVES = 4;                 // waves per block, stacked vertically
// rows produced per wave: kBStrip (a pass-B tile is 4 strips)

// Word `word` of row y of a bit plane, 0 outside the frame.  The load is
// issued at the clamped position either way (no branch around it), so a
// ring of such loads stays in flight.
__device__ __forceinline__ unsigned long long word_at(const uint64_t* plane, int y, int word,
                                                      int h, int wpr) {
  const bool in = y >= 0 && y < h && word >= 0 && word < wpr;
  const unsigned long long v = ldg(plane, (int64_t)clampi(y, h - 1) * wpr + clampi(word, wpr - 1));
  return in ? v : 0ull;
}

// Whole-wave lane shifts of a 64-bit value by one lane (DPP wave_shr:1 /
// wave_shl:1, one VALU move per 32-bit half instead of an LDS permute): lane
// i receives lane i - 1 (shr) or lane i + 1 (shl); lanes without a source get
// 0 (bound_ctrl: no zeroed destination needed).  Every lane of the wave must
// be active.
__device__ __forceinline__ unsigned long long from_left_lane(unsigned long long v) {
  const unsigned int lo = __builtin_amdgcn_update_dpp(0u, (unsigned int)v, 0x138, 0xf, 0xf, true);
  const unsigned int hi =
      __builtin_amdgcn_update_dpp(0u, (unsigned int)(v >> 32), 0x138, 0xf, 0xf, true);
  return ((unsigned long long)hi << 32) | lo;
}
__device__ __forceinline__ unsigned long long from_right_lane(unsigned long long v) {
  const unsigned int lo = __builtin_amdgcn_update_dpp(0u, (unsigned int)v, 0x130, 0xf, 0xf, true);
  const unsigned int hi =
      __builtin_amdgcn_update_dpp(0u, (unsigned int)(v >> 32), 0x130, 0xf, 0xf, true);
  return ((unsigned long long)hi << 32) | lo;
}

// Horizontal 3-pixel dilation of each lane's word, the neighbouring words'
// edge bits taken from the adjacent lanes.
__device__ __forceinline__ unsigned long long hdil_lanes(unsigned long long v) {
  const unsigned long long left = from_left_lane(v);
  const unsigned long long right = from_right_lane(v);
  return v | (v << 1) | (v >> 1) | (left >> 63) | (right << 63);
}
// Horizontal 5-pixel dilation, likewise.
__device__ __forceinline__ unsigned long long hdil5_lanes(unsigned long long v) {
  const unsigned long long left = from_left_lane(v);
  const unsigned long long right = from_right_lane(v);
  return v | (v << 1) | (v << 2) | (v >> 1) | (v >> 2) | (left >> 62) | (left >> 63) |
         (right << 62) | (right << 63);
}

// Inclusive prefix sum over the wave (lane order).
__device__ __forceinline__ unsigned int wave_scan(unsigned int x) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const unsigned int y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  return x;
}

// Lists the set bits of one plane (ANDed with a second plane when `mask` is
// given) over rows [y0, y1) of each output lane's word: one atomic per wave on
// the counter, then each lane expands its words, reading eight rows per round
// so the loads overlap.
__device__ __forceinline__ void list_strip(const uint64_t* plane, unsigned int* counter, int* list,
                                           unsigned int n, bool out_lane, int y0, int y1,
                                           int word, int wpr, int w,
                                           const uint64_t* mask = nullptr) {
  const int lane = threadIdx.x & 63;
  const unsigned int incl = wave_scan(n);
  const unsigned int total = __shfl(incl, 63);
  if (!total) return;
  unsigned int base = 0;
  if (lane == 63) base = atom_add(counter, total);
  base = __shfl(base, 63);
  int k = (int)(base + incl - n);
  if (out_lane && n) {
    #pragma unroll 1  // a strip is 2 such row groups: kept as a loop (registers)
    for (int yb = y0; yb < y1; yb += 8) {
      unsigned long long v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int64_t ro = (int64_t)min(yb + j, y1 - 1) * wpr;  // wave-uniform
        v[j] = ldg_u(plane + ro, (uint32_t)word);
        if (mask) v[j] &= ldg_u(mask + ro, (uint32_t)word);
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        unsigned long long bits = yb + j < y1 ? v[j] : 0ull;
        while (bits) {
          const int b = __ffsll((long long)bits) - 1;
          bits &= bits - 1;
          stg(list, k++, (yb + j) * w + word * TW + b);
        }
      }
    }
  }
}

// Marks, at the even bit of each column pair, whether either bit of the pair
// is set.
__device__ __forceinline__ unsigned long long pair_bits(unsigned long long v) {
  return (v | (v >> 1)) & 0x5555555555555555ull;
}

// Lists the aligned 2x2 blocks (top-left pixel index) holding a set bit of
// the plane over rows [y0, y1) of each output lane's word (y0 even; a block
// on the frame's last row when h is odd has one row); n is the lane's block
// count.  One atomic per wave on the counter; eight rows are read per round.
__device__ __forceinline__ void list_quads(const uint64_t* plane, unsigned int* counter, int* list,
                                           unsigned int n, bool out_lane, int y0, int y1,
                                           int word, int wpr, int w) {
  const int lane = threadIdx.x & 63;
  const unsigned int incl = wave_scan(n);
  const unsigned int total = __shfl(incl, 63);
  if (!total) return;
  unsigned int base = 0;
  if (lane == 63) base = atom_add(counter, total);
  base = __shfl(base, 63);
  int k = (int)(base + incl - n);
  if (out_lane && n) {
    #pragma unroll 1  // a strip is 2 such row groups: kept as a loop (registers)
    for (int yb = y0; yb < y1; yb += 8) {
      unsigned long long v[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) v[j] = ldg_u(plane + (int64_t)min(yb + j, y1 - 1) * wpr, (uint32_t)word);
#pragma unroll
      for (int j = 0; j < 8; j += 2) {
        const int y = yb + j;
        if (y >= y1) break;
        unsigned long long bits = pair_bits(v[j] | (y + 1 < y1 ? v[j + 1] : 0ull));
        while (bits) {
          const int b = __ffsll((long long)bits) - 1;
          bits &= bits - 1;
          stg(list, k++, y * w + word * TW + b);
        }
      }
    }
  }
}

// One wave's strip: rows [y0, y0 + nrows) of the strip column starting at
// word word0 (strip_word gives each lane's word).
// Step t reads B1 of row r = y0 - 8 + t and produces B2 of row r - 1; B3, M'
// and the new pixels of row r - 2; the recompute set of row r - 4 (mask
// pixels within 2 of a new one: new pixels of rows r - 6 .. r - 2); the
// S-recompute set RS of row r - 6 (within 2 of the recompute set: rows
// r - 8 .. r - 4); and R4 of row r - 8 (within 2 of RS: rows r - 10 .. r - 6).
// Rows outside the strip are produced only as far as the strip's rows need
// them.
__device__ __forceinline__ void strip_b(const FrameDev& f, int it, int y0, int word0) {
  constexpr int nrows = kBStrip;
  const int lane = threadIdx.x & 63;
  const int h = f.h, w = f.w, wpr = f.wpr;
  const int word = strip_word(f, word0, lane);
  const bool out_lane = strip_out_lane(f, word, lane);
  const int y1 = min(y0 + nrows, h);
  const uint64_t* mprev = mprev_of(f, it);
  uint64_t* mnext = mnext_of(f, it);
  if (stopped(f, it)) {  // the mask carries over
    if (out_lane)
      for (int y = y0; y < y1; ++y) stg(mnext, (int64_t)y * wpr + word, (uint64_t)word_at(mprev, y, word, h, wpr));
    return;
  }
  // no US after the last iteration, nor for a frame whose later iterations
  // run A1 (no supplied gain)
  const bool want_rs = it < f.niter - 1 && !f.est_gain;
  if (it > 0) {
    // Every output of the strip depends on B1 only within 8 rows and one
    // word of it, which lie in the strip and its eight neighbours (strips
    // are at least 8 rows tall).  Where none of them holds a B1 bit this
    // iteration (usual after iteration 0: B1 holds the few confirmed pixels)
    // the mask carries over, R4 is empty and nothing is listed.  If this
    // pass did the same here last iteration, both mask planes already agree
    // and R4 is already clear.
    const int ncol = strip_cols(f), nsy = (h + kBStrip - 1) / kBStrip;
    const int sy = y0 / kBStrip, sx = word0 / B_WORDS, me = sy * ncol + sx;
    const int stamp = it + 1;
    bool near = false;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int ty = sy + dy, tx = sx + dx;
        if (ty >= 0 && ty < nsy && tx >= 0 && tx < ncol) near |= ldg(f.b1s, ty * ncol + tx) == stamp;
      }
    if (!near) {
      if (out_lane && ldg(f.bq, me) != it) {
        #pragma unroll 1  // a strip is 2 such row groups: kept as a loop (registers)
        for (int yc = y0; yc < y1; yc += 8) {
          unsigned long long mw[8];  // eight rows in flight
#pragma unroll
          for (int j = 0; j < 8; ++j) mw[j] = word_at(mprev, min(yc + j, y1 - 1), word, h, wpr);
#pragma unroll
          for (int j = 0; j < 8; ++j) {
            if (yc + j < y1) {
              const int64_t wi = (int64_t)(yc + j) * wpr + word;
              stg(mnext, wi, (uint64_t)mw[j]);
              if (want_rs) stg(f.r4, wi, (uint64_t)0);
            }
          }
        }
      }
      if (lane == 0) stg(f.bq, me, stamp);
      return;
    }
  }
  unsigned int fresh = 0, nlist = 0, nrs = 0;  // nrs: 2x2 blocks holding an RS pixel
  unsigned long long rs_even = 0;              // RS of the last even row
  unsigned long long hd1a = 0, hd1b = 0;                  // hdil(B1) of rows r-2, r-1
  unsigned long long hd2a = 0, hd2b = 0;                  // hdil(B2) of rows r-3, r-2
  unsigned long long hn0 = 0, hn1 = 0, hn2 = 0, hn3 = 0;  // hdil5(new) of rows r-6 .. r-3
  unsigned long long mna = 0, mnb = 0;                    // M' of rows r-4, r-3
  unsigned long long hr0 = 0, hr1 = 0, hr2 = 0, hr3 = 0;  // hdil5(recompute) of rows r-8 .. r-5
  unsigned long long hs0 = 0, hs1 = 0, hs2 = 0, hs3 = 0;  // hdil5(RS) of rows r-10 .. r-7
  // The words step t reads (B1 of row r, G1 of r - 1, G2 and M of r - 2,
  // r = y0 - 8 + t), loaded kAhead steps ahead into a ring indexed
  // statically: the nrows + 16 steps are one fully unrolled sequence, so no
  // loaded value crosses a loop back edge and every wait counts exactly the
  // loads still needed.  The loads go to clamped in-frame positions
  // unconditionally; the step that uses a word zeroes it if its row or
  // column lies outside the frame, so nothing waits for a load before then.
  constexpr int kAhead = 4;
  // iteration 0 has no previous mask: its words load from B1 and are dropped
  const uint64_t* mp_src = mprev ? mprev : f.b1;
  const unsigned long long mp_keep = mprev ? ~0ull : 0ull;
  const bool wok = word >= 0 && word < wpr;
  const int wc = clampi(word, wpr - 1);
  unsigned long long qb1[kAhead], qg1[kAhead], qg2[kAhead], qmp[kAhead];
#pragma unroll
  for (int k = 0; k < kAhead; ++k) {
    const int rr = y0 - 8 + k;
    // row offsets are wave-uniform: scalar bases, one per-lane word offset
    qb1[k] = ldg_u(f.b1 + (int64_t)clampi(rr, h - 1) * wpr, (uint32_t)wc);
    qg1[k] = ldg_u(f.g1 + (int64_t)clampi(rr - 1, h - 1) * wpr, (uint32_t)wc);
    qg2[k] = ldg_u(f.g2 + (int64_t)clampi(rr - 2, h - 1) * wpr, (uint32_t)wc);
    qmp[k] = ldg_u(mp_src + (int64_t)clampi(rr - 2, h - 1) * wpr, (uint32_t)wc);
  }
#pragma unroll
  for (int t0 = 0; t0 < nrows + 16; t0 += kAhead)
#pragma unroll
  for (int k = 0; k < kAhead; ++k) {
    const int r = y0 - 8 + t0 + k;
    const unsigned long long k0 = (wok && r >= 0 && r < h) ? ~0ull : 0ull;
    const unsigned long long k1 = (wok && r >= 1 && r <= h) ? ~0ull : 0ull;
    const unsigned long long k2 = (wok && r >= 2 && r <= h + 1) ? ~0ull : 0ull;
    const unsigned long long wb1 = qb1[k] & k0, wg1 = qg1[k] & k1, wg2 = qg2[k] & k2;
    const unsigned long long mp = qmp[k] & k2 & mp_keep;
    const int rn = r + kAhead;  // the step this slot serves next
    qb1[k] = ldg_u(f.b1 + (int64_t)clampi(rn, h - 1) * wpr, (uint32_t)wc);
    qg1[k] = ldg_u(f.g1 + (int64_t)clampi(rn - 1, h - 1) * wpr, (uint32_t)wc);
    qg2[k] = ldg_u(f.g2 + (int64_t)clampi(rn - 2, h - 1) * wpr, (uint32_t)wc);
    qmp[k] = ldg_u(mp_src + (int64_t)clampi(rn - 2, h - 1) * wpr, (uint32_t)wc);
    const unsigned long long hd1c = hdil_lanes(wb1);
    const unsigned long long b2 = (hd1a | hd1b | hd1c) & wg1;  // row r - 1
    const unsigned long long hd2c = hdil_lanes(b2);
    const int nr = r - 2;
    const unsigned long long b3 = (hd2a | hd2b | hd2c) & wg2;  // row r - 2
    const unsigned long long mn = mp | b3;
    const unsigned long long nw = b3 & ~mp;
    const unsigned long long hnc = hdil5_lanes(nw);
    if (nr >= y0 && nr < y1 && out_lane) {
      stg_u(mnext + (int64_t)nr * wpr, (uint32_t)word, (uint64_t)mn);
      fresh += (unsigned int)__popcll(nw);
    }
    const int dy = r - 4;
    const unsigned long long d = mna & (hn0 | hn1 | hn2 | hn3 | hnc);  // row r - 4
    if (dy >= y0 && dy < y1 && out_lane) {
      stg_u(f.dirty + (int64_t)dy * wpr, (uint32_t)word, (uint64_t)d);
      nlist += (unsigned int)__popcll(d);
    }
    const unsigned long long hrc = hdil5_lanes(d);
    const int ry = r - 6;
    const unsigned long long rsw = hr0 | hr1 | hr2 | hr3 | hrc;  // row r - 6
    if (want_rs && ry >= y0 && ry < y1 && out_lane) {
      stg_u(f.rs + (int64_t)ry * wpr, (uint32_t)word, (uint64_t)rsw);
      if (ry & 1)  // y0 is even: rows ry - 1, ry form one block row
        nrs += (unsigned int)__popcll(pair_bits(rs_even | rsw));
      else if (ry + 1 == y1)  // the frame's last row, h odd
        nrs += (unsigned int)__popcll(pair_bits(rsw));
      rs_even = rsw;
    }
    const unsigned long long hsc = hdil5_lanes(rsw);
    const int qy = r - 8;
    if (want_rs && qy >= y0 && qy < y1 && out_lane)
      stg_u(f.r4 + (int64_t)qy * wpr, (uint32_t)word, (uint64_t)(hs0 | hs1 | hs2 | hs3 | hsc));  // row r - 8
    hd1a = hd1b;
    hd1b = hd1c;
    hd2a = hd2b;
    hd2b = hd2c;
    hn0 = hn1;
    hn1 = hn2;
    hn2 = hn3;
    hn3 = hnc;
    mna = mnb;
    mnb = mn;
    hr0 = hr1;
    hr1 = hr2;
    hr2 = hr3;
    hr3 = hrc;
    hs0 = hs1;
    hs1 = hs2;
    hs2 = hs3;
    hs3 = hsc;
  }
  // S2's list (recompute set) and the next US's list (2x2 blocks of RS)
  list_strip(f.dirty, count_of(f, it, kCntDirty), f.list, nlist, out_lane, y0, y1, word, wpr, w);
  if (want_rs)
    list_quads(f.rs, count_of(f, it, kCntRecomp), f.conf, nrs, out_lane, y0, y1, word, wpr, w);
  for (int off = 32; off > 0; off >>= 1) fresh += __shfl_down(fresh, off);
  if (lane == 0 && fresh) atom_add(f.n_new + it, (unsigned long long)fresh);
}

// SC on one wave's strip (the pass-B tiling).  Iteration 0 clears G1, G2 and
// B1 and lists every pixel of CB.  Later iterations keep the three planes
// outside R4 -- there S', the objlim inputs and so every bit are those of the
// previous iteration -- clear them inside R4, list the pixels of CB inside R4
// for S1 and list the kept B1 pixels (outside R4) as confirmed.  A strip
// where pass B of the previous iteration found no B1 bit within reach has R4
// and B1 empty, so there is nothing to do.  Words are read eight rows at a
// time so their loads overlap (the G1 and G2 words to clear inside R4 in a
// second round, before any store); lists take one atomic per wave.
__device__ __forceinline__ void strip_sc(const FrameDev& f, int it, int y0, int word0) {
  constexpr int nrows = kBStrip;
  if (stopped(f, it)) return;
  const int me = strip_of(f, y0, word0);
  // every iteration of a frame without a supplied gain starts afresh, as
  // iteration 0 does: its S, and so every bit, may change everywhere
  const bool first = it == 0 || f.est_gain;
  if (!first && ldg(f.bq, me) == it) return;
  const int lane = threadIdx.x & 63;
  const int w = f.w, wpr = f.wpr;
  const int word = strip_word(f, word0, lane);
  const bool out_lane = strip_out_lane(f, word, lane);
  const uint32_t lw = (uint32_t)clampi(word, wpr - 1);  // the lane's word, in the row
  const int y1 = min(y0 + nrows, f.h);
  unsigned int nc = 0, nk = 0;
  constexpr int kRows = 8;  // rows whose words are loaded together
  // rows are wave-uniform: each access is a scalar row base plus the lane's
  // word; the two forms (first or later iteration) are separate loops
  if (first) {
    if (out_lane) {
#pragma unroll 1  // a strip is 2 such row groups: kept as a loop (registers)
      for (int yb = y0; yb < y1; yb += kRows) {
        unsigned long long c[kRows];
#pragma unroll
        for (int j = 0; j < kRows; ++j) c[j] = ldg_u(f.cb + (int64_t)min(yb + j, y1 - 1) * wpr, lw);
#pragma unroll
        for (int j = 0; j < kRows; ++j) {
          if (yb + j < y1) {
            const int64_t ro = (int64_t)(yb + j) * wpr;
            stg_u(f.g1 + ro, lw, (uint64_t)0);
            stg_u(f.g2 + ro, lw, (uint64_t)0);
            stg_u(f.b1 + ro, lw, (uint64_t)0);
            nc += (unsigned int)__popcll(c[j]);
          }
        }
      }
    }
    list_strip(f.cb, count_of(f, it, kCntCand), f.list, nc, out_lane, y0, y1, word, wpr, w);
    return;
  }
  if (out_lane) {
#pragma unroll 1  // a strip is 2 such row groups: kept as a loop (registers)
    for (int yb = y0; yb < y1; yb += kRows) {
      unsigned long long c[kRows], r[kRows], b[kRows];
#pragma unroll
      for (int j = 0; j < kRows; ++j) {
        const int64_t ro = (int64_t)min(yb + j, y1 - 1) * wpr;
        c[j] = ldg_u(f.cb + ro, lw);
        r[j] = ldg_u(f.r4 + ro, lw);
        b[j] = ldg_u(f.b1 + ro, lw);
      }
      unsigned long long g1w[kRows], g2w[kRows];
#pragma unroll
      for (int j = 0; j < kRows; ++j) {
        g1w[j] = g2w[j] = 0ull;
        if (yb + j < y1 && r[j]) {
          const int64_t ro = (int64_t)(yb + j) * wpr;
          g1w[j] = ldg_u(f.g1 + ro, lw);
          g2w[j] = ldg_u(f.g2 + ro, lw);
        }
      }
#pragma unroll
      for (int j = 0; j < kRows; ++j) {
        if (yb + j < y1) {
          if (r[j]) {
            const int64_t ro = (int64_t)(yb + j) * wpr;
            stg_u(f.g1 + ro, lw, (uint64_t)(g1w[j] & ~r[j]));
            stg_u(f.g2 + ro, lw, (uint64_t)(g2w[j] & ~r[j]));
            stg_u(f.b1 + ro, lw, (uint64_t)(b[j] & ~r[j]));
          }
          nc += (unsigned int)__popcll(c[j] & r[j]);
          nk += (unsigned int)__popcll(b[j] & ~r[j]);
        }
      }
    }
  }
  if (__ballot(nk != 0u) != 0ull && lane == 0) stg(f.b1s, me, it + 1);  // kept B1 bits
  list_strip(f.cb, count_of(f, it, kCntCand), f.list, nc, out_lane, y0, y1, word, wpr, w, f.r4);
  list_strip(f.b1, count_of(f, it, kCntConf), f.conf, nk, out_lane, y0, y1, word, wpr, w);
}

// OUT (last iteration) on one wave's strip (the pass-B tiling): the final
// mask words of each row expanded to bytes.  Each lane loads the word it
// holds (strip_word).  When rows are 16-byte aligned, store k of a row writes
// 1 KB contiguously: lane l expands quarter (l & 3) of word
// word0 + 16k + (l >> 2), taken from its owner lane by a shuffle, into 16
// bytes.  Other frames use byte stores.
__device__ __forceinline__ unsigned int spread4(unsigned int b) {
  return (b & 1u) | ((b & 2u) << 7) | ((b & 4u) << 14) | ((b & 8u) << 21);
}
__device__ __forceinline__ void strip_out(const FrameDev& f, int it, int y0, int word0) {
  constexpr int nrows = kBStrip;
  if (it != f.niter - 1) return;
  const int lane = threadIdx.x & 63;
  const int w = f.w, wpr = f.wpr;
  const int word = strip_word(f, word0, lane);
  const bool out_lane = strip_out_lane(f, word, lane);
  const int y1 = min(y0 + nrows, f.h);
  const uint64_t* m = mnext_of(f, it);
  const bool vec = (w & 15) == 0 && ((uintptr_t)f.out_mask & 15u) == 0u;  // frame-uniform
  const bool one_col = wpr <= 64;  // lane l holds word l (else word word0 - 1 + l)
  if (!vec) {
    if (!out_lane) return;
    const int x0 = word * TW;
    const int nb = min(TW, w - x0);  // bytes of this word inside the row
    for (int y = y0; y < y1; ++y) {
      const unsigned long long wb = ldg(m, (int64_t)y * wpr + word);
      uint8_t* dst = f.out_mask + (int64_t)y * w + x0;
      for (int b = 0; b < nb; ++b) stg(dst, b, (uint8_t)((wb >> b) & 1ull));
    }
    return;
  }
  const int qq = lane & 3;  // the quarter this lane expands
  const uint32_t lw = (uint32_t)clampi(word, wpr - 1);
  typedef unsigned int u4v __attribute__((ext_vector_type(4)));
  // rows are wave-uniform: scalar row bases plus per-lane offsets
#pragma unroll 1  // a strip is 2 such row groups: kept as a loop (registers)
  for (int yb = y0; yb < y1; yb += 8) {
    unsigned long long wb[8];  // eight rows' words in flight at once
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const unsigned long long v = ldg_u(m + (int64_t)min(yb + j, y1 - 1) * wpr, lw);
      wb[j] = out_lane ? v : 0ull;
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int y = yb + j;
      if (y >= y1) break;
      u4v* row = reinterpret_cast<u4v*>(f.out_mask + (int64_t)y * w);  // 16-byte aligned
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int rw = 16 * k + (lane >> 2);  // word of the strip, 0 .. 63
        const unsigned long long v = __shfl(wb[j], one_col ? rw : min(rw + 1, 63));
        const int xb = (word0 + rw) * TW + 16 * qq;  // first byte; w % 16 == 0
        if ((one_col || rw < B_WORDS) && xb < w) {
          const unsigned int b16 = (unsigned int)(v >> (16 * qq)) & 0xffffu;
          const u4v o = {spread4(b16), spread4(b16 >> 4), spread4(b16 >> 8), spread4(b16 >> 12)};
          stg_u(row, (uint32_t)(xb >> 4), o);
        }
      }
    }
  }
}

// S2 at one listed (flagged) pixel: lower median of the un-flagged values of
// its clamped 5x5 window; unchanged if every cell is flagged.  Such a pixel
// is counted (n_new[niter]) in the iteration where its window first holds no
// un-flagged cell: the mask only grows, so it stays that way, and that
// iteration lists it (its window gained a new pixel, or it is new itself, or
// it is iteration 0, which lists every mask pixel).  Summed over the
// iterations the count is that of the final mask.
__device__ __forceinline__ void sparse_replace(const FrameDev& f, int it, int idx) {
  const int h = f.h, w = f.w, wpr = f.wpr;
  const int gy = row_of(f, idx), gx = idx - gy * w;
  const uint64_t* m = mnext_of(f, it);
  float* C = f.clean;
  // every load is issued before the mask is applied: the 25 window values
  // and, per window row, the mask words of its first and last column
  const int xl = clampi(gx - 2, w - 1), xh = clampi(gx + 2, w - 1);
  float c[25];
  unsigned long long mw[10];
  const bool inner = gy >= 2 && gy + 2 < h && gx >= 2 && gx + 2 < w;  // no clamping
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    const int qy = clampi(gy - 2 + a, h - 1);
    const int64_t row = (int64_t)qy * w;
    if (inner) {
      ldg_row<5>(C, row + (gx - 2), c + a * 5);
    } else {
#pragma unroll
      for (int b = 0; b < 5; ++b) c[a * 5 + b] = ldg((const float*)C, row + clampi(gx - 2 + b, w - 1));
    }
    mw[2 * a] = ldg(m, (int64_t)qy * wpr + (xl >> 6));
    mw[2 * a + 1] = ldg(m, (int64_t)qy * wpr + (xh >> 6));
  }
  int v[25];
  int n = 0;
#pragma unroll
  for (int a = 0; a < 5; ++a) {
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      const int qx = clampi(gx - 2 + b, w - 1);
      const unsigned long long word = (qx >> 6) == (xl >> 6) ? mw[2 * a] : mw[2 * a + 1];
      const bool use = ((word >> (qx & 63)) & 1ull) == 0ull;
      v[a * 5 + b] = use ? fkey(c[a * 5 + b]) : KEY_EXCLUDED;
      n += use ? 1 : 0;
    }
  }
  if (n > 0) {
    int srt[13];
    sort25_lo13(v, srt);  // ranks 0..12: the lower median of n <= 25 values
    const int r = (n - 1) >> 1;  // lower median of the n un-flagged values
    int sel = srt[0];
#pragma unroll
    for (int k = 1; k < 13; ++k) sel = (r == k) ? srt[k] : sel;
    stg(C, (int64_t)gy * w + gx, funkey(sel));
  } else {
    // counted only if the previous mask left an un-flagged cell in the window
    // (or did not hold the pixel): rare, so the previous words load only here
    const uint64_t* mp = mprev_of(f, it);
    bool first = true;
    if (mp && ((ldg(mp, (int64_t)gy * wpr + (gx >> 6)) >> (gx & 63)) & 1ull)) {
      first = false;
#pragma unroll
      for (int a = 0; a < 5; ++a) {
        const int64_t row = (int64_t)clampi(gy - 2 + a, h - 1) * wpr;
        const unsigned long long lw = ldg(mp, row + (xl >> 6)), hw = ldg(mp, row + (xh >> 6));
#pragma unroll
        for (int b = 0; b < 5; ++b) {
          const int qx = clampi(gx - 2 + b, w - 1);
          const unsigned long long word = (qx >> 6) == (xl >> 6) ? lw : hw;
          first |= ((word >> (qx & 63)) & 1ull) == 0ull;
        }
      }
    }
    if (first) atom_add(f.n_new + f.niter, 1ull);
  }
}



// Sparse passes: WHICH = 0 (S1 over the candidates), 2 (SG: 25 items per
// confirmed pixel), 1 (S2 over the recompute set), 3 (US over the 2x2 blocks
// the previous iteration's pass B listed).  Length of a frame's item range; the lists were
// filled by earlier launches.
template <int WHICH>
__device__ __forceinline__ long long sparse_len(const FrameDev& f, int it) {
  if (stopped(f, it)) return 0;
  switch (WHICH) {
    case 0: return (long long)ldg(count_of(f, it, kCntCand), 0);
    case 1: return (long long)ldg(count_of(f, it, kCntDirty), 0);
    case 2: return 25ll * ldg(count_of(f, it, kCntConf), 0);
    default: return it > 0 ? (long long)ldg(count_of(f, it - 1, kCntRecomp), 0) : 0ll;
  }
}

// S1 and SG in two stages: the first runs on every item and leaves most
// lanes without second-stage work (the objlim test; S' at a box pixel), so
// the items that need it are queued per wave in LDS and the second stage runs
// whenever 64 are queued, on full waves.  A queue holds items of one frame.
constexpr int kWaveQ = 128;  // < 64 queued, plus one chunk of 64
struct WaveQueue {
  int key[kWaveQ];
  float val[kWaveQ];
};

// Appends (key, val) of the lanes with need; returns the new length
// (wave-uniform).  Every lane of the wave calls it.
__device__ __forceinline__ int queue_push(WaveQueue* q, int n, bool need, int key, float val) {
  const unsigned long long bal = __ballot(need);
  if (need) {
    const int pos = n + __popcll(bal & lanes_below());
    q->key[pos] = key;
    q->val[pos] = val;
  }
  return n + __popcll(bal);
}

// The second stage of S1 (the objlim test) or SG (S' at a box pixel) on one
// item.  Every active lane of the wave calls it (S1 appends with wave_append).
template <int WHICH>
__device__ __forceinline__ void sparse_second(const FrameDev& f, int it, int key, int ky, int kx,
                                              float val) {
  if constexpr (WHICH == 0)
    s1_objlim(f, it, key, ky, kx, val);
  else
    sg_set(f, ky, kx);
}

// Runs the second stage on queued items, 64 at a time while 64 are queued
// (all of them with drain), newest first; returns what is left queued.  Every
// lane of the wave calls it.
template <int WHICH>
__device__ __forceinline__ int queue_run(const FrameDev& f, int it, WaveQueue* q, int n,
                                         bool drain) {
  const int lane = threadIdx.x & 63;
  while (n >= 64 || (drain && n > 0)) {
    const int take = n < 64 ? n : 64;
    n -= take;
    if (lane < take) {
      const int key = q->key[n + lane];
      const int ky = row_of(f, key);
      sparse_second<WHICH>(f, it, key, ky, key - ky * f.w, q->val[n + lane]);
    }
  }
  return n;
}

// First stage of item g of a frame's range (S1, SG), or the whole item (S2):
// returns the pixel index for the second stage (its row and column in ky,
// kx), or -1.
template <int WHICH>
__device__ __forceinline__ int sparse_item(const FrameDev& f, int it, long long g, int& ky,
                                           int& kx, float& val) {
  if constexpr (WHICH == 0) {
    const int idx = ldg(f.list, g);
    ky = row_of(f, idx);
    kx = idx - ky * f.w;
    return s1_sprime(f, idx, ky, kx, val) ? idx : -1;
  } else if constexpr (WHICH == 1) {
    sparse_replace(f, it, ldg(f.list, g));
    return -1;
  } else {
    static_assert(WHICH == 2, "US runs whole waves (sparse_frame)");
    // item g: box offset g % 25 of confirmed pixel g / 25 (32-bit arithmetic
    // while g fits)
    long long j;
    int o;
    if (g <= 0x7fffffffll) {
      const unsigned int g32 = (unsigned int)g, j32 = g32 / 25u;
      j = j32;
      o = (int)(g32 - j32 * 25u);
    } else {
      j = g / 25;
      o = (int)(g - j * 25);
    }
    const int q = sg_pixel(f, ldg(f.conf, j), o, ky, kx);
    return q < 0 ? -1 : ky * f.w + kx;
  }
}

// A frame's items gtid - lane + k * gstride + lane (whole waves: the queue and
// update_s_quad work across the wave's lanes).  QUEUED: S1's and SG's second
// stages go through the wave's queue q, else they run at once.
template <int WHICH, bool QUEUED>
__device__ __forceinline__ void sparse_frame(const FrameDev& f, int it, long long gtid,
                                             long long gstride, WaveQueue* q) {
  const long long n = sparse_len<WHICH>(f, it);
  const int lane = threadIdx.x & 63;
  if constexpr (WHICH == 3) {
    const NoiseCoef nc = noise_coef(f, it);
    for (long long g0 = gtid - lane; g0 < n; g0 += gstride) {
      const long long g = g0 + lane;
      const bool active = g < n;
      const int qq = active ? ldg(f.conf, g) : 0;
      const int qy = row_of(f, qq);
      update_s_quad(f, nc, qy, qq - qy * f.w, active);
    }
  } else if constexpr (WHICH == 1) {
    for (long long g = gtid; g < n; g += gstride) {
      int ky, kx;
      float unused;
      (void)sparse_item<1>(f, it, g, ky, kx, unused);
    }
  } else if constexpr (!QUEUED) {
    for (long long g = gtid; g < n; g += gstride) {
      int ky, kx;
      float val = 0.0f;
      const int key = sparse_item<WHICH>(f, it, g, ky, kx, val);
      if (key >= 0) sparse_second<WHICH>(f, it, key, ky, kx, val);
    }
  } else {
    int nq = 0;
    for (long long g0 = gtid - lane; g0 < n; g0 += gstride) {
      const long long g = g0 + lane;
      int ky = 0, kx = 0;
      float val = 0.0f;
      const int key = g < n ? sparse_item<WHICH>(f, it, g, ky, kx, val) : -1;
      nq = queue_push(q, nq, key >= 0, key, val);
      nq = queue_run<WHICH>(f, it, q, nq, false);
    }
    queue_run<WHICH>(f, it, q, nq, true);
  }
}

}  // namespace lac
