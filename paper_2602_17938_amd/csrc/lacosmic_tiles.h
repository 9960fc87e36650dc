// Tile-level device code of the L.A.Cosmic iteration for gfx950 (MI355X).
//
// One iteration is three dense passes over tiles of TH x 64 output pixels (a
// tile row is one 64-bit word of every bit plane) and two sparse passes over
// per-frame pixel lists:
//
//  A1 (steps 1-3a): stages C over the tile plus a 2-pixel ring (clamped) in
//     LDS and computes, per pixel, the Laplacian edge image L, med5(C), the
//     noise model N and S = L / (2N); writes the S plane.  The 5x5 medians of
//     a 2x2 block of pixels share one selection network.
//  A2 (steps 3b-5): stages S over the tile plus a 2-pixel ring (clamped:
//     med5(S) clamps on S's own grid), computes S' = S - med5(S) (2x2 blocks
//     again) wherever it can decide a threshold, writes the bit planes
//     G1 = [S' > sigclip] and G2 = [S' > sigfrac*sigclip], clears the tile's
//     words of the candidate plane B1 and lists the pixels of G1.
//  S1 (step 5, sparse): at the listed pixels only -- the objlim test is a
//     conjunction with S' > sigclip -- the fine-structure ratio
//     S' / max((med3 - med7(med3)) / N, 0.01) > objlim; sets B1 bits.
//  B  (step 6): bit-parallel on 64-bit row words, one wave streaming down a
//     strip of rows of 62 words: B2 = dil3(B1) & G1, B3 = dil3(B2) & G2, M' = M | B3
//     (ping-pong bit planes, plus the output bytes at the last iteration),
//     the count of new pixels, and the list of flagged pixels.
//  S2 (step 7, sparse): each listed pixel takes the lower median of its
//     un-flagged clamped 5x5 neighbours (a sorting network over 25 keys with
//     the flagged ones pushed to the top).  C is updated in place only at
//     flagged pixels and nothing reads a flagged pixel's value, so there is
//     no race on C.
//
// Medians run on 32-bit keys whose signed order is the float order, with
// min/max networks (v_min3/v_max3/v_med3_i32): they select exactly.  All
// arithmetic is binary32 in the same expression order as a plain evaluation
// of the method, compiled with -ffp-contract=off and IEEE division / sqrt.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lacosmic_device.h"
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
__device__ __forceinline__ bool finite_bits(float v) {
  return (__float_as_uint(v) & 0x7f800000u) != 0x7f800000u;
}

__device__ __forceinline__ const float* src_of(const FrameDev& f, int it) {
  return it == 0 ? f.img : f.clean;
}
__device__ __forceinline__ const uint64_t* mprev_of(const FrameDev& f, int it) {
  return it == 0 ? nullptr : f.mbits[(it - 1) & 1];
}
__device__ __forceinline__ uint64_t* mnext_of(const FrameDev& f, int it) {
  return f.mbits[it & 1];
}
// With early stop, iteration it is skipped when iteration it-1 added nothing.
__device__ __forceinline__ bool stopped(const FrameDev& f, int it) {
  return f.early_stop && it > 0 && f.n_new[it - 1] == 0ull;
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

// Step 2: noise model from med5(C), floored at 1e-4.
__device__ __forceinline__ float noise_from_med(float m5, float gain, float rn2) {
  const float m = (m5 > 1e-4f) ? m5 : 1e-4f;
  const float var = gain * m + rn2;
  return sqrtf(var) / gain;
}

// ------------------------------------------------------------------ A1
template <int TH>
struct SmemA1 {
  int ck[TH + 4][TW + 4];    // keys of C over the tile + 2
  float cf[TH + 4][TW + 4];  // C over the tile + 2
  float so[TH][TW];          // S of the tile, staged for a coalesced store
};

template <int TH, int NT>
__device__ void tile_a1(const FrameDev& f, int it, int y0, int x0, SmemA1<TH>& s) {
  const int tid = threadIdx.x;
  const int h = f.h, w = f.w;
  const float* src = src_of(f, it);
  if (y0 == 0 && x0 == 0 && tid == 0) f.counts[0] = 0u;  // A2 lists after A1 ends
  int bad = 0;
  for (int i = tid; i < (TH + 4) * (TW + 4); i += NT) {
    const int ly = i / (TW + 4), lx = i - ly * (TW + 4);
    const int cy = clampi(y0 - 2 + ly, h - 1), cx = clampi(x0 - 2 + lx, w - 1);
    const float v = src[(int64_t)cy * w + cx] + 0.0f;  // -0 becomes +0
    bad |= !finite_bits(v);
    s.cf[ly][lx] = v;
    s.ck[ly][lx] = fkey(v);
  }
  if (it == 0 && bad) atomicOr(f.status, 1);
  __syncthreads();
  if (it == 0) {  // C starts as the canonical input
    for (int i = tid; i < TH * TW; i += NT) {
      const int ty = i / TW, tx = i - ty * TW;
      const int gy = y0 + ty, gx = x0 + tx;
      if (gy < h && gx < w) f.clean[(int64_t)gy * w + gx] = s.cf[ty + 2][tx + 2];
    }
  }
  for (int blk = tid; blk < (TH / 2) * (TW / 2); blk += NT) {
    const int by = (blk / (TW / 2)) * 2, bx = (blk % (TW / 2)) * 2;
    int v[36];
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = 0; b < 6; ++b) v[a * 6 + b] = s.ck[by + a][bx + b];
    int m[4];
    med25_2x2(v, m);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ly = by + (q >> 1) + 2, lx = bx + (q & 1) + 2;
      const float L = lap_edge(s.cf[ly][lx], s.cf[ly - 1][lx], s.cf[ly + 1][lx],
                               s.cf[ly][lx - 1], s.cf[ly][lx + 1]);
      const float N = noise_from_med(funkey(m[q]), f.gain, f.rn2);
      s.so[ly - 2][lx - 2] = L / (2.0f * N);
    }
  }
  __syncthreads();
  for (int i = tid; i < TH * TW; i += NT) {
    const int ty = i / TW, tx = i - ty * TW;
    const int gy = y0 + ty, gx = x0 + tx;
    if (gy < h && gx < w) f.splane[(int64_t)gy * w + gx] = s.so[ty][tx];
  }
  __syncthreads();
}

// ------------------------------------------------------------------ A2
template <int TH>
struct SmemA2 {
  int sk[TH + 4][TW + 4];  // S over the tile + 2 (S >= +0: its bits are its key)
  float spo[TH][TW];       // S' of the tile (full S' plane only)
  unsigned long long g1w[TH], g2w[TH];
  unsigned short blist[TH * TW / 4];  // 2x2 blocks whose S' can decide a threshold
  int cidx[TH * TW];       // the tile's candidates (pixel indices) and their S'
  float csp[TH * TW];
  int nblk, ncand;
  int base;                // offset of the candidates in the frame's list
};

// Step 5 at one candidate pixel (gy, gx): fine structure F = med3 - med7(med3)
// (med7 clamps on med3's own grid), f = F / N floored at 0.01; returns
// whether S' / f exceeds objlim.  Reads C from global memory.  Away from the
// frame edges the 9x9 patch is loaded once; near them every med3 reads its
// own clamped neighbourhood.
__device__ __forceinline__ bool objlim_test(const FrameDev& f, const float* C, int gy, int gx,
                                            float spv) {
  const int h = f.h, w = f.w;
  int v49[49];
  int v25[25];
  if (gy >= 4 && gy < h - 4 && gx >= 4 && gx < w - 4) {
    int p[81];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      const float* row = C + (int64_t)(gy - 4 + a) * w + (gx - 4);
#pragma unroll
      for (int b = 0; b < 9; ++b) p[a * 9 + b] = fkey(row[b]);
    }
    // med3 of every 3x3 window of the patch from its three sorted columns:
    // the median of 9 is med3(max of the column minima, med3 of the column
    // medians, min of the column maxima).
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
#pragma unroll
    for (int a = 0; a < 5; ++a)
#pragma unroll
      for (int b = 0; b < 5; ++b) v25[a * 5 + b] = p[(a + 2) * 9 + (b + 2)];
  } else {
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
          for (int g = 0; g < 3; ++g) v9[e * 3 + g] = fkey(C[row + clampi(qx - 1 + g, w - 1)]);
        }
        v49[a * 7 + b] = med9(v9);
      }
    }
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const int64_t row = (int64_t)clampi(gy - 2 + a, h - 1) * w;
#pragma unroll
      for (int b = 0; b < 5; ++b) v25[a * 5 + b] = fkey(C[row + clampi(gx - 2 + b, w - 1)]);
    }
  }
  const float m3 = funkey(v49[24]);
  const float m7 = funkey(med49(v49));
  const float N = noise_from_med(funkey(med25(v25)), f.gain, f.rn2);
  const float F = m3 - m7;
  const float fr = F / N;
  const float fn = (fr > 0.01f) ? fr : 0.01f;
  return (spv / fn) > f.objlim;
}

// A2.  S' = S - med5(S) only matters through S' > sigclip and
// S' > sigfrac*sigclip, and S' <= S because med5 of S >= +0 is >= +0.  So
// wherever S <= min(sigclip, sigfrac*sigclip) both bits are 0 whatever
// med5(S) is; the 5x5 medians run only for the 2x2 blocks holding a pixel
// above that bound (all blocks with the full-S' flag), compacted into a list
// so every lane has a block.
template <int TH, int NT>
__device__ void tile_a2(const FrameDev& f, int it, int y0, int x0, int tx_word, SmemA2<TH>& s) {
  constexpr int NBLK = (TH / 2) * (TW / 2);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int h = f.h, w = f.w;
  if (tid == 0) {
    s.nblk = 0;
    s.ncand = 0;
  }
  if (tid < TH) s.g1w[tid] = s.g2w[tid] = 0ull;
  for (int i = tid; i < (TH + 4) * (TW + 4); i += NT) {
    const int ly = i / (TW + 4), lx = i - ly * (TW + 4);
    const int cy = clampi(y0 - 2 + ly, h - 1), cx = clampi(x0 - 2 + lx, w - 1);
    s.sk[ly][lx] = __float_as_int(f.splane[(int64_t)cy * w + cx]);
  }
  __syncthreads();
  // blocks that need their medians
  const float tmin = f.tmin;
  for (int blk = tid; blk < NBLK; blk += NT) {
    const int by = (blk / (TW / 2)) * 2, bx = (blk % (TW / 2)) * 2;
    bool need = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ty = by + (q >> 1), tx = bx + (q & 1);
      const bool in = y0 + ty < h && x0 + tx < w;
      need |= in && (f.full_sp || __int_as_float(s.sk[ty + 2][tx + 2]) > tmin);
    }
    const unsigned long long bal = __ballot(need);
    if (bal) {
      int base = 0;
      if (lane == 0) base = atomicAdd(&s.nblk, __popcll(bal));
      base = __shfl(base, 0);
      if (need) s.blist[base + __popcll(bal & ((1ull << lane) - 1ull))] = (unsigned short)blk;
    }
  }
  __syncthreads();
  const int nb = s.nblk;
  const float sigclip = f.sigclip, lo = f.lo;
  for (int i = tid; i < nb; i += NT) {
    const int blk = s.blist[i];
    const int by = (blk / (TW / 2)) * 2, bx = (blk % (TW / 2)) * 2;
    int v[36];
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = 0; b < 6; ++b) v[a * 6 + b] = s.sk[by + a][bx + b];
    int m[4];
    med25_2x2(v, m);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int ty = by + (q >> 1), tx = bx + (q & 1);
      const float S = __int_as_float(s.sk[ty + 2][tx + 2]);
      const float spv = S - funkey(m[q]);
      s.spo[ty][tx] = spv;
      if (y0 + ty < h && x0 + tx < w) {
        const unsigned long long bit = 1ull << tx;
        if (spv > lo) atomicOr(&s.g2w[ty], bit);
        if (spv > sigclip) {
          atomicOr(&s.g1w[ty], bit);
          const int c = atomicAdd(&s.ncand, 1);
          s.cidx[c] = (y0 + ty) * w + (x0 + tx);
          s.csp[c] = spv;
        }
      }
    }
  }
  __syncthreads();
  // one global atomic per tile reserves the tile's part of the frame's list
  if (tid == 0 && s.ncand) s.base = (int)atomicAdd(&f.counts[0], (unsigned int)s.ncand);
  if (f.full_sp) {
    for (int i = tid; i < TH * TW; i += NT) {
      const int ty = i / TW, tx = i - ty * TW;
      const int gy = y0 + ty, gx = x0 + tx;
      if (gy < h && gx < w) f.sp[(int64_t)gy * w + gx] = s.spo[ty][tx];
    }
  }
  if (tid < TH && y0 + tid < h) {
    const int64_t wi = (int64_t)(y0 + tid) * f.wpr + tx_word;
    f.g1[wi] = s.g1w[tid];
    f.g2[wi] = s.g2w[tid];
    f.b1[wi] = 0ull;  // S1 sets the bits of the candidates that pass
  }
  __syncthreads();
  const int nc = s.ncand;
  for (int c = tid; c < nc; c += NT) {
    f.list[s.base + c] = s.cidx[c];
    if (!f.full_sp) f.sp[s.cidx[c]] = s.csp[c];  // S1 reads S' at its candidates
  }
  __syncthreads();
}

// S1 at one listed pixel.
__device__ __forceinline__ void sparse_objlim(const FrameDev& f, int idx) {
  const int gy = idx / f.w, gx = idx - gy * f.w;
  if (objlim_test(f, f.clean, gy, gx, f.sp[idx]))
    atomicOr(reinterpret_cast<unsigned long long*>(f.b1) + (int64_t)gy * f.wpr + (gx >> 6),
             1ull << (gx & 63));
}

// ------------------------------------------------------------------ B
// Pass B: one wave streams down nrows rows of 64 consecutive bit-plane words
// (lane l holds word word0 - 1 + l, so every row is one coalesced 512-byte
// access).  Lanes 0 and 63 are a one-word halo: words word0 .. word0 + 61 are
// produced.  Horizontal neighbours' edge bits come from lane shuffles;
// vertical dilations use the last three rows held in registers.
constexpr int B_WORDS = 62;                // words produced per wave
constexpr int B_WAVES = 4;                 // waves per block, stacked vertically
// rows produced per wave: FrameDev::bstrip (a pass-B tile is 4 strips)

__device__ __forceinline__ unsigned long long word_at(const uint64_t* plane, int y, int word,
                                                      int h, int wpr) {
  return (plane && y >= 0 && y < h && word >= 0 && word < wpr)
             ? plane[(int64_t)y * wpr + word]
             : 0ull;
}

// Horizontal 3-pixel dilation of each lane's word, the neighbouring words'
// edge bits taken from the adjacent lanes.
__device__ __forceinline__ unsigned long long hdil_lanes(unsigned long long v) {
  const unsigned long long left = __shfl_up(v, 1);
  const unsigned long long right = __shfl_down(v, 1);
  return v | (v << 1) | (v >> 1) | (left >> 63) | (right << 63);
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

__device__ void strip_b(const FrameDev& f, int it, int y0, int word0, int nrows) {
  const int lane = threadIdx.x & 63;
  const int h = f.h, w = f.w, wpr = f.wpr;
  const int word = word0 - 1 + lane;
  const bool out_lane = lane >= 1 && lane <= B_WORDS && word < wpr;
  const uint64_t* mprev = mprev_of(f, it);
  uint64_t* mnext = mnext_of(f, it);
  const bool last = it == f.niter - 1;
  const bool skip = stopped(f, it);
  unsigned int fresh = 0, nflag = 0;
  // rolling rows: hd1 of rows t-2, t-1; hd2 of rows t-3, t-2
  unsigned long long hd1a = 0, hd1b = 0, hd2a = 0, hd2b = 0;
  for (int t = 0; t < nrows + 4; ++t) {
    const int r = y0 - 2 + t;  // row whose B1 word is read at this step
    unsigned long long mn = 0;
    int out_row = -1;
    if (skip) {
      if (t >= 4) {
        out_row = r - 2;
        mn = word_at(mprev, out_row, word, h, wpr);
      }
    } else {
      const unsigned long long hd1c = hdil_lanes(word_at(f.b1, r, word, h, wpr));
      if (t >= 2) {
        // B2 of row r-1, then its horizontal dilation
        const unsigned long long b2 = (hd1a | hd1b | hd1c) & word_at(f.g1, r - 1, word, h, wpr);
        const unsigned long long hd2c = hdil_lanes(b2);
        if (t >= 4) {
          // B3 of row r-2; M' = M | B3
          out_row = r - 2;
          const unsigned long long b3 = (hd2a | hd2b | hd2c) & word_at(f.g2, out_row, word, h, wpr);
          const unsigned long long mp = word_at(mprev, out_row, word, h, wpr);
          mn = mp | b3;
          if (out_lane) fresh += (unsigned int)__popcll(b3 & ~mp);
        }
        hd2a = hd2b;
        hd2b = hd2c;
      }
      hd1a = hd1b;
      hd1b = hd1c;
    }
    if (out_row < 0 || out_row >= h) continue;  // uniform over the wave
    if (out_lane && (!last || !skip)) mnext[(int64_t)out_row * wpr + word] = mn;
    if (!skip && out_lane) nflag += (unsigned int)__popcll(mn);
    if (last) {
      // mask bytes: one coalesced 64-byte store per word of the row
      uint8_t* orow = f.out_mask + (int64_t)out_row * w;
      for (int j = 1; j <= B_WORDS; ++j) {
        const unsigned long long wb = __shfl(mn, j);
        const int x = (word0 - 1 + j) * TW + lane;
        if (word0 - 1 + j < wpr && x < w) orow[x] = (uint8_t)((wb >> lane) & 1ull);
      }
    }
  }
  if (!skip) {
    // list the strip's flagged pixels for S2: one atomic per wave, then the
    // words just written are read back (they are in cache) and expanded
    const unsigned int incl = wave_scan(nflag);
    const unsigned int total = __shfl(incl, 63);
    if (total) {
      unsigned int base = 0;
      if (lane == 63) base = atomicAdd(&f.counts[1], total);
      base = __shfl(base, 63);
      int k = (int)(base + incl - nflag);
      if (out_lane) {
        const int yend = min(y0 + nrows, h);
        for (int y = y0; y < yend; ++y) {
          unsigned long long bits = mnext[(int64_t)y * wpr + word];
          while (bits) {
            const int b = __ffsll((long long)bits) - 1;
            bits &= bits - 1;
            f.list[k++] = y * w + word * TW + b;
          }
        }
      }
    }
  }
  if (!skip) {
    for (int off = 32; off > 0; off >>= 1) fresh += __shfl_down(fresh, off);
    if (lane == 0 && fresh) atomicAdd(&f.n_new[it], (unsigned long long)fresh);
  }
}

// S2 at one listed (flagged) pixel: lower median of the un-flagged values of
// its clamped 5x5 window; unchanged if every cell is flagged.
__device__ __forceinline__ void sparse_replace(const FrameDev& f, int it, int idx) {
  const int h = f.h, w = f.w, wpr = f.wpr;
  const int gy = idx / w, gx = idx - gy * w;
  const uint64_t* m = mnext_of(f, it);
  float* C = f.clean;
  int v[25];
  int n = 0;
#pragma unroll
  for (int a = 0; a < 5; ++a) {
    const int qy = clampi(gy - 2 + a, h - 1);
    const int64_t row = (int64_t)qy * w;
    const uint64_t* mrow = m + (int64_t)qy * wpr;
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      const int qx = clampi(gx - 2 + b, w - 1);
      const bool use = ((mrow[qx >> 6] >> (qx & 63)) & 1ull) == 0ull;
      v[a * 5 + b] = use ? fkey(C[row + qx]) : KEY_EXCLUDED;
      n += use ? 1 : 0;
    }
  }
  if (n > 0) {
    int srt[25];
    sort25(v, srt);
    const int r = (n - 1) >> 1;  // lower median of the n un-flagged values
    int sel = srt[0];
#pragma unroll
    for (int k = 1; k < 13; ++k) sel = (r == k) ? srt[k] : sel;
    C[(int64_t)gy * w + gx] = funkey(sel);
  }
}


// S1 (WHICH = 0) or S2 (WHICH = 1) over one frame's list; the list length
// was fixed by the previous launch.
template <int WHICH>
__device__ __forceinline__ void sparse_frame(const FrameDev& f, int it, int gtid, int gstride) {
  if (stopped(f, it)) return;
  const int n = (int)f.counts[WHICH];
  for (int i = gtid; i < n; i += gstride) {
    const int idx = f.list[i];
    if (WHICH == 0)
      sparse_objlim(f, idx);
    else
      sparse_replace(f, it, idx);
  }
}

}  // namespace lac
