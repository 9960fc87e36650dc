// Fused single-iteration pass for small frames.
//
// On a small frame the sparse passes' chain of short dependent launches
// (about six per iteration) costs more than their work.  One iteration of the
// method reads the previous image only within 8 pixels of an output pixel:
// the replacement reads the new mask within 2, the second growth B2 within 1
// more, the first growth B1 within 1 more, B1 needs S' and the objlim test
// (C within 4) at its pixel, and S' reads S within 2, which reads C within 2.
// So one launch per iteration can run every step for a 32 x 32 output tile
// from a 48 x 48 region of the previous image and mask in LDS:
//
//   1. stage C_k and M_k over the region (clamped coordinates, so a window
//      read at an offset from an in-frame pixel is the clamped window);
//   2. S = L / (2N) at the region's in-frame pixels 2 or more inside it
//      (the shared 2x2 median network), then the out-of-frame cells
//      of that area take the value of their clamped pixel (S's windows clamp
//      on S's own grid);
//   3. S' = S - med5(S) where it can decide a threshold: S > sigfrac*sigclip
//      (S' <= S), within 4 of the tile; G1, G2 and, where G1 holds, the objlim
//      test (49 med3 at clamped positions, med49, med25 for N) give B1;
//   4. B2 = dil3(B1) & G1 within 3, B3 = dil3(B2) & G2 within 2 (out-of-frame
//      cells unset), M_(k+1) = M_k | B3, the tile's new pixels counted;
//   5. the replacement of the tile's mask pixels from C_k and M_(k+1)
//      (clamp-filled), the unreplaceable ones counted as the sparse S2 does;
//   6. C_(k+1), the tile's mask bits (32-bit halves of the 64-bit words, so
//      tiles never share a store), S, S' and B1 for inspection, the mask
//      bytes after the last iteration.
//
// C ping-pongs between the output image and the workspace's first list
// plane, so that the last iteration writes the output; the mask between the
// two mask planes, as on the sparse path.  Every value is computed by the
// same expression as on the sparse path, so results are bit-identical.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lacosmic_device.h"
#include "lacosmic_tiles.h"

namespace lac {

constexpr int FT = 32;            // output tile side
constexpr int FH = 8;             // the iteration's dependency radius
constexpr int FR = FT + 2 * FH;   // region side (48)
constexpr int kFusedThreads = 256;

struct SmemFused {
  float cf[FR][FR];  // C_k at the clamped region coordinates
  int ck[FR][FR];    // their keys
  float sv[FR][FR];  // S (in-frame cells; out-of-frame cells clamp-filled)
  uint8_t mk[FR][FR], mn[FR][FR];            // M_k (clamped), M_(k+1) (clamp-filled)
  uint8_t g1[FR][FR], g2[FR][FR], b1[FR][FR], b2[FR][FR];
  float spv[FR][FR];                          // S' where computed
  uint16_t lst[FR * FR];                      // cells whose S' is computed
  unsigned int nlst, nnew, nunrep;
  int bad;
};

// The image iteration it writes (iteration it + 1 reads it): C ping-pongs
// between the output image and the workspace's first list plane, ending in
// the output (the gain estimate reads it the same way).
__device__ __forceinline__ float* fused_dst(const FrameDev& f, int it) {
  return ((f.niter - 1 - it) & 1) == 0 ? f.clean : reinterpret_cast<float*>(f.list);
}

__device__ __forceinline__ bool fused_in(const FrameDev& f, int gy, int gx) {
  return gy >= 0 && gy < f.h && gx >= 0 && gx < f.w;
}

// Step 5's objlim test at LDS cell (qy, qx) (in-frame): the same arithmetic as
// objlim_test, reading C from the staged region.
__device__ __forceinline__ bool objlim_lds(const FrameDev& f, const NoiseCoef& nc,
                                           const SmemFused& s, int ry0, int rx0, int qy, int qx,
                                           float spv) {
  int v25[25];
#pragma unroll
  for (int a = 0; a < 5; ++a)
#pragma unroll
    for (int b = 0; b < 5; ++b) v25[a * 5 + b] = s.ck[qy - 2 + a][qx - 2 + b];
  const float N = noise_from_med(med25_of(v25, f.sepmed), nc, f.rn2);
  const int gy = ry0 + qy, gx = rx0 + qx;
  int v49[49];
#pragma unroll
  for (int a = 0; a < 7; ++a) {
    const int py = clampi(gy - 3 + a, f.h - 1) - ry0;  // m3 at the clamped position
#pragma unroll
    for (int b = 0; b < 7; ++b) {
      const int px = clampi(gx - 3 + b, f.w - 1) - rx0;
      int v9[9];
#pragma unroll
      for (int e = 0; e < 3; ++e)
#pragma unroll
        for (int g = 0; g < 3; ++g) v9[e * 3 + g] = s.ck[py - 1 + e][px - 1 + g];
      v49[a * 7 + b] = med9_of(v9, f.sepmed);
    }
  }
  const float m3 = funkey(v49[24]);
  const float m7 = funkey(med49_of(v49, f.sepmed));
  const float F = m3 - m7;
  const float fr = F / N;
  const float fn = (fr > 0.01f) ? fr : 0.01f;
  return (spv / fn) > f.objlim;
}

template <int NT>
__device__ __forceinline__ void tile_fused(const FrameDev& f, int it, int tile, SmemFused& s) {
  const int tid = threadIdx.x;
  const int h = f.h, w = f.w;
  const int tiles_x = (w + FT - 1) / FT;
  const int ty = tile / tiles_x, tx = tile - ty * tiles_x;
  const int y0 = ty * FT, x0 = tx * FT;
  const int ry0 = y0 - FH, rx0 = x0 - FH;
  const uint64_t* mprev = mprev_of(f, it);
  uint64_t* mnext = mnext_of(f, it);
  float* dst = fused_dst(f, it);
  const float* src = it == 0 ? f.img : fused_dst(f, it - 1);
  const uint16_t* src16 = it == 0 ? f.img16 : nullptr;
  const bool last = it == f.niter - 1;
  if (tid == 0) {
    s.nlst = 0u;
    s.nnew = 0u;
    s.nunrep = 0u;
    s.bad = 0;
  }
  // 1. stage C_k and M_k over the region
  int bad = 0;
  for (int i = tid; i < FR * FR; i += NT) {
    const int ly = i / FR, lx = i - ly * FR;
    const int gy = clampi(ry0 + ly, h - 1), gx = clampi(rx0 + lx, w - 1);
    const int64_t gi = (int64_t)gy * w + gx;
    const float v = (src16 ? (float)ldg(src16, gi) : ldg(src, gi)) + 0.0f;  // -0 becomes +0
    bad |= !finite_bits(v);
    s.cf[ly][lx] = v;
    s.ck[ly][lx] = fkey(v);
    s.mk[ly][lx] = mprev ? (uint8_t)((ldg(mprev, (int64_t)gy * f.wpr + (gx >> 6)) >> (gx & 63)) & 1ull) : 0;
    s.g1[ly][lx] = s.g2[ly][lx] = s.b1[ly][lx] = s.b2[ly][lx] = s.mn[ly][lx] = 0;
  }
  if (bad) atom_or(f.status, 1);
  __syncthreads();
  if (stopped(f, it)) {  // the mask carries over and C stays: the iteration would repeat
    for (int i = tid; i < FT * FT; i += NT) {
      const int ly = FH + i / FT, lx = FH + i % FT;
      const int gy = ry0 + ly, gx = rx0 + lx;
      if (gy < h && gx < w) {
        stg(dst, (int64_t)gy * w + gx, s.cf[ly][lx]);
        if (last) stg(f.out_mask, (int64_t)gy * w + gx, s.mk[ly][lx]);
      }
    }
    if (tid < FT && y0 + tid < h) {
      uint32_t word = 0;
      for (int b = 0; b < FT; ++b)
        if (x0 + b < w) word |= (uint32_t)s.mk[FH + tid][FH + b] << b;
      stg(reinterpret_cast<uint32_t*>(mnext), ((int64_t)(y0 + tid) * f.wpr + (x0 >> 6)) * 2 + ((x0 >> 5) & 1), word);
    }
    return;
  }
  // 2. S at the in-frame cells of [2, FR - 2), by 2x2 blocks
  const NoiseCoef nc = noise_coef(f, it);
  const float rn2 = f.rn2;
  constexpr int NB = (FR - 4) / 2;  // blocks per side
  for (int blk = tid; blk < NB * NB; blk += NT) {
    const int by = 2 + (blk / NB) * 2, bx = 2 + (blk % NB) * 2;
    const int gy = ry0 + by, gx = rx0 + bx;
    if (!fused_in(f, gy, gx) && !fused_in(f, gy, gx + 1) && !fused_in(f, gy + 1, gx) &&
        !fused_in(f, gy + 1, gx + 1))
      continue;  // no cell of the block is in the frame
    int v[36];
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = 0; b < 6; ++b) v[a * 6 + b] = s.ck[by - 2 + a][bx - 2 + b];
    int m[4];
    med25_block(v, m, f.sepmed);
    auto outputs = [&](auto fast) {  // the noise model's form chosen once
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int ly = by + (q >> 1), lx = bx + (q & 1);
        if (!fused_in(f, ry0 + ly, rx0 + lx)) continue;
        const float L = lap_edge(s.cf[ly][lx], s.cf[ly - 1][lx], s.cf[ly + 1][lx],
                                 s.cf[ly][lx - 1], s.cf[ly][lx + 1]);
        const float N = noise_from_med<decltype(fast)::value>(m[q], nc, rn2);
        s.sv[ly][lx] = L / (2.0f * N);
      }
    };
    if (noise_fast(nc))
      outputs(std::true_type{});
    else
      outputs(std::false_type{});
  }
  __syncthreads();
  for (int i = tid; i < FR * FR; i += NT) {  // clamp-fill S's out-of-frame cells
    const int ly = i / FR, lx = i - ly * FR;
    if (ly < 2 || ly >= FR - 2 || lx < 2 || lx >= FR - 2) continue;
    const int gy = ry0 + ly, gx = rx0 + lx;
    if (fused_in(f, gy, gx)) continue;
    s.sv[ly][lx] = s.sv[clampi(gy, h - 1) - ry0][clampi(gx, w - 1) - rx0];
  }
  __syncthreads();
  // 3. S' where S > sigfrac * sigclip, within 4 of the tile
  const float lo = f.lo, sigclip = f.sigclip;
  for (int i = tid; i < FR * FR; i += NT) {
    const int ly = i / FR, lx = i - ly * FR;
    if (ly < FH - 4 || ly >= FH + FT + 4 || lx < FH - 4 || lx >= FH + FT + 4) continue;
    if (!fused_in(f, ry0 + ly, rx0 + lx) || !(s.sv[ly][lx] > lo)) continue;
    s.lst[atomicAdd(&s.nlst, 1u)] = (uint16_t)i;
  }
  __syncthreads();
  const unsigned int nl = s.nlst;
  for (unsigned int j = tid; j < nl; j += NT) {
    const int i = s.lst[j];
    const int ly = i / FR, lx = i - ly * FR;
    int v[25];
#pragma unroll
    for (int a = 0; a < 5; ++a)
#pragma unroll
      for (int b = 0; b < 5; ++b) v[a * 5 + b] = __float_as_int(s.sv[ly - 2 + a][lx - 2 + b]);
    const float spv = s.sv[ly][lx] - funkey(med25_of(v, f.sepmed));  // S >= +0: bits = key
    s.spv[ly][lx] = spv;
    s.g2[ly][lx] = spv > lo ? 1 : 0;
    if (spv > sigclip) {
      s.g1[ly][lx] = 1;
      s.b1[ly][lx] = objlim_lds(f, nc, s, ry0, rx0, ly, lx, spv) ? 1 : 0;
    }
  }
  __syncthreads();
  // 4. growth: B2 within 3 of the tile, then B3 and M_(k+1) within 2
  for (int i = tid; i < FR * FR; i += NT) {
    const int ly = i / FR, lx = i - ly * FR;
    if (ly < FH - 3 || ly >= FH + FT + 3 || lx < FH - 3 || lx >= FH + FT + 3) continue;
    if (!s.g1[ly][lx]) continue;
    int d = 0;
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
      for (int b = -1; b <= 1; ++b) d |= s.b1[ly + a][lx + b];
    s.b2[ly][lx] = (uint8_t)d;
  }
  __syncthreads();
  unsigned int fresh = 0;
  for (int i = tid; i < FR * FR; i += NT) {
    const int ly = i / FR, lx = i - ly * FR;
    if (ly < FH - 2 || ly >= FH + FT + 2 || lx < FH - 2 || lx >= FH + FT + 2) continue;
    const int gy = ry0 + ly, gx = rx0 + lx;
    if (!fused_in(f, gy, gx)) continue;
    int d = 0;
#pragma unroll
    for (int a = -1; a <= 1; ++a)
#pragma unroll
      for (int b = -1; b <= 1; ++b) d |= s.b2[ly + a][lx + b];
    const int b3 = d & s.g2[ly][lx];
    s.mn[ly][lx] = (uint8_t)(s.mk[ly][lx] | b3);
    const bool own = ly >= FH && ly < FH + FT && lx >= FH && lx < FH + FT;
    if (own && b3 && !s.mk[ly][lx]) ++fresh;
  }
  if (fresh) atomicAdd(&s.nnew, fresh);
  __syncthreads();
  for (int i = tid; i < FR * FR; i += NT) {  // clamp-fill M_(k+1)'s out-of-frame cells
    const int ly = i / FR, lx = i - ly * FR;
    if (ly < FH - 2 || ly >= FH + FT + 2 || lx < FH - 2 || lx >= FH + FT + 2) continue;
    const int gy = ry0 + ly, gx = rx0 + lx;
    if (fused_in(f, gy, gx)) continue;
    s.mn[ly][lx] = s.mn[clampi(gy, h - 1) - ry0][clampi(gx, w - 1) - rx0];
  }
  __syncthreads();
  // 5. replacement of the tile's mask pixels, from C_k under M_(k+1)
  unsigned int unrep = 0;
  for (int i = tid; i < FT * FT; i += NT) {
    const int ly = FH + i / FT, lx = FH + i % FT;
    const int gy = ry0 + ly, gx = rx0 + lx;
    if (gy >= h || gx >= w) continue;
    float out = s.cf[ly][lx];
    if (s.mn[ly][lx]) {
      int v[25];
      int n = 0;
#pragma unroll
      for (int a = 0; a < 5; ++a)
#pragma unroll
        for (int b = 0; b < 5; ++b) {
          const bool use = s.mn[ly - 2 + a][lx - 2 + b] == 0;
          v[a * 5 + b] = use ? s.ck[ly - 2 + a][lx - 2 + b] : KEY_EXCLUDED;
          n += use ? 1 : 0;
        }
      if (n > 0) {
        int srt[13];
        sort25_lo13(v, srt);  // ranks 0..12: the lower median of n <= 25 values
        const int r = (n - 1) >> 1;
        int sel = srt[0];
#pragma unroll
        for (int k = 1; k < 13; ++k) sel = (r == k) ? srt[k] : sel;
        out = funkey(sel);
      } else {
        // counted when the previous mask still left an un-flagged cell (or
        // did not hold the pixel), as the sparse replacement counts it
        bool first = !s.mk[ly][lx];
        for (int a = 0; a < 5 && !first; ++a)
          for (int b = 0; b < 5 && !first; ++b) first = s.mk[ly - 2 + a][lx - 2 + b] == 0;
        unrep += first ? 1u : 0u;
      }
    }
    const int64_t gi = (int64_t)gy * w + gx;
    stg(dst, gi, out);
    if (last) stg(f.out_mask, gi, s.mn[ly][lx]);
    // S, S' (where computed) and B1 for inspection, as the sparse path leaves them
    stg(f.splane, gi, s.sv[ly][lx]);
    if (s.sv[ly][lx] > lo) stg(f.sp, gi, s.spv[ly][lx]);
  }
  if (unrep) atomicAdd(&s.nunrep, unrep);
  // 6. the tile's bits of M_(k+1) and B1: one 32-bit half word per row
  if (tid < 2 * FT) {
    const int row = tid & (FT - 1);
    const bool is_b1 = tid >= FT;
    if (y0 + row < h) {
      uint32_t word = 0;
      for (int b = 0; b < FT; ++b)
        if (x0 + b < w)
          word |= (uint32_t)(is_b1 ? s.b1[FH + row][FH + b] : s.mn[FH + row][FH + b]) << b;
      uint64_t* plane = is_b1 ? f.b1 : mnext;
      stg(reinterpret_cast<uint32_t*>(plane), ((int64_t)(y0 + row) * f.wpr + (x0 >> 6)) * 2 + ((x0 >> 5) & 1), word);
    }
  }
  __syncthreads();
  if (tid == 0) {
    if (s.nnew) atom_add(f.n_new + it, (unsigned long long)s.nnew);
    if (s.nunrep) atom_add(f.n_new + f.niter, (unsigned long long)s.nunrep);
  }
}

}  // namespace lac
