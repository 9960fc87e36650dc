// HIP kernels of the L.A.Cosmic iteration for gfx950 (MI355X).
//
// One iteration is two launches over tiles of TH x TW output pixels:
//
//  pass A  (steps 1-5 of the method): stages the current image C of the tile
//          plus a 4-pixel ring in LDS; computes the Laplacian edge image L,
//          the noise model N and S = L / (2N) over the tile plus a 2-pixel
//          ring (clamped to the frame); S' = S - med5(S) on the tile, written
//          to HBM; the candidate test S' > sigclip, and, for candidates only,
//          the fine-structure ratio test S' / max((med3 - med7(med3)) / N,
//          0.01) > objlim, written as a 0/1 byte plane.  The ratio test is a
//          conjunction with S' > sigclip, so med7(med3) is evaluated at the
//          (sparse) pixels where it decides the result.
//  pass B  (steps 6-7): two 3x3 dilations thresholded on S' (tile plus a
//          3- and 2-pixel ring), the cumulative mask M' = M | B3 (written
//          ping-pong, never in place), the count of new pixels, and the
//          replacement of flagged pixels by the lower median of their
//          un-flagged 5x5 neighbours.  C is updated in place only at flagged
//          pixels, and no tile reads a flagged pixel's value, so tiles never
//          race on C.
//
// All medians run on 32-bit keys whose signed order is the float order, with
// min/max networks (v_min3/v_max3/v_med3_i32), so they select exactly.  All
// arithmetic is binary32 in the same expression order as a plain evaluation
// of the method, compiled with -ffp-contract=off and IEEE division/sqrt.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lacosmic_device.h"
#include "lacosmic_launch.h"
#include "median_net.gen.h"

namespace lac {

constexpr int NT = 256;  // threads per block (4 waves of 64)
constexpr int KEY_EXCLUDED = 0x7fffffff;  // above every finite or infinite float key

__device__ __forceinline__ int fkey(float f) {
  const int b = __float_as_int(f);
  return b ^ ((b >> 31) & 0x7fffffff);
}
__device__ __forceinline__ float funkey(int k) {
  return __int_as_float(k ^ ((k >> 31) & 0x7fffffff));
}
__device__ __forceinline__ int clampi(int v, int hi) { return v < 0 ? 0 : (v > hi ? hi : v); }
__device__ __forceinline__ bool finite_bits(float v) {
  return (__float_as_uint(v) & 0x7f800000u) != 0x7f800000u;
}

__device__ __forceinline__ const float* src_of(const FrameDev& f, int it) {
  return it == 0 ? f.img : f.clean;
}
__device__ __forceinline__ const uint8_t* mprev_of(const FrameDev& f, int it) {
  return it == 0 ? nullptr : f.mbuf[(it - 1) & 1];
}
__device__ __forceinline__ uint8_t* mnext_of(const FrameDev& f, int it) {
  return it == f.niter - 1 ? f.out_mask : f.mbuf[it & 1];
}
// With early stop, iteration it is skipped when iteration it-1 added nothing.
__device__ __forceinline__ bool stopped(const FrameDev& f, int it) {
  return f.early_stop && it > 0 && f.n_new[it - 1] == 0ull;
}

// Logical tile of a block: consecutive tiles go to the same XCD (blocks are
// dispatched round-robin over the 8 XCDs), so neighbouring tiles share their
// halo rows in that XCD's L2.
__device__ __forceinline__ int xcd_remap(int b, int n) {
  const int q = n >> 3, rem = n & 7;
  const int x = b & 7, j = b >> 3;
  return x * q + (x < rem ? x : rem) + j;
}

// ---------------------------------------------------------------- step 1
// Laplacian edge image at one pixel from its clamped 4-neighbourhood.  The
// 2x replicated pixel has four sub-pixels; each sees the Laplacian kernel's
// taps (-up, -left, +4 centre, -right, -down, summed in that order) on the
// replicated grid, is clipped at zero, and the four are averaged.
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

// ---------------------------------------------------------------- step 2
__device__ __forceinline__ float noise_from_med(float m5, float gain, float rn2) {
  const float m = (m5 > 1e-4f) ? m5 : 1e-4f;
  const float var = gain * m + rn2;
  return sqrtf(var) / gain;
}

template <int TH, int TW>
struct SmemA {
  int ck[TH + 8][TW + 8];    // keys of C over the tile + 4
  float cf[TH + 8][TW + 8];  // C over the tile + 4
  int sk[TH + 4][TW + 4];    // S over the tile + 2 (S >= +0, so bits are keys)
  float csp[TH * TW];        // S' of each candidate
  unsigned short cidx[TH * TW];
  int ncand;
};

template <int TH, int TW>
__device__ __forceinline__ int med25_c(const SmemA<TH, TW>& s, int ly, int lx) {
  int v[25];
#pragma unroll
  for (int a = 0; a < 5; ++a)
#pragma unroll
    for (int b = 0; b < 5; ++b) v[a * 5 + b] = s.ck[ly - 2 + a][lx - 2 + b];
  return med25(v);
}

template <int TH, int TW>
__device__ void tile_pass_a(const FrameDev& f, int it, int y0, int x0, SmemA<TH, TW>& s) {
  const int tid = threadIdx.x;
  const int h = f.h, w = f.w;
  const float* src = src_of(f, it);
  if (tid == 0) s.ncand = 0;

  // Stage C (canonical: -0 becomes +0) over the tile + 4, clamped.
  int bad = 0;
  for (int i = tid; i < (TH + 8) * (TW + 8); i += NT) {
    const int ly = i / (TW + 8), lx = i - ly * (TW + 8);
    const int cy = clampi(y0 - 4 + ly, h - 1), cx = clampi(x0 - 4 + lx, w - 1);
    const float v = src[(int64_t)cy * w + cx] + 0.0f;
    bad |= !finite_bits(v);
    s.cf[ly][lx] = v;
    s.ck[ly][lx] = fkey(v);
  }
  if (it == 0 && bad) atomicOr(f.status, 1);
  __syncthreads();

  // Steps 1-3: S over the tile + 2.  A ring position outside the frame holds
  // S of its clamped in-frame position (med5(S) clamps on S's own grid).
  for (int i = tid; i < (TH + 4) * (TW + 4); i += NT) {
    const int sy = i / (TW + 4), sx = i - sy * (TW + 4);
    const int ly = clampi(y0 - 2 + sy, h - 1) - y0 + 4;
    const int lx = clampi(x0 - 2 + sx, w - 1) - x0 + 4;
    const float L = lap_edge(s.cf[ly][lx], s.cf[ly - 1][lx], s.cf[ly + 1][lx], s.cf[ly][lx - 1],
                             s.cf[ly][lx + 1]);
    const float N = noise_from_med(funkey(med25_c(s, ly, lx)), f.gain, f.rn2);
    const float S = L / (2.0f * N);
    s.sk[sy][sx] = __float_as_int(S);
  }
  __syncthreads();

  // Step 3 (cont.) and step 4: S' = S - med5(S); candidates S' > sigclip.
  for (int i = tid; i < TH * TW; i += NT) {
    const int ty = i / TW, tx = i - ty * TW;
    const int gy = y0 + ty, gx = x0 + tx;
    if (gy >= h || gx >= w) continue;
    int v[25];
#pragma unroll
    for (int a = 0; a < 5; ++a)
#pragma unroll
      for (int b = 0; b < 5; ++b) v[a * 5 + b] = s.sk[ty + a][tx + b];
    const float S = __int_as_float(s.sk[ty + 2][tx + 2]);
    const float spv = S - funkey(med25(v));
    const int64_t p = (int64_t)gy * w + gx;
    f.sp[p] = spv;
    if (spv > f.sigclip) {
      const int c = atomicAdd(&s.ncand, 1);
      s.cidx[c] = (unsigned short)i;
      s.csp[c] = spv;
    } else {
      f.cand[p] = 0;
    }
  }
  __syncthreads();

  // Step 5 at candidates: F = med3 - med7(med3) (med7 clamps on med3's own
  // grid), f = F / N floored at 0.01, keep if S' / f > objlim.
  const int nc = s.ncand;
  for (int c = tid; c < nc; c += NT) {
    const int i = s.cidx[c];
    const int ty = i / TW, tx = i - ty * TW;
    const int gy = y0 + ty, gx = x0 + tx;
    int v49[49];
#pragma unroll
    for (int a = 0; a < 7; ++a) {
      const int ly = clampi(gy - 3 + a, h - 1) - y0 + 4;
#pragma unroll
      for (int b = 0; b < 7; ++b) {
        const int lx = clampi(gx - 3 + b, w - 1) - x0 + 4;
        int v9[9];
#pragma unroll
        for (int e = 0; e < 3; ++e)
#pragma unroll
          for (int g = 0; g < 3; ++g) v9[e * 3 + g] = s.ck[ly - 1 + e][lx - 1 + g];
        v49[a * 7 + b] = med9(v9);
      }
    }
    const float m3 = funkey(v49[24]);
    const float m7 = funkey(med49(v49));
    const float F = m3 - m7;
    const float N = noise_from_med(funkey(med25_c(s, ty + 4, tx + 4)), f.gain, f.rn2);
    const float fr = F / N;
    const float fn = (fr > 0.01f) ? fr : 0.01f;
    f.cand[(int64_t)gy * w + gx] = ((s.csp[c] / fn) > f.objlim) ? 1 : 0;
  }
  __syncthreads();
}

template <int TH, int TW>
struct SmemB {
  uint8_t b1[TH + 8][TW + 8];  // candidates over the tile + 4 (0 outside the frame)
  uint8_t b2[TH + 6][TW + 6];  // first growth over the tile + 3
  uint8_t m[TH + 4][TW + 4];   // M' over the tile + 2, at clamped positions
  float sp[TH + 6][TW + 6];    // S' over the tile + 3
  unsigned short ridx[TH * TW];
  int nrep;
  unsigned int fresh;
};

// Lower median of the keys not equal to KEY_EXCLUDED: the r-th smallest of
// all 25 with r = (n - 1) / 2 (excluded keys sort last).
__device__ __forceinline__ int select_rank25(const int* v, int r) {
  int res = KEY_EXCLUDED;
#pragma unroll
  for (int i = 0; i < 25; ++i) {
    int lt = 0, le = 0;
#pragma unroll
    for (int j = 0; j < 25; ++j) {
      lt += v[j] < v[i];
      le += v[j] <= v[i];
    }
    res = (lt <= r && r < le) ? v[i] : res;
  }
  return res;
}

template <int TH, int TW>
__device__ void tile_pass_b(const FrameDev& f, int it, int y0, int x0, SmemB<TH, TW>& s) {
  const int tid = threadIdx.x;
  const int h = f.h, w = f.w;
  const uint8_t* mprev = mprev_of(f, it);
  uint8_t* mnext = mnext_of(f, it);
  const float* src = src_of(f, it);
  if (tid == 0) {
    s.nrep = 0;
    s.fresh = 0;
  }
  for (int i = tid; i < (TH + 8) * (TW + 8); i += NT) {
    const int ly = i / (TW + 8), lx = i - ly * (TW + 8);
    const int gy = y0 - 4 + ly, gx = x0 - 4 + lx;
    const bool in = gy >= 0 && gy < h && gx >= 0 && gx < w;
    s.b1[ly][lx] = in ? f.cand[(int64_t)gy * w + gx] : 0;
  }
  for (int i = tid; i < (TH + 6) * (TW + 6); i += NT) {
    const int ly = i / (TW + 6), lx = i - ly * (TW + 6);
    const int gy = y0 - 3 + ly, gx = x0 - 3 + lx;
    const bool in = gy >= 0 && gy < h && gx >= 0 && gx < w;
    s.sp[ly][lx] = in ? f.sp[(int64_t)gy * w + gx] : 0.0f;
  }
  __syncthreads();

  // Step 6a: B2 = dil3(B1) and S' > sigclip, over the tile + 3 (0 outside).
  for (int i = tid; i < (TH + 6) * (TW + 6); i += NT) {
    const int ly = i / (TW + 6), lx = i - ly * (TW + 6);
    const int gy = y0 - 3 + ly, gx = x0 - 3 + lx;
    uint8_t v = 0;
    if (gy >= 0 && gy < h && gx >= 0 && gx < w) {
      const uint8_t d = s.b1[ly][lx] | s.b1[ly][lx + 1] | s.b1[ly][lx + 2] |
                        s.b1[ly + 1][lx] | s.b1[ly + 1][lx + 1] | s.b1[ly + 1][lx + 2] |
                        s.b1[ly + 2][lx] | s.b1[ly + 2][lx + 1] | s.b1[ly + 2][lx + 2];
      v = (d && s.sp[ly][lx] > f.sigclip) ? 1 : 0;
    }
    s.b2[ly][lx] = v;
  }
  __syncthreads();

  // Step 6b and accumulation: B3 = dil3(B2) and S' > sigfrac*sigclip;
  // M' = M | B3 over the tile + 2 at clamped positions.
  unsigned int fresh = 0;
  for (int i = tid; i < (TH + 4) * (TW + 4); i += NT) {
    const int ly = i / (TW + 4), lx = i - ly * (TW + 4);
    const int uy = y0 - 2 + ly, ux = x0 - 2 + lx;
    const int cy = clampi(uy, h - 1), cx = clampi(ux, w - 1);
    const int by = cy - y0 + 3, bx = cx - x0 + 3;
    const uint8_t d = s.b2[by - 1][bx - 1] | s.b2[by - 1][bx] | s.b2[by - 1][bx + 1] |
                      s.b2[by][bx - 1] | s.b2[by][bx] | s.b2[by][bx + 1] |
                      s.b2[by + 1][bx - 1] | s.b2[by + 1][bx] | s.b2[by + 1][bx + 1];
    const uint8_t b3 = (d && s.sp[by][bx] > f.lo) ? 1 : 0;
    const int64_t q = (int64_t)cy * w + cx;
    const uint8_t mp = mprev ? mprev[q] : 0;
    const uint8_t mn = mp | b3;
    s.m[ly][lx] = mn;
    if (uy == cy && ux == cx && ly >= 2 && ly < TH + 2 && lx >= 2 && lx < TW + 2) {
      mnext[q] = mn;
      fresh += (b3 && !mp) ? 1u : 0u;
    }
  }
  if (fresh) atomicAdd(&s.fresh, fresh);
  __syncthreads();
  if (tid == 0 && s.fresh) atomicAdd(&f.n_new[it], (unsigned long long)s.fresh);

  // Step 7: list the flagged pixels of the tile; iteration 0 also copies the
  // un-flagged ones into C.
  for (int i = tid; i < TH * TW; i += NT) {
    const int ty = i / TW, tx = i - ty * TW;
    const int gy = y0 + ty, gx = x0 + tx;
    if (gy >= h || gx >= w) continue;
    if (s.m[ty + 2][tx + 2]) {
      const int c = atomicAdd(&s.nrep, 1);
      s.ridx[c] = (unsigned short)i;
    } else if (it == 0) {
      const int64_t p = (int64_t)gy * w + gx;
      f.clean[p] = src[p] + 0.0f;
    }
  }
  __syncthreads();
  const int nr = s.nrep;
  for (int c = tid; c < nr; c += NT) {
    const int i = s.ridx[c];
    const int ty = i / TW, tx = i - ty * TW;
    const int gy = y0 + ty, gx = x0 + tx;
    int v[25];
    int n = 0;
#pragma unroll
    for (int a = 0; a < 5; ++a) {
      const int qy = clampi(gy - 2 + a, h - 1);
#pragma unroll
      for (int b = 0; b < 5; ++b) {
        const int qx = clampi(gx - 2 + b, w - 1);
        const bool use = s.m[qy - y0 + 2][qx - x0 + 2] == 0;
        v[a * 5 + b] = use ? fkey(src[(int64_t)qy * w + qx] + 0.0f) : KEY_EXCLUDED;
        n += use ? 1 : 0;
      }
    }
    const int64_t p = (int64_t)gy * w + gx;
    f.clean[p] = (n == 0) ? src[p] + 0.0f : funkey(select_rank25(v, (n - 1) >> 1));
  }
  __syncthreads();
}

// With early stop, a skipped pass B still hands the mask on unchanged.
template <int TH, int TW>
__device__ void tile_copy_mask(const FrameDev& f, int it, int y0, int x0) {
  const uint8_t* mprev = mprev_of(f, it);
  uint8_t* mnext = mnext_of(f, it);
  for (int i = threadIdx.x; i < TH * TW; i += NT) {
    const int ty = i / TW, tx = i - ty * TW;
    const int gy = y0 + ty, gx = x0 + tx;
    if (gy >= f.h || gx >= f.w) continue;
    const int64_t p = (int64_t)gy * f.w + gx;
    mnext[p] = mprev[p];
  }
}

// ------------------------------------------------------------ plain kernels
template <int TH, int TW>
__global__ __launch_bounds__(NT) void k_pass_a(FrameDev f, int it) {
  __shared__ SmemA<TH, TW> s;
  if (stopped(f, it)) return;
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int ty = t / f.tiles_x, tx = t - ty * f.tiles_x;
  tile_pass_a<TH, TW>(f, it, ty * TH, tx * TW, s);
}

template <int TH, int TW>
__global__ __launch_bounds__(NT) void k_pass_b(FrameDev f, int it) {
  __shared__ SmemB<TH, TW> s;
  const int t = xcd_remap(blockIdx.x, gridDim.x);
  const int ty = t / f.tiles_x, tx = t - ty * f.tiles_x;
  if (stopped(f, it)) {
    tile_copy_mask<TH, TW>(f, it, ty * TH, tx * TW);
    return;
  }
  tile_pass_b<TH, TW>(f, it, ty * TH, tx * TW, s);
}

__global__ void k_init(unsigned long long* n_new, int niter, int* status) {
  for (int i = threadIdx.x; i < niter; i += blockDim.x) n_new[i] = 0ull;
  if (threadIdx.x == 0) *status = 0;
}

// ------------------------------------------------------------ launchers
template <int TH, int TW>
static hipError_t launch_iter_t(const FrameDev& f, int it, hipStream_t st) {
  const unsigned nb = (unsigned)f.tiles;
  k_pass_a<TH, TW><<<nb, NT, 0, st>>>(f, it);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  k_pass_b<TH, TW><<<nb, NT, 0, st>>>(f, it);
  return hipGetLastError();
}

TileShape tile_shape(int cfg) {
  switch (cfg) {
    case 1: return TileShape{32, 64};
    case 2: return TileShape{8, 64};
    default: return TileShape{16, 64};
  }
}

hipError_t launch_init(unsigned long long* n_new, int niter, int* status, hipStream_t st) {
  k_init<<<1, 256, 0, st>>>(n_new, niter, status);
  return hipGetLastError();
}

hipError_t launch_iteration(const FrameDev& f, int it, int cfg, hipStream_t st) {
  switch (cfg) {
    case 1: return launch_iter_t<32, 64>(f, it, st);
    case 2: return launch_iter_t<8, 64>(f, it, st);
    default: return launch_iter_t<16, 64>(f, it, st);
  }
}

}  // namespace lac
