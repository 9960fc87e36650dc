// Gain estimation on the device, for frames whose gain is not supplied
// (Methods, "Main parameters": the gain is then estimated at each
// iteration).  The estimate of an iteration comes from the current image C:
//
//   1. sigma clipping: starting from every pixel, up to 5 rounds, each
//      keeping the values within 3 standard deviations (population) of the
//      lower median of the values kept so far; a round that keeps every value
//      ends the clipping;
//   2. the mean m and variance v (population) of the kept values;
//   3. g = (m + sqrt(m^2 + 4 v rn^2)) / (2 v): the gain for which the noise
//      model's variance of a pixel in ADU, m / g + rn^2 / g^2, equals v.
//
// All of it in binary64.  The sums are exact: each value x = M 2^(e-150)
// (M its 24-bit significand, e its biased exponent, at least 1) adds M to an
// integer accumulator of its exponent (positive and negative values apart),
// and M^2 = Mh^2 2^24 + Mh Ml 2^13 + Ml^2 (Mh, Ml the 12-bit halves) adds to
// three more, every partial sum below 2^55; the accumulators of all exponents
// are then added as one wide integer and rounded once to binary64.  So the
// sums, and everything computed from them, do not depend on the order in
// which the pixels were visited.
//
// A clipping round keeps the values x with |x - median| <= 3 sd (in
// binary64), a set that is an interval of binary32 values (the test is
// monotone on either side of the median); the rounds intersect such
// intervals, so the kept set is always one interval [lo, hi] of
// order-preserving 32-bit keys, and every pass filters on it.
//
// The median is a radix selection over the keys in three passes (key bits
// 31-20, 19-10, 9-0), each a histogram of the values in the interval that
// share the digits found so far.  The first pass of a round also forms the
// sums.  Each pass is one launch over the frame's pixels; its last block to
// finish (a counter taken after a device-scope fence) reads the histogram
// and sums, takes the round's decisions and clears them for the next pass.
// The estimate ends after a round that keeps every value or after 5 rounds;
// the launches of the rounds not needed return at once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lacosmic_device.h"
#include "lacosmic_mem.h"

namespace lac {

// Order-preserving 32-bit key of a binary32 value (unsigned order).
__device__ __forceinline__ uint32_t gkey(float x) {
  const uint32_t b = __float_as_uint(x);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float gkey_value(uint32_t k) {
  return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

__device__ __forceinline__ uint32_t gain_atomic_load(const uint32_t* p) {
  return __hip_atomic_load(gp(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long gain_atomic_load(const unsigned long long* p) {
  return __hip_atomic_load(gp(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Pixel i of the current image, canonical (-0 as +0): the input in
// iteration 0 (float32 or uint16), the cleaned image after that -- which the
// fused small-frame launches keep alternately in the output image and the
// workspace's first list plane, the previous iteration's output holding it.
__device__ __forceinline__ float gain_pixel(const FrameDev& f, int it, int64_t i) {
  if (it > 0) {
    const float* c = (!f.fused || ((f.niter - it) & 1) == 0) ? f.clean
                                                             : reinterpret_cast<const float*>(f.list);
    return ldg(c, i);
  }
  if (f.img16) return (float)ldg(f.img16, i);
  return ldg(f.img, i) + 0.0f;
}

// ---------------------------------------------------------- wide integers
// Adds v * 2^shift to the nl-limb unsigned integer L (little-endian limbs).
__device__ __forceinline__ void big_add(uint64_t* L, int nl, uint64_t v, int shift) {
  int w = shift >> 6;
  const int s = shift & 63;
  uint64_t lo = v << s, hi = s ? (v >> (64 - s)) : 0ull;
  uint64_t carry = 0;
  for (; w < nl; ++w) {
    const uint64_t a = L[w];
    const uint64_t add = lo;
    uint64_t t = a + add;
    uint64_t c1 = t < a ? 1ull : 0ull;
    const uint64_t t2 = t + carry;
    c1 += t2 < t ? 1ull : 0ull;
    L[w] = t2;
    carry = c1;
    lo = hi;
    hi = 0;
    if (!lo && !carry) break;
  }
}

// a <- a - b for a >= b.
__device__ __forceinline__ void big_sub(uint64_t* a, const uint64_t* b, int nl) {
  uint64_t borrow = 0;
  for (int w = 0; w < nl; ++w) {
    const uint64_t x = a[w], y = b[w];
    const uint64_t d = x - y;
    const uint64_t d2 = d - borrow;
    borrow = (x < y ? 1ull : 0ull) | (d < borrow ? 1ull : 0ull);
    a[w] = d2;
  }
}

__device__ __forceinline__ bool big_less(const uint64_t* a, const uint64_t* b, int nl) {
  for (int w = nl - 1; w >= 0; --w)
    if (a[w] != b[w]) return a[w] < b[w];
  return false;
}

__device__ __forceinline__ int big_bit(const uint64_t* L, int p) { return (int)((L[p >> 6] >> (p & 63)) & 1ull); }

// The value L * 2^lsb_exp rounded to the nearest binary64 (ties to even).
__device__ double big_to_double(const uint64_t* L, int nl, int lsb_exp) {
  int top = nl - 1;
  while (top >= 0 && L[top] == 0ull) --top;
  if (top < 0) return 0.0;
  int p = top * 64 + 63 - __clzll((long long)L[top]);  // most significant set bit
  if (p < 53) return ldexp((double)L[0], lsb_exp);
  const int lo = p - 52;  // the 53 bits [lo, p] form the significand
  uint64_t m = L[lo >> 6] >> (lo & 63);
  if ((lo & 63) && (lo >> 6) + 1 < nl) m |= L[(lo >> 6) + 1] << (64 - (lo & 63));
  m &= (1ull << 53) - 1ull;
  const int guard = big_bit(L, lo - 1);  // lo >= 1: p >= 53
  bool sticky = false;                   // any set bit in [0, lo - 2]
  const int last = lo - 2;
  if (last >= 0) {
    const int lw = last >> 6;
    for (int w = 0; w < lw; ++w) sticky = sticky || L[w] != 0ull;
    const uint64_t below = ((last & 63) == 63) ? ~0ull : ((2ull << (last & 63)) - 1ull);
    sticky = sticky || (L[lw] & below) != 0ull;
  }
  if (guard && (sticky || (m & 1ull))) {
    m += 1ull;
    if (m >> 53) {
      m >>= 1;
      p += 1;
    }
  }
  return ldexp((double)m, p - 52 + lsb_exp);
}

// ---------------------------------------------------------- noise coefficients
// The per-iteration constants of the noise model for gain g: the exact
// reciprocal when g is a power of two whose reciprocal is a normal number, and
// whether the variance at the median floor, fl(fl(g * 1e-4) + rn2), is at
// least 2^-96 (then the square root skips its small-argument path).
__device__ __forceinline__ NoiseCoef noise_coef_for(float g, float rn2) {
  NoiseCoef c;
  c.gain = g;
  const uint32_t b = __float_as_uint(g);
  const float r = 1.0f / g;
  const bool pow2 = (b & 0x007fffffu) == 0u && ((b >> 23) & 0xffu) != 0u;
  const uint32_t rb = __float_as_uint(r);
  const bool rnormal = ((rb >> 23) & 0xffu) != 0u && ((rb >> 23) & 0xffu) != 0xffu;
  c.inv_gain = (pow2 && rnormal && r * g == 1.0f) ? r : 0.0f;
  const float gm = g * 1e-4f;
  const float vmin = gm + rn2;
  c.fast_sqrt = vmin >= 0x1p-96f ? 1 : 0;
  c.valid = 1;
  return c;
}

// ---------------------------------------------------------- passes
constexpr int kGainBins0 = 4096;  // key bits 31-20
constexpr int kGainBins = 1024;   // key bits 19-10, then 9-0
constexpr int kGainRounds = 5;
constexpr int kGainThreads = 256;
// Passes launched per iteration: 5 rounds of three, then the sums of the
// values kept after the fifth.
constexpr int kGainLaunches = 3 * kGainRounds + 1;

struct GainShared {
  unsigned int hist[kGainBins0];
  unsigned long long acc[5][256];  // by exponent: sum M (x > 0), sum M (x < 0), Mh^2, Mh Ml, Ml^2
  unsigned int part[kGainThreads];
  int last, done, bin;
  uint32_t rank;
};

// Resets the frame's estimator at the start of an iteration.
__device__ __forceinline__ void gain_reset(const FrameDev& f) {
  GainWork* g = f.gw;
  for (int i = threadIdx.x; i < kGainBins0; i += blockDim.x) stg(g->hist, i, 0u);
  for (int i = threadIdx.x; i < 5 * 256; i += blockDim.x) stg(&g->acc[0][0], i, 0ull);
  if (threadIdx.x == 0) {
    g->klo = 0u;
    g->khi = 0xffffffffu;
    g->prefix = 0u;
    g->rank = 0u;
    g->round = 0;
    g->done = 0;
    g->blocks_done = 0u;
    g->n_prev = -1;
    g->n_cur = 0;
    g->mean = 0.0;
    g->var = 0.0;
  }
}

// Adds `add` to LDS counter slot key of the lanes that share each distinct
// key (pred lanes only): one LDS atomic per distinct key in the wave.
__device__ __forceinline__ void wave_hist_add(unsigned int* hist, int key, bool pred) {
  unsigned long long pending = __ballot(pred);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int k = __shfl(key, leader);
    const unsigned long long same = __ballot(pred && key == k);
    if ((int)(threadIdx.x & 63) == leader) atomicAdd(&hist[k], (unsigned int)__popcll(same));
    pending &= ~same;
  }
}

// Wave sum of a 32-bit value (every lane of the wave calls it).
__device__ __forceinline__ unsigned int wave_sum_u32(unsigned int v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// Exact sums of one value per lane (pred lanes), grouped by exponent: one
// set of LDS atomics per distinct exponent in the wave.
__device__ __forceinline__ void wave_sums_add(GainShared& sh, float x, bool pred) {
  const uint32_t b = __float_as_uint(x);
  const int ex = (int)((b >> 23) & 0xffu);
  const int e = ex ? ex : 1;
  const uint32_t M = (b & 0x007fffffu) | (ex ? 0x00800000u : 0u);
  const bool neg = (b >> 31) != 0u;
  const uint32_t mh = M >> 12, ml = M & 0xfffu;
  unsigned long long pending = __ballot(pred);
  while (pending) {
    const int leader = __ffsll((long long)pending) - 1;
    const int k = __shfl(e, leader);
    const bool mine = pred && e == k;
    // each term < 2^24, so a wave's sum < 2^30 fits 32 bits
    const unsigned int sp = wave_sum_u32(mine && !neg ? M : 0u);
    const unsigned int sn = wave_sum_u32(mine && neg ? M : 0u);
    const unsigned int sa = wave_sum_u32(mine ? mh * mh : 0u);
    const unsigned int sb = wave_sum_u32(mine ? mh * ml : 0u);
    const unsigned int sc = wave_sum_u32(mine ? ml * ml : 0u);
    if ((int)(threadIdx.x & 63) == leader) {
      if (sp) atomicAdd(&sh.acc[0][k], (unsigned long long)sp);
      if (sn) atomicAdd(&sh.acc[1][k], (unsigned long long)sn);
      if (sa) atomicAdd(&sh.acc[2][k], (unsigned long long)sa);
      if (sb) atomicAdd(&sh.acc[3][k], (unsigned long long)sb);
      if (sc) atomicAdd(&sh.acc[4][k], (unsigned long long)sc);
    }
    pending &= ~__ballot(mine);
  }
}

// Block-wide search of the bin holding rank `rank` in the nb-bin global
// histogram hist (read coherently): returns the bin, and the rank within it
// in *rank_in.  Every thread of the block calls it.
__device__ int gain_find_bin(GainShared& sh, const unsigned int* hist, int nb, uint32_t rank,
                             uint32_t* rank_in) {
  const int per = nb / kGainThreads;  // bins per thread (16 or 4)
  unsigned int mine = 0;
  for (int j = 0; j < per; ++j) {
    const unsigned int v = gain_atomic_load(&hist[threadIdx.x * per + j]);
    sh.hist[threadIdx.x * per + j] = v;
    mine += v;
  }
  sh.part[threadIdx.x] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t below = 0;
    int t = 0;
    while (t < kGainThreads - 1 && below + sh.part[t] <= rank) below += sh.part[t++];
    int bin = t * per;
    while (bin < t * per + per - 1 && below + sh.hist[bin] <= rank) below += sh.hist[bin++];
    sh.bin = bin;
    sh.rank = rank - below;
  }
  __syncthreads();
  *rank_in = sh.rank;
  return sh.bin;
}

// Smallest (dir < 0) or largest (dir > 0) key of a binary32 value x on that
// side of the median c with |x - c| <= lim in binary64: the clipping test is
// monotone on either side of c, so the kept values form an interval.
__device__ uint32_t clip_bound(float c, double lim, int dir) {
  auto keep = [&](uint32_t k) {
    const float x = gkey_value(k);
    return fabs((double)x - (double)c) <= lim;
  };
  const double t = dir > 0 ? (double)c + lim : (double)c - lim;
  uint32_t k = gkey((float)t);
  const uint32_t kc = gkey(c);
  if (dir > 0) {
    if (k < kc) k = kc;
    while (k > kc && !keep(k)) --k;
    while (k < 0xff800000u && keep(k + 1)) ++k;  // 0xff800000: the key of +inf
  } else {
    if (k > kc) k = kc;
    while (k < kc && !keep(k)) ++k;
    while (k > 0x007fffffu && keep(k - 1)) --k;  // 0x007fffff: the key of -inf
  }
  return k;
}

// The exact sums of a round from the exponent accumulators in LDS, rounded
// once to binary64: *s1 = sum of the values, *s2 = sum of their squares.
__device__ void gain_exact_sums(const GainShared& sh, double* s1, double* s2) {
  // sum x: LSB 2^-149 (exponent 1); M 2^(e-150) is M << (e-1) of it
  uint64_t pos[5] = {0, 0, 0, 0, 0}, negs[5] = {0, 0, 0, 0, 0};
  // sum x^2: LSB 2^-298; M^2 2^(2e-300) = (Mh^2 << 24 + Mh Ml << 13 + Ml^2) << (2e-2)
  uint64_t sq[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int e = 1; e < 256; ++e) {
    if (sh.acc[0][e]) big_add(pos, 5, sh.acc[0][e], e - 1);
    if (sh.acc[1][e]) big_add(negs, 5, sh.acc[1][e], e - 1);
    if (sh.acc[2][e]) big_add(sq, 10, sh.acc[2][e], 2 * e - 2 + 24);
    if (sh.acc[3][e]) big_add(sq, 10, sh.acc[3][e], 2 * e - 2 + 13);
    if (sh.acc[4][e]) big_add(sq, 10, sh.acc[4][e], 2 * e - 2);
  }
  if (big_less(pos, negs, 5)) {
    big_sub(negs, pos, 5);
    *s1 = -big_to_double(negs, 5, -149);
  } else {
    big_sub(pos, negs, 5);
    *s1 = big_to_double(pos, 5, -149);
  }
  *s2 = big_to_double(sq, 10, -298);
}

// The noise-model constants of iteration it from the final mean and
// variance: the estimated gain, or gain 1 when there is no estimate (no
// spread, or a result that is not a positive normal binary32 number).
__device__ NoiseCoef gain_final(const FrameDev& f, double mean, double var) {
  double est = 1.0;
  bool ok = false;
  if (var > 0.0) {
    const double rn = (double)f.readnoise;
    const double rn2 = rn * rn;
    const double gg = (mean + sqrt(mean * mean + 4.0 * var * rn2)) / (2.0 * var);
    const uint32_t fb = __float_as_uint((float)gg);
    const uint32_t fe = (fb >> 23) & 0xffu;
    ok = isfinite(gg) && (fb >> 31) == 0u && fe != 0u && fe != 0xffu;
    if (ok) est = gg;
  }
  NoiseCoef c = noise_coef_for((float)est, f.rn2);
  c.valid = ok ? 1 : 0;
  return c;
}

// One pass of a clipping round (P = 0: count, sums and key bits 31-20;
// 1: bits 19-10; 2: bits 9-0) by block bx of nbx over frame f's pixels.
template <int P>
__device__ __forceinline__ void gain_pass(const FrameDev& f, int it, int bx, int nbx, GainShared& sh) {
  GainWork* g = f.gw;
  if (ldg(&g->done, 0)) return;
  const uint32_t klo = ldg(&g->klo, 0), khi = ldg(&g->khi, 0), prefix = ldg(&g->prefix, 0);
  constexpr int NB = P == 0 ? kGainBins0 : kGainBins;
  for (int i = threadIdx.x; i < NB; i += blockDim.x) sh.hist[i] = 0u;
  if (P == 0)
    for (int i = threadIdx.x; i < 5 * 256; i += blockDim.x) (&sh.acc[0][0])[i] = 0ull;
  __syncthreads();
  const int64_t n = (int64_t)f.h * f.w;
  const int64_t stride = (int64_t)nbx * blockDim.x;
  // whole waves stay in the loop (the wave-aggregated updates use ballots)
  for (int64_t base = (int64_t)bx * blockDim.x + (threadIdx.x & ~63); base < n; base += stride) {
    const int64_t i = base + (threadIdx.x & 63);
    const bool valid = i < n;
    const float x = valid ? gain_pixel(f, it, i) : 0.0f;
    const uint32_t k = gkey(x);
    bool in = valid && k >= klo && k <= khi;
    if (P == 0) {
      wave_hist_add(sh.hist, (int)(k >> 20), in);
      wave_sums_add(sh, x, in);
    } else if (P == 1) {
      in = in && (k >> 20) == prefix;
      if (in) atomicAdd(&sh.hist[(k >> 10) & 0x3ffu], 1u);
    } else {
      in = in && (k >> 10) == prefix;
      if (in) atomicAdd(&sh.hist[k & 0x3ffu], 1u);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < NB; i += blockDim.x)
    if (sh.hist[i]) atom_add(&g->hist[i], sh.hist[i]);
  if (P == 0)
    for (int i = threadIdx.x; i < 5 * 256; i += blockDim.x) {
      const unsigned long long v = (&sh.acc[0][0])[i];
      if (v) atom_add(&(&g->acc[0][0])[i], v);
    }
  // the last block of the frame to finish takes the round's decisions
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    sh.last = atom_add(&g->blocks_done, 1u) == (unsigned int)(nbx - 1) ? 1 : 0;
  }
  __syncthreads();
  if (!sh.last) return;
  __threadfence();
  if (P == 0) {
    unsigned int c = 0;
    for (int i = threadIdx.x; i < NB; i += blockDim.x) c += gain_atomic_load(&g->hist[i]);
    sh.part[threadIdx.x] = c;
    for (int i = threadIdx.x; i < 5 * 256; i += blockDim.x)
      (&sh.acc[0][0])[i] = gain_atomic_load(&(&g->acc[0][0])[i]);
    __syncthreads();
    if (threadIdx.x == 0) {
      long long cnt = 0;
      for (int t = 0; t < kGainThreads; ++t) cnt += sh.part[t];
      double s1 = 0.0, s2 = 0.0;
      gain_exact_sums(sh, &s1, &s2);
      const double mean = s1 / (double)cnt;
      const double var = s2 / (double)cnt - mean * mean;
      g->mean = mean;
      g->var = var;
      g->n_cur = cnt;
      // final after a round that clipped nothing, or after the last round
      const bool fin = cnt == g->n_prev || g->round == kGainRounds;
      if (fin) {
        f.coef[it] = gain_final(f, mean, var);
        g->done = 1;
      }
      sh.done = fin ? 1 : 0;
      sh.rank = (uint32_t)((cnt - 1) / 2);  // rank of the lower median
    }
    __syncthreads();
    if (!sh.done) {
      uint32_t r_in = 0;
      const int bin = gain_find_bin(sh, g->hist, NB, sh.rank, &r_in);
      if (threadIdx.x == 0) {
        g->prefix = (uint32_t)bin;
        g->rank = r_in;
      }
    }
  } else {
    uint32_t r_in = 0;
    const int bin = gain_find_bin(sh, g->hist, NB, g->rank, &r_in);
    if (threadIdx.x == 0) {
      const uint32_t pre = (prefix << 10) | (uint32_t)bin;
      if (P == 1) {
        g->prefix = pre;
        g->rank = r_in;
      } else {  // the lower median is found: the next round's interval
        const float med = gkey_value(pre);
        const double var = g->var;
        const double lim = 3.0 * (var > 0.0 ? sqrt(var) : 0.0);
        const uint32_t a = clip_bound(med, lim, -1), b = clip_bound(med, lim, +1);
        g->klo = a > klo ? a : klo;
        g->khi = b < khi ? b : khi;
        g->n_prev = g->n_cur;
        g->round = g->round + 1;
        g->prefix = 0u;
        g->rank = 0u;
      }
    }
  }
  __syncthreads();
  // clear the global histogram (and sums) for the next pass
  for (int i = threadIdx.x; i < NB; i += blockDim.x) stg(g->hist, i, 0u);
  if (P == 0)
    for (int i = threadIdx.x; i < 5 * 256; i += blockDim.x) stg(&g->acc[0][0], i, 0ull);
  if (threadIdx.x == 0) stg(&g->blocks_done, 0, 0u);
}

}  // namespace lac
