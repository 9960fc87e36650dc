// L.A.Cosmic CPU oracle -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow, obviously-correct CPU implementation of the L.A.Cosmic
// iteration as the dfcosmic paper lists it (Methods, "Algorithm", steps 1-7;
// "Main parameters" for objlim, sigfrac, sigclip, gain and readnoise), with the
// details the paper delegates to van Dokkum (2001) filled in by the readings
// recorded in the design notes (Laplacian kernel and subsampling, noise floor,
// objlim ratio form, growth thresholds, lower median for replacement, nearest
// boundary).
//
// Only the test-suite, the package smoke check and the CPU-baseline leg of the
// benchmark may load this file's library.  The product path (the HIP library)
// shares no code with it.
//
// Every stage keeps a full intermediate image, every window median is a
// std::sort of the window, and every floating-point expression is written in
// the order it is meant to be evaluated.  It is compiled with
// -ffp-contract=off -fno-fast-math so the float instantiation evaluates each
// operation in IEEE binary32 with round-to-nearest-even; the double
// instantiation is the high-precision reference used for error reports.
//
// Threads: an OpenMP "parallel for" over image rows in each stage; the result
// does not depend on the thread count (all reductions are integer counts).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// Constants of the method in the precision of the instantiation.
template <typename T> struct Consts;
template <> struct Consts<float> {
  static constexpr float noise_floor = 1e-4f;  // floor on med5 in the noise model
  static constexpr float fine_floor = 0.01f;   // floor on the fine-structure ratio
};
template <> struct Consts<double> {
  static constexpr double noise_floor = 1e-4;
  static constexpr double fine_floor = 0.01;
};

inline int64_t clampi(int64_t v, int64_t lo, int64_t hi) {
  return v < lo ? lo : (v > hi ? hi : v);
}

// Step 1, "Run laplacian detection".  The image is block-replicated by 2 onto
// a 2h x 2w grid, convolved with the 3x3 Laplacian kernel
//     [[ 0,-1, 0],
//      [-1, 4,-1],
//      [ 0,-1, 0]]
// (nearest boundary on the replicated grid; non-zero taps summed in row-major
// order, starting from the first tap's product), negative values are clipped
// to zero, and the result is block-averaged back by 2 (the four values summed
// in row-major order, then multiplied by 1/4).
template <typename T>
void laplacian_edge(const T* C, int64_t h, int64_t w, T* L, int nt) {
  const int64_t H = 2 * h, W = 2 * w;
  std::vector<T> U(static_cast<size_t>(H * W));
  std::vector<T> lap(static_cast<size_t>(H * W));
  static const int kern[3][3] = {{0, -1, 0}, {-1, 4, -1}, {0, -1, 0}};

#pragma omp parallel for num_threads(nt) schedule(static)
  for (int64_t y = 0; y < H; ++y)
    for (int64_t x = 0; x < W; ++x) U[y * W + x] = C[(y / 2) * w + (x / 2)];

#pragma omp parallel for num_threads(nt) schedule(static)
  for (int64_t y = 0; y < H; ++y) {
    for (int64_t x = 0; x < W; ++x) {
      T acc = 0;
      bool first = true;
      for (int dy = -1; dy <= 1; ++dy) {
        for (int dx = -1; dx <= 1; ++dx) {
          const int kv = kern[dy + 1][dx + 1];
          if (kv == 0) continue;
          const int64_t yy = clampi(y + dy, 0, H - 1);
          const int64_t xx = clampi(x + dx, 0, W - 1);
          const T term = static_cast<T>(kv) * U[yy * W + xx];
          acc = first ? term : acc + term;
          first = false;
        }
      }
      lap[y * W + x] = (acc > static_cast<T>(0)) ? acc : static_cast<T>(0);
    }
  }

#pragma omp parallel for num_threads(nt) schedule(static)
  for (int64_t i = 0; i < h; ++i) {
    for (int64_t j = 0; j < w; ++j) {
      const T a = lap[(2 * i) * W + 2 * j];
      const T b = lap[(2 * i) * W + 2 * j + 1];
      const T c = lap[(2 * i + 1) * W + 2 * j];
      const T d = lap[(2 * i + 1) * W + 2 * j + 1];
      L[i * w + j] = (((a + b) + c) + d) * static_cast<T>(0.25);
    }
  }
}

// True (non-separable) k x k median with the nearest boundary: the median of
// the k*k values X[clamp(y+dy), clamp(x+dx)], duplicates made by clamping
// counted.  k*k is odd, so the median is the middle element of the sorted
// window.  The paper insists on this classic median rather than a separable
// approximation (Methods, "Algorithm"; State of the field).
template <typename T>
void median_filter(const T* X, int64_t h, int64_t w, int k, T* out, int nt) {
  const int r = k / 2;
#pragma omp parallel for num_threads(nt) schedule(static)
  for (int64_t y = 0; y < h; ++y) {
    std::vector<T> win(static_cast<size_t>(k * k));
    for (int64_t x = 0; x < w; ++x) {
      int n = 0;
      for (int dy = -r; dy <= r; ++dy)
        for (int dx = -r; dx <= r; ++dx)
          win[n++] = X[clampi(y + dy, 0, h - 1) * w + clampi(x + dx, 0, w - 1)];
      std::sort(win.begin(), win.end());
      out[y * w + x] = win[(k * k - 1) / 2];
    }
  }
}

// Separable approximation of the k x k median -- the "sepmed" option of the
// astroscrappy implementation the paper compares against (State of the
// field), kept as a speed and accuracy comparison point: the 1-D median of
// the k values along each row (clamped), then the 1-D median of k of those
// row medians along each column (clamped on the row medians' grid).  It is
// not the classic median the method calls for.
template <typename T>
void sep_median_filter(const T* X, int64_t h, int64_t w, int k, T* out, int nt) {
  const int r = k / 2;
  std::vector<T> R(static_cast<size_t>(h * w));
#pragma omp parallel for num_threads(nt) schedule(static)
  for (int64_t y = 0; y < h; ++y) {
    std::vector<T> win(static_cast<size_t>(k));
    for (int64_t x = 0; x < w; ++x) {
      for (int d = -r; d <= r; ++d) win[d + r] = X[y * w + clampi(x + d, 0, w - 1)];
      std::sort(win.begin(), win.end());
      R[y * w + x] = win[r];
    }
  }
#pragma omp parallel for num_threads(nt) schedule(static)
  for (int64_t y = 0; y < h; ++y) {
    std::vector<T> win(static_cast<size_t>(k));
    for (int64_t x = 0; x < w; ++x) {
      for (int d = -r; d <= r; ++d) win[d + r] = R[clampi(y + d, 0, h - 1) * w + x];
      std::sort(win.begin(), win.end());
      out[y * w + x] = win[r];
    }
  }
}

// The k x k median of the detection steps: the classic one, or with sep the
// separable approximation.
template <typename T>
void window_median(const T* X, int64_t h, int64_t w, int k, T* out, int nt, int sep) {
  if (sep)
    sep_median_filter(X, h, w, k, out, nt);
  else
    median_filter(X, h, w, k, out, nt);
}

// Step 2, "Create a noise model": N = sqrt(gain * med5 + readnoise^2) / gain,
// with med5 floored at 1e-4 so the square root never sees a negative value.
template <typename T>
void noise_model(const T* C, int64_t h, int64_t w, T gain, T readnoise, T* N, int nt,
                 int sep = 0) {
  std::vector<T> m5(static_cast<size_t>(h * w));
  window_median(C, h, w, 5, m5.data(), nt, sep);
  const T rn2 = readnoise * readnoise;
  const T floor = Consts<T>::noise_floor;
#pragma omp parallel for num_threads(nt) schedule(static)
  for (int64_t i = 0; i < h * w; ++i) {
    const T m = (m5[i] > floor) ? m5[i] : floor;
    const T var = gain * m + rn2;
    N[i] = std::sqrt(var) / gain;
  }
}

// 3x3 binary dilation; cells outside the frame count as unset.
void dilate3(const uint8_t* B, int64_t h, int64_t w, uint8_t* out, int nt) {
#pragma omp parallel for num_threads(nt) schedule(static)
  for (int64_t y = 0; y < h; ++y) {
    for (int64_t x = 0; x < w; ++x) {
      uint8_t v = 0;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          const int64_t yy = y + dy, xx = x + dx;
          if (yy < 0 || yy >= h || xx < 0 || xx >= w) continue;
          if (B[yy * w + xx]) v = 1;
        }
      out[y * w + x] = v;
    }
  }
}

// Step 7, "Replace cosmic rays with median of neighbors": for each masked
// pixel, the lower median of the un-masked values in its clamped 5 x 5 window
// (a cell is excluded by its mask bit, duplicates made by clamping counted).
// A pixel whose window holds no un-masked cell keeps its value.  All reads see
// the image before this step.  Returns the number of such kept pixels.
template <typename T>
int64_t masked_median5(const T* C, const uint8_t* M, int64_t h, int64_t w, T* out, int nt) {
  int64_t kept = 0;
#pragma omp parallel for num_threads(nt) schedule(static) reduction(+ : kept)
  for (int64_t y = 0; y < h; ++y) {
    std::vector<T> win;
    win.reserve(25);
    for (int64_t x = 0; x < w; ++x) {
      const int64_t p = y * w + x;
      if (!M[p]) {
        out[p] = C[p];
        continue;
      }
      win.clear();
      for (int dy = -2; dy <= 2; ++dy)
        for (int dx = -2; dx <= 2; ++dx) {
          const int64_t q = clampi(y + dy, 0, h - 1) * w + clampi(x + dx, 0, w - 1);
          if (!M[q]) win.push_back(C[q]);
        }
      if (win.empty()) {
        out[p] = C[p];
        ++kept;
        continue;
      }
      std::sort(win.begin(), win.end());
      out[p] = win[(win.size() - 1) / 2];
    }
  }
  return kept;
}

// ---------------------------------------------------------------- gain
// "If a gain is not supplied, then it will be estimated at each iteration"
// (Methods, "Main parameters"; Software design names a sigma-clipping
// routine among the package's functions).  The estimator itself is not given;
// the reading implemented here:
//   1. sigma-clip the current image: starting from every pixel, repeat up to
//      5 times -- centre = the lower median of the kept values, spread = their
//      standard deviation (population) -- and keep the values within 3 spreads
//      of the centre (|x - centre| <= 3 sd); stop early when a round keeps
//      every value;
//   2. mean m and variance v (population) of the kept values;
//   3. the gain g for which the noise model's variance of an ADU pixel,
//      m / g + readnoise^2 / g^2, equals v:  g = (m + sqrt(m^2 + 4 v rn^2)) / (2 v)
//      (with rn = 0 this is m / v, the photon-transfer estimate).
// Arithmetic in binary64 throughout; the sums are the exact sums of the
// pixel values (and of their squares), rounded once to binary64, so the
// result does not depend on any summation order.  A frame without spread
// (v <= 0) or a result that is not a positive normal binary32 number gives no
// estimate, and gain 1 is used instead.

// Correctly rounded binary64 sum of xs: Shewchuk's exact partials (the
// running sum is kept exactly as a list of non-overlapping binary64 values,
// each new term added with error-free two-sums), then the partials are
// summed from the largest down with a final half-even correction, as
// described for Python's math.fsum.  No term may be infinite or NaN and no
// partial may overflow (true for image values).
double exact_sum(const double* xs, int64_t n) {
  std::vector<double> part;
  for (int64_t k = 0; k < n; ++k) {
    double x = xs[k];
    size_t used = 0;
    for (size_t j = 0; j < part.size(); ++j) {
      double y = part[j];
      if (std::fabs(x) < std::fabs(y)) std::swap(x, y);
      const double hi = x + y;
      const double lo = y - (hi - x);
      if (lo != 0.0) part[used++] = lo;
      x = hi;
    }
    part.resize(used);
    part.push_back(x);
  }
  if (part.empty()) return 0.0;
  size_t i = part.size();
  double hi = part[--i];
  double lo = 0.0;
  while (i > 0) {
    const double x = hi;
    const double y = part[--i];
    hi = x + y;
    lo = y - (hi - x);
    if (lo != 0.0) break;
  }
  // the rest of the partials decides a tie in the rounding of hi + lo
  if (i > 0 && ((lo < 0.0 && part[i - 1] < 0.0) || (lo > 0.0 && part[i - 1] > 0.0))) {
    const double y = lo * 2.0;
    const double x = hi + y;
    if (y == x - hi) hi = x;
  }
  return hi;
}

struct GainEstimate {
  double gain;      // the estimate (binary64), or 1 when there is none
  int valid;        // 0: no estimate, gain 1 used
  int rounds;       // clipping rounds applied
  int64_t kept;     // values kept after clipping
  double mean, var; // of the kept values
};

constexpr int kClipRounds = 5;
constexpr double kClipSigma = 3.0;

// The estimate from the n values of img (the current image, canonical).
template <typename T>
GainEstimate estimate_gain(const T* img, int64_t n, double readnoise) {
  std::vector<double> cur(static_cast<size_t>(n)), tmp, sq;
  for (int64_t i = 0; i < n; ++i) cur[i] = static_cast<double>(img[i]);
  GainEstimate r{};
  int64_t prev = -1;
  double mean = 0.0, var = 0.0;
  for (int round = 0;; ++round) {
    const int64_t m = static_cast<int64_t>(cur.size());
    sq.resize(cur.size());
    // the square of a binary32 value is exact in binary64 (48 significant
    // bits); the binary64 oracle rounds each square once
    for (size_t i = 0; i < cur.size(); ++i) sq[i] = cur[i] * cur[i];
    const double s1 = exact_sum(cur.data(), m);
    const double s2 = exact_sum(sq.data(), m);
    mean = s1 / static_cast<double>(m);
    var = s2 / static_cast<double>(m) - mean * mean;
    r.rounds = round;
    if (m == prev || round == kClipRounds) break;  // nothing clipped, or rounds used up
    tmp = cur;
    std::sort(tmp.begin(), tmp.end());
    const double centre = tmp[static_cast<size_t>((m - 1) / 2)];  // lower median
    const double sd = var > 0.0 ? std::sqrt(var) : 0.0;
    const double lim = kClipSigma * sd;
    tmp.clear();
    for (double x : cur)
      if (std::fabs(x - centre) <= lim) tmp.push_back(x);
    prev = m;
    cur.swap(tmp);
  }
  r.kept = static_cast<int64_t>(cur.size());
  r.mean = mean;
  r.var = var;
  r.valid = 0;
  r.gain = 1.0;
  if (var > 0.0) {
    const double rn2 = readnoise * readnoise;
    const double g = (mean + std::sqrt(mean * mean + 4.0 * var * rn2)) / (2.0 * var);
    const float gf = static_cast<float>(g);
    if (std::isfinite(g) && std::isnormal(gf) && gf > 0.0f) {
      r.gain = g;
      r.valid = 1;
    }
  }
  return r;
}

// The gain an iteration uses: the binary32 rounding of the estimate for the
// binary32 oracle, the estimate itself for the binary64 one.
inline float gain_of(const GainEstimate& e, float*) { return static_cast<float>(e.gain); }
inline double gain_of(const GainEstimate& e, double*) { return e.gain; }

struct Params64 {
  double gain, readnoise, sigclip, sigfrac, objlim;
};

// One full run of the method.  Each iteration: steps 1-7 on the current
// image, the mask accumulated over iterations, detection on the cleaned image
// of the previous iteration.  With early_stop, the loop ends after the first
// iteration that adds no new mask pixel (further iterations would repeat it
// exactly).
template <typename T>
int run(const T* img, int64_t h, int64_t w, T gain, T readnoise, T sigclip, T sigfrac,
        T objlim, int niter, int early_stop, int estimate, int sepmed, int nt, uint8_t* out_mask,
        T* out_clean, T* trace_s, T* trace_sp, uint8_t* trace_b1, uint8_t* trace_mask,
        T* trace_clean, int64_t* n_new_out, int* iters_run, int64_t* n_unreplaced,
        double* gains_out) {
  if (h < 1 || w < 1 || niter < 1) return -1;
  const int64_t n = h * w;
  std::vector<T> C(static_cast<size_t>(n)), Cn(static_cast<size_t>(n));
  std::vector<T> L(static_cast<size_t>(n)), N(static_cast<size_t>(n)), S(static_cast<size_t>(n)),
      mS(static_cast<size_t>(n)), Sp(static_cast<size_t>(n)), m3(static_cast<size_t>(n)),
      m7(static_cast<size_t>(n));
  std::vector<uint8_t> B1(static_cast<size_t>(n)), D(static_cast<size_t>(n)),
      B2(static_cast<size_t>(n)), B3(static_cast<size_t>(n)), M(static_cast<size_t>(n), 0);

  // Ingest: -0 becomes +0 (x + 0 is +0 for x = -0 and x otherwise).
  for (int64_t i = 0; i < n; ++i) C[i] = img[i] + static_cast<T>(0);

  const T lo = sigfrac * sigclip;
  const T ffloor = Consts<T>::fine_floor;
  int done = 0;
  int64_t kept = 0;
  for (int k = 0; k < niter; ++k) {
    // Without a supplied gain, this iteration's gain is estimated from the
    // current image.
    if (estimate) {
      const GainEstimate e = estimate_gain(C.data(), n, static_cast<double>(readnoise));
      gain = gain_of(e, static_cast<T*>(nullptr));
    }
    if (gains_out) gains_out[k] = static_cast<double>(gain);
    // Step 1: Laplacian edge image.
    laplacian_edge(C.data(), h, w, L.data(), nt);
    // Step 2: noise model.
    noise_model(C.data(), h, w, gain, readnoise, N.data(), nt, sepmed);
    // Step 3: significance, S = L / (2 N) (2 = the subsampling factor), and
    // removal of large-scale structure, S' = S - med5(S).
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int64_t i = 0; i < n; ++i) S[i] = L[i] / (static_cast<T>(2) * N[i]);
    window_median(S.data(), h, w, 5, mS.data(), nt, sepmed);
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int64_t i = 0; i < n; ++i) Sp[i] = S[i] - mS[i];
    // Step 5 (inputs): fine-structure image F = med3 - med7(med3), divided by
    // the noise and floored at 0.01.
    window_median(C.data(), h, w, 3, m3.data(), nt, sepmed);
    window_median(m3.data(), h, w, 7, m7.data(), nt, sepmed);
    // Steps 4 and 5: candidates above sigclip whose ratio S' / F exceeds objlim.
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
      const T F = m3[i] - m7[i];
      const T f = F / N[i];
      const T fn = (f > ffloor) ? f : ffloor;
      B1[i] = (Sp[i] > sigclip) && ((Sp[i] / fn) > objlim);
    }
    // Step 6: two rounds of 3x3 growth, the first kept where S' > sigclip, the
    // second where S' > sigfrac * sigclip.
    dilate3(B1.data(), h, w, D.data(), nt);
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int64_t i = 0; i < n; ++i) B2[i] = D[i] && (Sp[i] > sigclip);
    dilate3(B2.data(), h, w, D.data(), nt);
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int64_t i = 0; i < n; ++i) B3[i] = D[i] && (Sp[i] > lo);
    // Accumulate the mask and count the new pixels.
    int64_t fresh = 0;
#pragma omp parallel for num_threads(nt) schedule(static) reduction(+ : fresh)
    for (int64_t i = 0; i < n; ++i) {
      if (B3[i] && !M[i]) ++fresh;
      M[i] = static_cast<uint8_t>(M[i] | B3[i]);
    }
    // Step 7: replace masked pixels.
    kept = masked_median5(C.data(), M.data(), h, w, Cn.data(), nt);
    C.swap(Cn);

    if (n_new_out) n_new_out[k] = fresh;
    if (trace_s) std::memcpy(trace_s + k * n, S.data(), sizeof(T) * n);
    if (trace_sp) std::memcpy(trace_sp + k * n, Sp.data(), sizeof(T) * n);
    if (trace_b1) std::memcpy(trace_b1 + k * n, B1.data(), n);
    if (trace_mask) std::memcpy(trace_mask + k * n, M.data(), n);
    if (trace_clean) std::memcpy(trace_clean + k * n, C.data(), sizeof(T) * n);
    done = k + 1;
    if (early_stop && fresh == 0) break;
  }
  if (out_mask) std::memcpy(out_mask, M.data(), n);
  if (out_clean) std::memcpy(out_clean, C.data(), sizeof(T) * n);
  if (iters_run) *iters_run = done;
  if (n_unreplaced) *n_unreplaced = kept;
  return 0;
}

int threads_or_default(int nt) {
#ifdef _OPENMP
  return nt > 0 ? nt : omp_get_max_threads();
#else
  (void)nt;
  return 1;
#endif
}

}  // namespace

extern "C" {

int oracle_max_threads(void) { return threads_or_default(0); }

int oracle_lacosmic_f32(const float* img, int64_t h, int64_t w, float gain, float readnoise,
                        float sigclip, float sigfrac, float objlim, int niter, int early_stop,
                        int estimate_gain, int sepmed, int nthreads, uint8_t* out_mask,
                        float* out_clean,
                        float* trace_s, float* trace_sp, uint8_t* trace_b1, uint8_t* trace_mask,
                        float* trace_clean, int64_t* n_new, int* iters_run,
                        int64_t* n_unreplaced, double* gains) {
  return run<float>(img, h, w, gain, readnoise, sigclip, sigfrac, objlim, niter, early_stop,
                    estimate_gain, sepmed, threads_or_default(nthreads), out_mask, out_clean, trace_s,
                    trace_sp, trace_b1, trace_mask, trace_clean, n_new, iters_run, n_unreplaced,
                    gains);
}

int oracle_lacosmic_f64(const double* img, int64_t h, int64_t w, double gain, double readnoise,
                        double sigclip, double sigfrac, double objlim, int niter, int early_stop,
                        int estimate_gain, int sepmed, int nthreads, uint8_t* out_mask,
                        double* out_clean,
                        double* trace_s, double* trace_sp, uint8_t* trace_b1, uint8_t* trace_mask,
                        double* trace_clean, int64_t* n_new, int* iters_run,
                        int64_t* n_unreplaced, double* gains) {
  return run<double>(img, h, w, gain, readnoise, sigclip, sigfrac, objlim, niter, early_stop,
                     estimate_gain, sepmed, threads_or_default(nthreads), out_mask, out_clean, trace_s,
                     trace_sp, trace_b1, trace_mask, trace_clean, n_new, iters_run, n_unreplaced,
                     gains);
}

double oracle_exact_sum(const double* xs, int64_t n) { return exact_sum(xs, n); }

// The gain estimate of a float32 image: the estimate (1 when there is none),
// validity, clipping rounds, kept values, their mean and variance.
int oracle_estimate_gain_f32(const float* img, int64_t n, float readnoise, double* gain,
                             int* rounds, int64_t* kept, double* mean, double* var) {
  const GainEstimate e = estimate_gain(img, n, static_cast<double>(readnoise));
  *gain = e.gain;
  *rounds = e.rounds;
  *kept = e.kept;
  *mean = e.mean;
  *var = e.var;
  return e.valid;
}

void oracle_laplacian_f32(const float* C, int64_t h, int64_t w, float* L) {
  laplacian_edge(C, h, w, L, 1);
}
void oracle_laplacian_f64(const double* C, int64_t h, int64_t w, double* L) {
  laplacian_edge(C, h, w, L, 1);
}
void oracle_median_f32(const float* X, int64_t h, int64_t w, int k, float* out) {
  median_filter(X, h, w, k, out, 1);
}
void oracle_median_f64(const double* X, int64_t h, int64_t w, int k, double* out) {
  median_filter(X, h, w, k, out, 1);
}
void oracle_sep_median_f32(const float* X, int64_t h, int64_t w, int k, float* out) {
  sep_median_filter(X, h, w, k, out, 1);
}
void oracle_noise_f32(const float* C, int64_t h, int64_t w, float gain, float readnoise,
                      float* N) {
  noise_model(C, h, w, gain, readnoise, N, 1);
}
void oracle_dilate3(const uint8_t* B, int64_t h, int64_t w, uint8_t* out) {
  dilate3(B, h, w, out, 1);
}
int64_t oracle_masked_median5_f32(const float* C, const uint8_t* M, int64_t h, int64_t w,
                                  float* out) {
  return masked_median5(C, M, h, w, out, 1);
}
int64_t oracle_masked_median5_f64(const double* C, const uint8_t* M, int64_t h, int64_t w,
                                  double* out) {
  return masked_median5(C, M, h, w, out, 1);
}

}  // extern "C"
