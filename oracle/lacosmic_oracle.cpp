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

// Step 2, "Create a noise model": N = sqrt(gain * med5 + readnoise^2) / gain,
// with med5 floored at 1e-4 so the square root never sees a negative value.
template <typename T>
void noise_model(const T* C, int64_t h, int64_t w, T gain, T readnoise, T* N, int nt) {
  std::vector<T> m5(static_cast<size_t>(h * w));
  median_filter(C, h, w, 5, m5.data(), nt);
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
        T objlim, int niter, int early_stop, int nt, uint8_t* out_mask, T* out_clean,
        T* trace_s, T* trace_sp, uint8_t* trace_b1, uint8_t* trace_mask, T* trace_clean,
        int64_t* n_new_out, int* iters_run, int64_t* n_unreplaced) {
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
    // Step 1: Laplacian edge image.
    laplacian_edge(C.data(), h, w, L.data(), nt);
    // Step 2: noise model.
    noise_model(C.data(), h, w, gain, readnoise, N.data(), nt);
    // Step 3: significance, S = L / (2 N) (2 = the subsampling factor), and
    // removal of large-scale structure, S' = S - med5(S).
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int64_t i = 0; i < n; ++i) S[i] = L[i] / (static_cast<T>(2) * N[i]);
    median_filter(S.data(), h, w, 5, mS.data(), nt);
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int64_t i = 0; i < n; ++i) Sp[i] = S[i] - mS[i];
    // Step 5 (inputs): fine-structure image F = med3 - med7(med3), divided by
    // the noise and floored at 0.01.
    median_filter(C.data(), h, w, 3, m3.data(), nt);
    median_filter(m3.data(), h, w, 7, m7.data(), nt);
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
                        int nthreads, uint8_t* out_mask, float* out_clean, float* trace_s,
                        float* trace_sp,
                        uint8_t* trace_b1, uint8_t* trace_mask, float* trace_clean,
                        int64_t* n_new, int* iters_run, int64_t* n_unreplaced) {
  return run<float>(img, h, w, gain, readnoise, sigclip, sigfrac, objlim, niter, early_stop,
                    threads_or_default(nthreads), out_mask, out_clean, trace_s, trace_sp, trace_b1,
                    trace_mask, trace_clean, n_new, iters_run, n_unreplaced);
}

int oracle_lacosmic_f64(const double* img, int64_t h, int64_t w, double gain, double readnoise,
                        double sigclip, double sigfrac, double objlim, int niter, int early_stop,
                        int nthreads, uint8_t* out_mask, double* out_clean, double* trace_s,
                        double* trace_sp,
                        uint8_t* trace_b1, uint8_t* trace_mask, double* trace_clean,
                        int64_t* n_new, int* iters_run, int64_t* n_unreplaced) {
  return run<double>(img, h, w, gain, readnoise, sigclip, sigfrac, objlim, niter, early_stop,
                     threads_or_default(nthreads), out_mask, out_clean, trace_s, trace_sp, trace_b1,
                     trace_mask, trace_clean, n_new, iters_run, n_unreplaced);
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
