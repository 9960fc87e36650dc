/*
 * lacosmic.h -- C ABI of liblacosmic.so, an MI355X (gfx950) implementation of
 * the L.A.Cosmic cosmic-ray detection and removal iteration.
 *
 * The method is the one the dfcosmic paper ports (arXiv 2602.17938, Methods:
 * "Algorithm", steps 1-7, and "Main parameters"):
 *   1. Laplacian edge image of the 2x block-replicated frame (3x3 Laplacian,
 *      negatives clipped, 2x2 block average);
 *   2. noise model N = sqrt(gain * med5(C) + readnoise^2) / gain;
 *   3. significance S = L / (2 N) and S' = S - med5(S);
 *   4. candidates S' > sigclip;
 *   5. rejection of compact objects: S' / max((med3 - med7(med3)) / N, 0.01)
 *      must exceed objlim;
 *   6. growth by two 3x3 dilations, kept where S' > sigclip, then where
 *      S' > sigfrac * sigclip;
 *   7. replacement of flagged pixels by the lower median of the un-flagged
 *      values of their 5x5 neighbourhood;
 * repeated niter times on the cleaned frame with a cumulative mask.  Every
 * window clamps to the frame ("nearest" boundary); every median is a true 2-D
 * median.  Arithmetic is IEEE binary32, round-to-nearest-even, without
 * contraction, in the expression order documented with the implementation, so
 * results are bit-identical to a plain CPU evaluation of the same steps.
 *
 * Conventions for every entry point:
 *  - Image, mask and clean pointers are DEVICE pointers (HIP / torch.cuda
 *    memory on the current device), row-major, contiguous, row pitch = w.
 *  - The caller owns every buffer it passes.  The library owns only its
 *    cached per-device workspace and stream, released by lacosmic_shutdown().
 *  - img is never written.  out_mask receives 0/1 bytes, out_clean floats.
 *  - Return value: LACOSMIC_OK (0) or a negative lacosmic_status.  Argument
 *    checks (EINVAL, EALIAS) happen before any HIP call.  On error the output
 *    buffers are unspecified.  There is no global error state.
 *  - Calls are thread-safe (one mutex-guarded context per device).
 */
#ifndef LACOSMIC_H
#define LACOSMIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LACOSMIC_OK = 0,
  LACOSMIC_EINVAL = -1,     /* null pointer, h or w < 1, h or w > 2^24,
                               h * w > 2^31 - 1, niter < 1 or > 1024, gain <= 0 or
                               non-finite, readnoise < 0, sigclip <= 0,
                               sigfrac <= 0, objlim < 0, non-finite parameter,
                               workspace not 256-byte aligned, server input
                               on another device, bad server handle/ticket */
  LACOSMIC_ENOMEM = -2,     /* device or host allocation failed */
  LACOSMIC_EHIP = -3,       /* a HIP runtime call failed */
  LACOSMIC_ENONFINITE = -4, /* the input image holds NaN or Inf */
  LACOSMIC_EALIAS = -5,     /* an output buffer overlaps the input or the other output */
  LACOSMIC_EBUDGET = -6,    /* a server frame can never fit the HBM budget */
  LACOSMIC_ESCRATCH = -7    /* lacosmic_run_noalloc: the frame needs more than the
                               static scratch buffer */
} lacosmic_status;

/* Method parameters ("Main parameters" of the paper, plus the iteration
 * count).  gain in e-/ADU, readnoise in e-, the image in ADU. */
typedef struct {
  float gain;
  float readnoise;
  float sigclip;  /* detection limit for cosmic rays, in units of N */
  float sigfrac;  /* fractional detection limit for neighbouring pixels */
  float objlim;   /* contrast limit between cosmic rays and underlying objects */
  int32_t niter;
  uint32_t flags; /* LACOSMIC_F_* */
} lacosmic_params;

/* Stop after the first iteration that adds no new mask pixel.  Exact: the
 * remaining iterations would repeat it bit for bit. */
#define LACOSMIC_F_EARLY_STOP 1u
/* Compute S' = S - med5(S) at every pixel and keep the whole S' plane in the
 * workspace (for inspection).  Without it S' is evaluated only where it can
 * decide a threshold: at the pixels with S > sigclip (S' <= S), and, for the
 * sigfrac * sigclip test of the growth, within 2 pixels of the confirmed
 * candidates, the only pixels the growth can reach; the plane then holds S'
 * at the pixels with S > sigclip.  Masks and cleaned images are identical
 * either way.  The batched and serving paths, which keep no caller-visible
 * workspace, ignore the flag. */
#define LACOSMIC_F_FULL_SP 2u
/* The input is uint16 ADU (CMOS frames, Statement of need): img points to
 * h*w uint16 values (pass it cast to const float*), which the first pass
 * widens exactly to binary32 as it stages them.  Per frame in
 * lacosmic_run_batch; the server takes is_u16 instead. */
#define LACOSMIC_F_INPUT_U16 4u
/* No gain is supplied: it is estimated at the start of each iteration from
 * the current image (Methods, "Main parameters"), and the gain field is
 * ignored (it must be finite and >= 0).  The estimate, all in binary64:
 * sigma clipping -- up to 5 rounds keeping the values within 3 standard
 * deviations (population) of the lower median of the values kept so far,
 * ending early after a round that keeps every value -- then the mean m and
 * variance v of the kept values, and the gain g that makes the noise model's
 * variance of a pixel in ADU, m / g + readnoise^2 / g^2, equal v:
 * g = (m + sqrt(m^2 + 4 v readnoise^2)) / (2 v), rounded to binary32.  The
 * sums are exact (rounded once), so the estimate does not depend on
 * summation order.  A frame without spread (v <= 0), or a result that is not
 * a positive normal binary32 number, uses gain 1 for that iteration.  Every
 * iteration of such a frame recomputes S at every pixel. */
#define LACOSMIC_F_ESTIMATE_GAIN 8u
/* Separable detection medians, the speed and accuracy comparison point the
 * paper discusses (State of the field: astroscrappy's sepmed option; the
 * method itself uses the classic median): every median of steps 2-5 -- the
 * noise model's 5x5, S' = S - med5(S), the fine structure's 3x3 and 7x7 --
 * becomes the median along each row of the window followed by the median of
 * those row medians (on clamped windows: a row pass, then a column pass,
 * each clamped on its own grid).  The replacement keeps the true median.
 * Per frame in lacosmic_run_batch. */
#define LACOSMIC_F_SEPMED 16u

typedef struct {
  int32_t iters_run;     /* iterations executed (< niter only with early stop) */
  int64_t n_flagged;     /* mask pixels after the run */
  int64_t n_unreplaced;  /* mask pixels whose clamped 5x5 window holds no
                            un-flagged cell under the final mask: step 7 has
                            no value to replace them with, so they keep their
                            value (Methods, "Algorithm", step 7) */
  int64_t n_new[16];     /* new mask pixels found by iteration k (k < 16) */
  float gain[16];        /* gain iteration k used (k < 16): the supplied one, or the
                            estimate with LACOSMIC_F_ESTIMATE_GAIN (0: not run) */
  int8_t gain_estimated[16]; /* with LACOSMIC_F_ESTIMATE_GAIN: 1 = estimated,
                                -1 = no estimate (gain 1 used), 0 = not run */
} lacosmic_stats;

/* One frame, synchronous, early stop on.  gain, readnoise, sigclip, sigfrac,
 * objlim as in lacosmic_params.  out_mask: h*w bytes; out_clean: h*w floats. */
int lacosmic_run(const float* img, int64_t h, int64_t w, float gain, float readnoise,
                 float sigclip, float sigfrac, float objlim, int32_t niter, uint8_t* out_mask,
                 float* out_clean);

/* One frame with explicit parameters, flags, workspace and stream.
 *  workspace: NULL = the library's cached workspace; otherwise a device
 *    buffer of at least lacosmic_workspace_bytes(h, w) bytes, 256-byte
 *    aligned (LACOSMIC_EINVAL otherwise), owned by the caller and not used
 *    concurrently by another call.  The library cannot check its size: a
 *    smaller buffer is overrun.
 *  hip_stream: NULL = the library's stream, ordered after the work already
 *    enqueued on the legacy null stream (the default stream of a caller that
 *    uses no other), and the call is synchronous; otherwise a hipStream_t
 *    and the call only enqueues (asynchronous) unless st is non-NULL.
 *  st: if non-NULL the call waits for the work, checks the input for NaN/Inf
 *    (LACOSMIC_ENONFINITE) and fills the statistics.  An asynchronous call
 *    (non-NULL stream, NULL st) cannot report LACOSMIC_ENONFINITE: the
 *    outputs of a non-finite input are then unspecified. */
int lacosmic_run_ex(const float* img, int64_t h, int64_t w, const lacosmic_params* p,
                    uint8_t* out_mask, float* out_clean, void* workspace, void* hip_stream,
                    lacosmic_stats* st);

/* For callers that cannot allocate -- code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation: lacosmic_run_ex with the
 * cached workspace replaced by a static device array of 128 MiB inside the
 * library (each device holds its own copy from the moment the library's code
 * is loaded on it until the process ends).  The call allocates nothing: no
 * device memory, no pinned memory, no library context or recorded graph; it
 * launches the single-frame kernels eagerly on hip_stream (NULL = the legacy
 * null stream) and, when hip_stream is NULL or st is non-NULL, waits and
 * fills st as lacosmic_run_ex does (reading back through the calling
 * thread's stack).  The first call on a device resolves the array's address
 * there.  Frames whose workspace (lacosmic_workspace_bytes) exceeds 128 MiB
 * -- about 7.8 Mpx, e.g. larger than 2048 x 3800 -- are rejected with
 * LACOSMIC_ESCRATCH before any HIP call.  Every call on a device uses that
 * device's one array and leaves its contents behind; the kernels clear what
 * must start at zero, so calls in sequence are independent, but calls that
 * overlap on one device (another thread, or another stream without ordering
 * between them) race and their results are undefined.  Arguments, flags and
 * results otherwise as lacosmic_run_ex; results are bit-identical to it. */
int lacosmic_run_noalloc(const float* img, int64_t h, int64_t w, const lacosmic_params* p,
                         uint8_t* out_mask, float* out_clean, void* hip_stream,
                         lacosmic_stats* st);

/* Device workspace a frame of h x w needs (0 for sizes lacosmic_run_ex
 * rejects). */
size_t lacosmic_workspace_bytes(int64_t h, int64_t w);

/* Byte offsets inside a caller-provided workspace of the planes the last
 * iteration run leaves behind, for inspection and testing:
 *  s_offset:    S = L / (2N), float, h*w, every pixel;
 *  sp_offset:   S' = S - med5(S), float, h*w: every pixel with
 *               LACOSMIC_F_FULL_SP, else the pixels with S > sigclip only;
 *  cand_offset: the candidate map of steps 4-5 as a bit plane: row y holds
 *               row_words 64-bit words, bit i of word j is pixel (y, 64j + i).
 *  mask_bits_offset: the cumulative mask after the first iteration, as a bit
 *               plane of the same layout. */
typedef struct {
  size_t s_offset;
  size_t sp_offset;
  size_t cand_offset;
  size_t mask_bits_offset;
  size_t row_words;
  size_t total_bytes;
} lacosmic_ws_layout;
int lacosmic_workspace_layout(int64_t h, int64_t w, lacosmic_ws_layout* out);

/* Many frames of different sizes, one launch per pass over the tiles of all
 * frames of a group (a persistent launch pulling tiles from a shared queue, or
 * one block per tile); the frames are split into groups of about equal pixel
 * counts whose chains of launches run concurrently.  Tile shape, launch form
 * and group count are the fastest on the first call for the batch shape; the
 * niter loop is recorded once per batch shape as a HIP graph and replayed.  imgs, hs, ws, out_masks, out_cleans are HOST arrays of n
 * entries (the pointers they hold are device pointers); p holds n parameter
 * sets (gain and readnoise may differ per frame; niter and flags are taken
 * from p[0] and must agree).  Results are bit-identical to lacosmic_run_ex on
 * each frame alone.  hip_stream as in lacosmic_run_ex (NULL = synchronous). */
int lacosmic_run_batch(int32_t n, const float* const* imgs, const int64_t* hs, const int64_t* ws,
                       const lacosmic_params* p, uint8_t* const* out_masks,
                       float* const* out_cleans, void* hip_stream);

/* Index of the tile shape (see lacosmic_get_tile_shape) the batched path
 * chose, by timing, for the most recent batch shape on the current device;
 * -1 before the first batch.  LACOSMIC_AUTOTUNE=0 disables the timing. */
int lacosmic_batch_tile_shape(void);
/* Launch form the batched path chose with it: 0 = one persistent launch per
 * pass pulling tiles from a queue, 1 = one block per tile; -1 before the
 * first batch. */
int lacosmic_batch_launch_mode(void);
/* Number of frame groups (concurrent chains of launches) the batched path
 * chose with it; -1 before the first batch.  LACOSMIC_BATCH_GROUPS (1 .. 8)
 * pins it. */
int lacosmic_batch_groups(void);

/* Durations in milliseconds of the kernel passes of the most recent batch
 * shape run by lacosmic_run_batch on the current device -- for each
 * iteration, 9 values in launch order: GAIN (the gain estimate of frames
 * without a supplied gain), US (S updated near the pixels the previous
 * iteration rewrote; iterations >= 1), A1 (steps 1-3a at every pixel:
 * Laplacian edge image, noise model, S; iteration 0, and every iteration of
 * frames without a supplied gain), SC (candidate list), S1 (S', thresholds
 * and the objlim test at the candidates), SG (the sigfrac threshold around
 * confirmed candidates), B (growth and mask), S2 (replacement), OUT (mask
 * bytes; last iteration); a pass the iteration does not launch reads 0.  The
 * call replays that batch's kernels once, eagerly (same kernels and grids as
 * the recorded graph, same buffers, identical outputs), on hip_stream (NULL =
 * the library stream) with events between the passes, the frame groups one
 * after another (each value is summed over the groups, so the values add up
 * to more than a concurrent graph run), and waits for it.  Writes at most n
 * values and returns how many it wrote (0 before the first batch), or a
 * negative status. */
int lacosmic_batch_pass_ms(float* ms, int32_t n, void* hip_stream);

/* Continuous-batching server.  A host thread admits submitted frames while
 * their device state fits hbm_budget_bytes and fewer than max_frames are in
 * flight, and advances every admitted frame by one iteration per step (frames
 * at different iterations share each step's launches).  Results are
 * bit-identical to lacosmic_run_ex on each frame alone.  Inputs and results
 * are staged in a pinned host pool the server allocates (a quarter of the
 * budget, 256 MiB to 8 GiB; LACOSMIC_SERVER_PINNED_MB overrides, 0 disables)
 * and in pageable host memory when the pool is full. */
typedef struct lacosmic_server lacosmic_server;
int lacosmic_server_create(uint64_t hbm_budget_bytes, int32_t max_frames, lacosmic_server** out);
/* Queue one frame.  img holds h*w float32 values, or uint16 ADU if is_u16
 * (converted exactly to float32 on the device), in HOST or DEVICE memory (the
 * library tells them apart by the pointer's attributes).  Host memory is
 * copied before return.  Device memory, on the server's device, is read in
 * place when the frame is admitted: it must stay valid and unchanged until
 * lacosmic_server_poll has returned 1 or an error for the ticket.  ticket
 * receives the request id.  Non-blocking. */
int lacosmic_server_submit(lacosmic_server* s, const void* img, int is_u16, int64_t h, int64_t w,
                           const lacosmic_params* p, uint64_t* ticket);
/* 1 = done (results copied to the HOST buffers out_mask / out_clean, which may
 * be NULL to skip, and the ticket released), 0 = pending, <0 = error: the
 * frame's own (LACOSMIC_ENONFINITE, the ticket is released), or, for a frame
 * still pending, the error that stopped the server (a runtime failure; the
 * frame will never finish).
 * t_submit_ns / t_done_ns (may be NULL) receive steady-clock timestamps of
 * submission and of completion of the result's device-to-host copy. */
int lacosmic_server_poll(lacosmic_server* s, uint64_t ticket, uint8_t* out_mask, float* out_clean,
                         double* t_submit_ns, double* t_done_ns);
/* Wait until every submitted frame is done. */
int lacosmic_server_drain(lacosmic_server* s);
int lacosmic_server_destroy(lacosmic_server* s);

/* Tile shapes compiled into the library, indexed 0..k-1: *th x *tw output
 * pixels per tile.  Returns LACOSMIC_EINVAL past the last one.  Results never
 * depend on the tile shape; only speed does. */
int lacosmic_get_tile_shape(int32_t cfg, int32_t* th, int32_t* tw);
/* Select the tile shape of the single-frame path on the current device (the
 * autotuner's hook; the LACOSMIC_TILE_CFG environment variable sets the
 * initial choice). */
int lacosmic_set_tile_shape(int32_t cfg);

/* Single-frame runs of frames of at most 2^19 pixels (LACOSMIC_FUSED_MAX_PX,
 * read at each call, overrides; 0 turns it off) without LACOSMIC_F_FULL_SP
 * run each iteration as one launch over 32 x 32 output tiles, every step of
 * the iteration computed from a 48 x 48 region of the previous image and
 * mask in LDS (one iteration reads them within 8 pixels); larger frames run
 * the sparse passes.  Results are identical either way; the fused launch is
 * faster where launch latency dominates (a 512 x 512 frame). */

/* Whether lacosmic_run_ex and lacosmic_run replay recorded graphs (1;
 * LACOSMIC_FRAME_GRAPH=1 sets 1 initially) or launch every kernel eagerly
 * (0, the default) on the current device.  A graph is recorded once per
 * workspace address, frame shape, tile shape, iteration count and full-S'
 * choice (the kernels read the frame's buffers and parameters from a record
 * the call stores in the workspace, so one graph serves every call of that
 * key; at most 8 are kept per device) and replays the counter reset and every
 * launch of the run.  Results are identical either way.  On MI355X the eager
 * launches take less time per run (512 x 512: 0.148 against 0.159 ms per
 * isolated call, 4096 x 4096: 0.456 against 0.465 ms); the graph saves the
 * host the launches, for callers whose thread is the limit. */
int lacosmic_set_frame_graphs(int32_t on);

/* Self-check of the square root the noise model uses when a frame's noise
 * variance cannot fall below 2^-96 (the case for any gain >= 2^-82, and with
 * read noise >= 2^-48 for any gain): the correctly rounded binary32 root
 * without the compiler's rescaling of smaller arguments.  Compares it, bit
 * for bit, with the compiler's sqrtf on every binary32 value whose bit
 * pattern lies in [lo_bits, hi_bits] (which must stay within [2^-96, +inf],
 * i.e. 0x0f800000 .. 0x7f800000) on the current device, synchronously, and
 * stores the number of differing inputs in *mismatches.  LACOSMIC_EINVAL for
 * a range outside that interval or a NULL pointer, LACOSMIC_EHIP on a
 * runtime error. */
int lacosmic_check_sqrt(uint32_t lo_bits, uint32_t hi_bits, uint64_t* mismatches);

/* Static description of a status code. */
const char* lacosmic_strerror(int status);

/* Release the cached workspaces, graphs and streams of every device. */
void lacosmic_shutdown(void);

#ifdef __cplusplus
}
#endif

#endif /* LACOSMIC_H */
