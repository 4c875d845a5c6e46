/*
 * rpca.h - C ABI of the MI355X RPCA library (librpca_mi355x.so).
 *
 * The library decomposes a Casorati matrix M (pixels x frames) into a
 * low-rank part L and a sparse part S by the inexact augmented-Lagrangian
 * (ADMM) iteration of principal component pursuit:
 *
 *   minimise ||L||_* + lambda ||S||_1  subject to  L + S = M      (paper Eq. 2)
 *
 *   repeat  L = D_{1/mu}(M - S + Y/mu)       singular value thresholding (Eq. 4)
 *           S = shrink_{lambda/mu}(M - L + Y/mu)                         (Eq. 5)
 *           Y = Y + mu (M - L - S)                                       (Eq. 6)
 *   until   ||M - L - S||_F < tol ||M||_F        (Sec. II-A, after Eq. 6)
 *
 * with S and Y starting at zero and mu fixed.  The singular value
 * thresholding is computed through the n x n Gram matrix A^T A of
 * A = M - S + Y/mu and its FP64 eigendecomposition on the GPU; the result is
 * the same operator D_tau(A) (a spectral function of A).
 *
 * Layout of every matrix argument: m x n, column-major, leading dimension m.
 * Element (p, t) - pixel p, frame t - is at offset p + t*m, so frame t is
 * contiguous (each frame is one column of the Casorati matrix, Sec. II-A).
 * A C-contiguous (n_frames, H, W) image stack is exactly this layout with
 * m = H*W.
 *
 * Memory: M, L and S are DEVICE pointers allocated by the caller on the
 * current HIP device.  M is read only.  L and S are fully overwritten and
 * must not overlap M or each other.  The library allocates and owns its
 * workspace (stream-ordered, from a cached pool; see rpca_footprint_bytes).
 *
 * Streams: `stream` is a hipStream_t (NULL = the null stream).  All work is
 * enqueued on it; the calls return after the work has completed and write
 * their host-side outputs then.
 *
 * Threads: calls are thread-safe; calls on different streams run
 * independently.
 */
#ifndef RPCA_MI355X_H
#define RPCA_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define RPCA_OK                 0  /* converged: ||M-L-S||_F < tol ||M||_F   */
#define RPCA_NOT_CONVERGED      1  /* ran maxit iterations; L, S valid       */
#define RPCA_ERR_ARG           -1  /* invalid argument; nothing was run      */
#define RPCA_ERR_NOMEM         -2  /* device allocation failed               */
#define RPCA_ERR_DEVICE        -3  /* HIP runtime error                      */
#define RPCA_ERR_NONFINITE     -4  /* NaN or Inf in M (or in the iteration)  */
#define RPCA_ERR_UNSUPPORTED   -5  /* shape not supported by the library     */
#define RPCA_ERR_TIMEOUT       -6  /* server: the request's timeout passed   */
/* Negative codes leave L and S unspecified. */

/* ---- element types and contraction modes -------------------------------- */
#define RPCA_F64 0   /* double storage, FP64 arithmetic throughout             */
#define RPCA_F32 1   /* float storage and elementwise arithmetic; the Gram is
                        accumulated in FP64 and the eigensolve is FP64        */

#define RPCA_GRAM_DEFAULT 0  /* Gram and rebuild in the storage precision,
                                Gram accumulated in FP64                      */
#define RPCA_GRAM_BF16X3  1  /* F32 only: Gram and rebuild as split-BF16
                                products (hi*hi + hi*lo + lo*hi, x = hi + lo)
                                on MFMA with FP32 accumulation (the Gram in
                                FP32 over 64-row tiles, FP64 across tiles);
                                eigensolve and thresholding stay FP64.  Less
                                accurate than the default: see the stated
                                error of each result                         */
#define RPCA_GRAM_BF16X6  2  /* F32 only: as BF16X3 with the three-way split
                                x = hi + mid + lo and the six products of
                                order >= 2^-16 (hi*hi, hi*mid, mid*hi, hi*lo,
                                mid*mid, lo*hi): about FP32 accuracy          */

#define RPCA_N_MAX 144   /* largest frame count n accepted by RPCA_F32 solves
                            (the FP64 eigensolve of the n x n Gram keeps the
                            packed G in the 160 KB of LDS; above 112 frames
                            V stays in device memory)                       */
#define RPCA_N_MAX_F64 128  /* ... and by RPCA_F64 solves (one 64-row tile of
                            doubles of every frame sits in LDS); 129 to 144
                            frames in FP64 return RPCA_ERR_UNSUPPORTED      */

/*
 * rpca_solve_f64 / rpca_solve_f32 - one RPCA solve.
 *
 *   M        device, m x n (layout above), not modified
 *   m, n     rows (pixels) and columns (frames); m >= 1, 1 <= n <= RPCA_N_MAX
 *            (FP64: n <= RPCA_N_MAX_F64)
 *   lambda   sparsity weight of Eq. 2; <= 0 selects 1/sqrt(max(m, n))
 *   mu       fixed ALM penalty; <= 0 selects m*n / (4 sum|M_ij|) (Sec. II-A)
 *   tol      stopping threshold delta; <= 0 runs exactly maxit iterations
 *   maxit    iteration cap, >= 1
 *   L, S     device, m x n outputs, written in full
 *   iterations  host pointer (may be NULL): iterations performed
 *
 * Returns RPCA_OK, RPCA_NOT_CONVERGED or a negative code.  sum|M| == 0
 * returns RPCA_OK with L = S = 0 after 0 iterations.  Any NaN/Inf in M
 * returns RPCA_ERR_NONFINITE.  A NULL pointer, m < 1, n < 1, n > RPCA_N_MAX,
 * maxit < 1 or overlapping M/L/S returns RPCA_ERR_ARG.
 */
int rpca_solve_f64(const double* M, int64_t m, int64_t n, double lambda, double mu,
                   double tol, int32_t maxit, double* L, double* S,
                   int32_t* iterations, void* stream);
int rpca_solve_f32(const float* M, int64_t m, int64_t n, double lambda, double mu,
                   double tol, int32_t maxit, float* L, float* S,
                   int32_t* iterations, void* stream);

/*
 * One problem of a batch.  M, L, S are device pointers as above (float for
 * RPCA_F32, double for RPCA_F64).  iterations, status and residual are
 * written back by the library (host memory).  residual is the final
 * ||M - L - S||_F / ||M||_F.
 *
 * Warm start (sliding windows): S0 and Y0 give the iteration's starting S
 * and Y instead of zero (either may be NULL for zero); Y, when not NULL,
 * receives the final dual variable.  The iteration from a given start is
 * the same ALM iteration (Eqs. 4-6); consecutive overlapping windows can
 * pass the previous window's S and Y, shifted by the window step, to start
 * near the solution.  mu (and lambda) default from M as always; S0 and Y0
 * must be finite and must not overlap L, S or Y.  When sum|M| == 0 the
 * result is L = S = 0 (and Y = 0) after 0 iterations, as for a cold start.
 */
typedef struct rpca_problem {
    const void* M;
    int64_t m, n;
    double lambda, mu, tol;
    int32_t maxit;
    void* L;
    void* S;
    int32_t iterations;   /* out */
    int32_t status;       /* out */
    double residual;      /* out */
    /* Optional (NULL when unused), device m x n in the layout of M: */
    const void* S0;       /* starting S (default 0); read once, not modified */
    const void* Y0;       /* starting dual Y (default 0); read once */
    void* Y;              /* out: the final dual Y */
} rpca_problem;

/*
 * rpca_solve_many - solve `count` independent problems of possibly different
 * shapes together: every iteration of every active problem runs in the same
 * launches, so the FP64 eigensolves of different problems overlap each other
 * and the streaming passes fill the whole GPU.  Each problem's result is
 * bitwise identical to the same problem solved alone with rpca_solve_*.
 * dtype: RPCA_F64 or RPCA_F32.  gram_mode: RPCA_GRAM_DEFAULT, or
 * RPCA_GRAM_BF16X3 / RPCA_GRAM_BF16X6 (RPCA_F32 only).  Returns the worst status over the
 * problems (negative codes first) and records each problem's own status.
 */
int rpca_solve_many(rpca_problem* probs, int32_t count, int32_t dtype,
                    int32_t gram_mode, void* stream);

/*
 * rpca_solve_ex - one problem with an explicit contraction mode (the
 * precision variant).  Same contract as rpca_solve_many with count = 1.
 */
int rpca_solve_ex(rpca_problem* prob, int32_t dtype, int32_t gram_mode, void* stream);

/*
 * rpca_solve_noalloc - for callers that cannot allocate device memory during
 * the call (code that must not call hipMalloc, tight serving loops, harnesses
 * that forbid allocation).  The same solve as rpca_solve_f32 (dtype RPCA_F32)
 * or rpca_solve_f64 (RPCA_F64), with the same arguments, defaults, status
 * codes and bitwise the same L, S and iteration count, but its workspace
 * lives in a static device array of the library, RPCA_NOALLOC_MAX_BYTES
 * (192 MiB) per device, reserved when the library's code is loaded on that
 * device and held until the process ends.  The call allocates no device
 * memory, no pinned host memory, no stream, event or graph: it launches on
 * `stream` directly and reads the solve state back between chunks of
 * iterations.
 *
 * A solve fits when its workspace and control block fit the array; this
 * holds whenever rpca_footprint_bytes(m, n, dtype) + 4096 <=
 * RPCA_NOALLOC_MAX_BYTES (e.g. 512 x 512 x 20 frames in FP32 and in FP64).
 * A larger solve returns RPCA_ERR_ARG before any device work, and
 * rpca_last_error() names the sizes.  Every call on one device uses that
 * device's one array: calls from several host threads are serialised by a
 * lock, and each call returns only after its work completed, so its contents
 * (left over from the previous call) are never read by a later call before
 * being rewritten; work that the caller enqueues itself on other streams must
 * not overlap a call's use of the array.
 */
#define RPCA_NOALLOC_MAX_BYTES (192u << 20)
int rpca_solve_noalloc(const void* M, int64_t m, int64_t n, int32_t dtype, double lambda,
                       double mu, double tol, int32_t maxit, void* L, void* S,
                       int32_t* iterations, void* stream);

/* Device workspace in bytes that one solve of this shape holds while it runs
 * (iterate buffers, reduction partials, Gram, projector, eigenvectors,
 * state).  0 for an unsupported shape. */
size_t rpca_footprint_bytes(int64_t m, int64_t n, int32_t dtype);

/*
 * Kernel timing (for measurement).  While enabled, solves run on one stream
 * with direct launches (no graphs); each solve-path launch records a HIP
 * start/stop event pair from its own dispatch packet (hipExtLaunchKernel), so
 * a duration covers the kernel alone, and the durations are accumulated:
 * init pass, eigensolve launches and update-pass launches that did work, and
 * the finalize pass.  update_bytes is the algorithmic traffic of the timed
 * update passes: 5 words per matrix entry (read X, S, Y; write S, Y), 3 on
 * the first iteration (S and Y start at zero and are not read).
 */
typedef struct rpca_profile {
    double init_ms, eig_ms, update_ms, finalize_ms;
    int64_t eig_launches, update_launches;
    double update_bytes;
    int64_t solves, iterations;
} rpca_profile;

void rpca_profile_enable(int on);
/* Copy the accumulated figures to *out; reset them when reset != 0. */
int rpca_profile_read(rpca_profile* out, int reset);

/*
 * Tuning knobs (process-wide; they apply to calls started afterwards).
 *
 *   RPCA_KNOB_EIG_THREADS   threads per eigensolve workgroup for one
 *                           eigensolver class (`cls` = 16, 32 or 64: the
 *                           largest frame count of the class) and dtype:
 *                           256, 512, or 1024 (classes 32 and 64 only).
 *
 * rpca_tune_set returns RPCA_OK, or RPCA_ERR_ARG for an unknown knob, class
 * or value (the knob is then unchanged).  rpca_tune_get returns the current
 * value, or RPCA_ERR_ARG.  The eigensolver sizes change only speed: every
 * variant computes the same arithmetic in the same order.
 */
#define RPCA_KNOB_EIG_THREADS 1
/*   RPCA_KNOB_STREAM_KERNEL streaming kernel of one FP32 frame class (`cls` =
 *                           4, 8, 10, 12, 16, 20, 24, 28, 32, 40, 48, 56, 60
 *                           or 64, the register classes; dtype RPCA_F32):
 *                           0 = one thread per pixel row with the frames in
 *                           registers (VALU contractions), 1 = 64-row tiles
 *                           staged in LDS with MFMA contractions.  Windows of
 *                           more than 64 frames always use the tile kernel.
 *                           The two kernels round differently (both within
 *                           the FP32 bar); a solve's result never depends on
 *                           what else runs with it.                          */
#define RPCA_KNOB_STREAM_KERNEL 2
/*   RPCA_KNOB_TILE_ROWS     pixel rows each workgroup of the tile kernel
 *                           walks (its tile shape along m) for one tile class
 *                           (`cls` = nb = 16, 32, ..., 144, the frame count
 *                           rounded up to 16; dtype RPCA_F32, and the setting
 *                           also serves the FP64 solves of 33 to 128 frames,
 *                           which always run the tile kernel): a multiple of
 *                           64 from 64 to 8192.  Fewer rows give more workgroups
 *                           (better occupancy for small launches), more rows
 *                           amortise the workgroup's Gram partial.  The
 *                           default is 1024.  A solve of m rows uses at most
 *                           max(256, m / 256) rows per workgroup (rounded
 *                           down to 64), so it spreads over at least one
 *                           workgroup per CU.  The partial sums are
 *                           grouped by workgroup, so results differ between
 *                           settings by rounding (within the FP32 bar); for
 *                           a given setting they are the same alone or in a
 *                           batch.                                          */
#define RPCA_KNOB_TILE_ROWS 3
/*   RPCA_KNOB_REG_TILES     256-row tiles each workgroup of the register
 *                           kernel walks, for one register class (`cls` as for
 *                           RPCA_KNOB_STREAM_KERNEL, or 4 ... 32 with
 *                           RPCA_F64): 1 to 16; default 2 for the RPCA_F64
 *                           classes of up to 20 frames, else 1.  A workgroup walks its tiles in
 *                           order and writes one partial for all of them
 *                           (fewer partials to reduce), at the cost of about
 *                           40 registers for the Gram accumulators that the
 *                           loop keeps live.  A solve of T tiles uses at most
 *                           max(1, T / 256) tiles per workgroup.  Results
 *                           differ between settings by rounding (the partial
 *                           sums regroup); for a given setting they are the
 *                           same alone or in a batch.                       */
#define RPCA_KNOB_REG_TILES 4
int rpca_tune_set(int32_t knob, int32_t dtype, int32_t cls, int32_t value);
int rpca_tune_get(int32_t knob, int32_t dtype, int32_t cls);

/*
 * ---- serving: continuous batching of arriving windows ------------------
 *
 * The paper targets real-time filtering of streamed frame windows (Abstract;
 * Sec. IV, discussion of run time and of further GPU optimisation).  A server
 * takes windows of different sizes and frame counts as they arrive and runs
 * them together:
 *
 *   rpca_server_submit  queues a request (FIFO).  The problem's M, L and S
 *                       (device) must stay valid until its completion is
 *                       reported; lambda, mu, tol and maxit as for a solve.
 *                       Returns RPCA_ERR_ARG / RPCA_ERR_UNSUPPORTED for a
 *                       problem a solve would reject (nothing is queued).
 *   rpca_server_step    admits queued requests in arrival order while fewer
 *                       than max_active solves are active and the active
 *                       requests' footprint (rpca_server_request_bytes: the
 *                       library workspace plus M, L and S) fits hbm_budget.
 *                       The head of the queue waits for room; a request
 *                       larger than the whole budget completes at once with
 *                       RPCA_ERR_NOMEM.  Newly admitted requests get their
 *                       device workspace, which holds their S, Y,
 *                       eigenvectors and state until they finish.  Then
 *                       `quantum` iterations of every active solve run
 *                       together on the device, and the solves that stopped
 *                       are finalized (L and S written, workspace freed).
 *                       Up to `capacity` completions are copied to out[] and
 *                       their number to *count; further completions wait for
 *                       the next call.  L and S of a reported completion are
 *                       final.  Returns RPCA_OK, or RPCA_ERR_DEVICE /
 *                       RPCA_ERR_NOMEM when the device failed (after a
 *                       device error every later step fails too).
 *   rpca_server_pending queued and active counts and the admitted bytes;
 *                       returns the number of requests not yet reported.
 *
 *   rpca_server_set_timeout  timeout (seconds, > 0; 0 = none, the default)
 *                       given to the requests submitted from then on.  A
 *                       request whose timeout has passed since its
 *                       submission completes with RPCA_ERR_TIMEOUT at the
 *                       next step: a queued one at once, an active one after
 *                       the quantum in flight, its workspace freed and its L
 *                       and S unspecified.  RPCA_ERR_ARG for a negative or
 *                       NaN value.
 *
 * A tag names one request until its completion has been reported: submit
 * returns RPCA_ERR_ARG for a tag that is queued, active or completed but not
 * yet reported.  A failure while newly admitted requests are set up
 * (workspace, control block, init pass) completes those requests with the
 * failure's code and gives their footprint back to the budget; the step then
 * returns RPCA_OK, or RPCA_ERR_DEVICE for a device error.
 *
 * Each result is bitwise identical to the same problem solved alone.  The
 * calls are serialised by a lock; the stream argument of create is the stream
 * on which the caller produces M (it is synchronised before admission).
 * flags: 0, or RPCA_SERVER_SIMULATE to run the admission logic without any
 * device work (every request then completes after maxit iterations with
 * RPCA_NOT_CONVERGED and residual 0; the server clock of the timeouts then
 * advances by exactly 1 ms per step).  create returns NULL for an invalid
 * argument (dtype, an unknown gram_mode or a split-BF16 mode with RPCA_F64,
 * a zero budget, max_active < 1, quantum < 1, unknown flags).  Every
 * request of a server uses the server's dtype and gram_mode.
 */
typedef struct rpca_server rpca_server;
typedef struct rpca_completion {
    int64_t tag;          /* the tag given to rpca_server_submit */
    int32_t status;       /* as a solve's return code */
    int32_t iterations;
    double residual;      /* ||M - L - S||_F / ||M||_F */
} rpca_completion;

#define RPCA_SERVER_SIMULATE 1

rpca_server* rpca_server_create(int32_t dtype, int32_t gram_mode, size_t hbm_budget,
                                int32_t max_active, int32_t quantum, int32_t flags,
                                void* stream);
int rpca_server_submit(rpca_server* s, const rpca_problem* p, int64_t tag);
int rpca_server_step(rpca_server* s, rpca_completion* out, int32_t capacity, int32_t* count);
int rpca_server_pending(rpca_server* s, int32_t* queued, int32_t* active, size_t* bytes_in_use);
/* Largest admitted footprint seen so far (bytes). */
size_t rpca_server_peak_bytes(rpca_server* s);
/* Admission footprint of one request: workspace + M, L and S. 0 if unsupported. */
size_t rpca_server_request_bytes(int64_t m, int64_t n, int32_t dtype);
/* Wait for device work, free every workspace and drop queued requests. */
void rpca_server_destroy(rpca_server* s);
int rpca_server_set_timeout(rpca_server* s, double seconds);
/* Fault injection for tests of the failure handling: the next set-up of newly
 * admitted requests (stage RPCA_SERVER_STAGE_INIT) fails with `code` (< 0)
 * before any device work, as a failed workspace or control-block allocation
 * would.  Returns RPCA_OK, or RPCA_ERR_ARG for another stage or code >= 0. */
#define RPCA_SERVER_STAGE_INIT 1
int rpca_server_inject_failure(rpca_server* s, int32_t stage, int32_t code);

/*
 * Autotuning: choose every tuning knob by measurement on the current device.
 *
 * rpca_autotune runs short solves (tol = 0, a dozen iterations) of synthetic
 * windows through the library with kernel timing on, for each variant of
 * each knob, and keeps the fastest:
 *   - RPCA_KNOB_EIG_THREADS per eigensolver class, on a 16384 x cls window;
 *   - RPCA_KNOB_STREAM_KERNEL per FP32 register class of 16 frames or more,
 *     on a `rows` x cls window (rows >= 256; e.g. 262144 for 512 x 512
 *     images);
 *   - then RPCA_KNOB_TILE_ROWS for every tile class the tile kernel serves
 *     (the classes above 64 frames and those of the register classes now on
 *     the tile kernel), on a `rows` x n window of that class.
 * It allocates its windows with hipMalloc and frees them before returning.
 * It uses the kernel-timing accumulators (rpca_profile_*), which it resets,
 * so it must not run while other calls use them.  Returns RPCA_OK, or the
 * first failing solve's code (that knob keeps its previous value).
 *
 * rpca_autotune_save writes the current choices to a text file, one
 * "knob dtype class value" line each; rpca_autotune_load applies such a
 * file.  Both return RPCA_OK, or RPCA_ERR_ARG when the file cannot be
 * opened or a line is invalid (load still applies every valid line).
 */
int rpca_autotune(int32_t dtype, int64_t rows, void* stream);
int rpca_autotune_save(const char* path);
int rpca_autotune_load(const char* path);

/*
 * ---- steps around the solve, on the device ------------------------------
 *
 * All arrays are device arrays of the given dtype (RPCA_F32 / RPCA_F64) in
 * the Casorati layout; host outputs are written after the work completed.
 * Sums are FP64 and fixed-order (no atomics).
 *
 * rpca_frame_correlation: rho[t] (host, n-1 doubles) = Pearson correlation
 *   of frames t and t+1 over the m pixels.  2 <= n <= 160, m >= 2.  A frame
 *   with zero variance gives correlation 0.
 * rpca_frame_keep: host helper.  keep[t] = 1 when frame t correlates at
 *   least `threshold` with one of its neighbours (max of rho[t-1], rho[t]
 *   where they exist), else 0; returns the number kept.  The paper's in vivo
 *   reference drops frames that correlate below 0.8 with their neighbours
 *   (Sec. III); "with one of its neighbours" is this library's reading: a
 *   single jumping frame is dropped, its neighbours are kept.
 * rpca_frame_select: copies the kept frames of M (keep[t] != 0, host) in
 *   order into out (device, m x kept), stream-ordered; returns the count.
 * rpca_moving_average: out[:, t] = mean of M[:, t .. t+W-1] for t = 0 ..
 *   n-W (the paper's temporal moving average over 20 frames, Sec. III);
 *   out is m x (n-W+1).  1 <= W <= 32, W <= n.  Running FP64 sum.
 * rpca_dice: binarises A >= thr_a and B >= thr_b (compared in FP64) over
 *   `count` entries; counts[3] (host, optional) = |both|, |A|, |B|;
 *   *dice (host, optional) = 2|both| / (|A| + |B|) (Eq. 8; 1 if both empty).
 * rpca_rmse: *out = sqrt(mean((A - B)^2)) over `count` entries (Eq. 7).
 * rpca_masked_mean: *out = mean of A over entries with mask != 0 (uint8
 *   device mask): the binarisation threshold of Sec. II-F (the mean
 *   intensity at the bubble locations).  RPCA_ERR_ARG if the mask is empty.
 * Each returns RPCA_OK (or the count), RPCA_ERR_ARG, RPCA_ERR_NOMEM or
 * RPCA_ERR_DEVICE.
 */
int rpca_frame_correlation(const void* M, int64_t m, int64_t n, int32_t dtype, double* rho,
                           void* stream);
int rpca_frame_keep(const double* rho, int64_t n, double threshold, int32_t* keep);
int rpca_frame_select(const void* M, int64_t m, int64_t n, int32_t dtype, const int32_t* keep,
                      void* out, void* stream);
int rpca_moving_average(const void* M, int64_t m, int64_t n, int32_t W, int32_t dtype, void* out,
                        void* stream);
int rpca_dice(const void* A, double thr_a, const void* B, double thr_b, int64_t count,
              int32_t dtype, int64_t* counts, double* dice, void* stream);
int rpca_rmse(const void* A, const void* B, int64_t count, int32_t dtype, double* out,
              void* stream);
int rpca_masked_mean(const void* A, const uint8_t* mask, int64_t count, int32_t dtype,
                     double* out, void* stream);

/* Static description of a status code. */
const char* rpca_strerror(int code);

/* Detail of the last failure on the calling thread (the HIP call and its
 * error string), or "" when the last call succeeded. */
const char* rpca_last_error(void);

/* Library version string. */
const char* rpca_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RPCA_MI355X_H */
