/*
 * libfv -- Fisher-vector encoding of local descriptors against a diagonal GMM, on AMD
 * Instinct MI355X (gfx950).  C ABI: plain pointers and sizes, no C++ or framework types.
 *
 * The operation (Ma et al., "GPU-FV: Realtime Fisher Vector and Its Applications in Video
 * Monitoring", ICMR 2016, Sec. 3.1 and Algorithm 1; normalisation of the improved Fisher
 * vector of Perronnin et al. / Sanchez et al., which the paper cites and whose VLFeat
 * implementation its experiments follow, Sec. 4):
 *
 *   input   N descriptors x_t in R^D; a K-component diagonal GMM (weights w_k, means mu_k,
 *           variances var_k = sigma_k^2)
 *   gamma   gamma_tk = w_k N(x_t; mu_k, var_k) / sum_j w_j N(x_t; mu_j, var_j)
 *           (the per-descriptor posterior / soft assignment, Algorithm 1 first loop)
 *   u_kd    = 1/(N sqrt(w_k))   sum_t gamma_tk (x_td - mu_kd) / sigma_kd
 *   v_kd    = 1/(N sqrt(2 w_k)) sum_t gamma_tk [((x_td - mu_kd) / sigma_kd)^2 - 1]
 *           (Algorithm 1 second loop, with the Fisher-information scaling)
 *   phi     = [u ; v], each block component-major (index k*D + d), length 2*K*D
 *   unless FV_NO_POWER_NORM: phi_i <- sign(phi_i) sqrt(|phi_i|)
 *   unless FV_NO_L2_NORM:    phi   <- phi / ||phi||_2  (left unscaled when the norm is 0)
 *
 * No posterior threshold is applied (every term is accumulated) unless FV_THRESHOLD asks for
 * the paper's mode: a term (t, k) then enters u, v (and the gamma sum inside v) only if
 * gamma_tk > FV_THRESHOLD_TAU (Algorithm 1's test), and groups of MFMA steps whose terms all
 * fall below it are skipped (the paper's early termination of Phase 2, Sec. 3.3).  A frame with
 * N = 0 encodes to 2KD zeros.  Non-finite descriptor values are not checked: a NaN makes every
 * statistic of its frame NaN, so with FV_NO_POWER_NORM the vector is NaN, while the signed
 * square root takes the sign of NaN as 0 and the normalised vector is then all zeros.
 *
 * Return codes: FV_OK (0), FV_PENDING (1), or a negative FV_E_* code; fv_strerror() names
 * them.  No C++ exception crosses this interface.  Functions are thread-safe unless stated.
 */
#ifndef FV_H_
#define FV_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------------------------- */
#define FV_OK 0
#define FV_PENDING 1
#define FV_E_INVAL (-1)       /* bad argument (sizes, null pointers, GMM values, flags) */
#define FV_E_NOMEM (-2)       /* device or pinned host allocation failed */
#define FV_E_DEVICE (-3)      /* a HIP runtime call failed; see fv_last_device_error() */
#define FV_E_BUDGET (-4)      /* a request can never fit the server's device-memory budget */
#define FV_E_AGAIN (-5)       /* server queue full; retry later */
#define FV_E_NOTFOUND (-6)    /* unknown server ticket */
#define FV_E_TIMEOUT (-7)     /* request exceeded its deadline */
#define FV_E_UNSUPPORTED (-8) /* valid request outside this build's limits (see fv_limits) */

/* ---- arithmetic forms ------------------------------------------------------------------ */
#define FV_PREC_FP32 0        /* both contractions on FP32 MFMA, FP32 accumulate */
#define FV_PREC_BF16_SPLIT 1  /* bf16 hi/lo operands, 3 products (hi*hi + hi*lo + lo*hi) */
#define FV_PREC_FP16_SPLIT 2  /* fp16 hi/lo operands, 3 products */
#define FV_PREC_BF16 3        /* plain bf16 operands (accuracy control only) */
/*
 * Range of the fp16 split: the operand entries mu/sigma^2 and 1/(2 sigma^2) (times log2 e)
 * and the descriptor values x and x^2 are rounded to fp16, whose largest finite value is
 * 65504.  A model with an entry beyond it (a variance below about 1.1e-5, or a large
 * |mu|/sigma^2) is refused for this form with FV_E_UNSUPPORTED; descriptors need |x| < 255.9,
 * else the result is not finite.  Entries below 2^-14 lose relative precision (fp16
 * subnormals).  The bf16 forms have the FP32 exponent range.
 */

/* ---- flags ----------------------------------------------------------------------------- */
#define FV_X_DEVICE 1u        /* X (and offsets' rows) live in device memory; else host memory */
#define FV_OUT_DEVICE 2u      /* out lives in device memory; else host memory */
#define FV_NO_POWER_NORM 4u   /* skip the signed square root */
#define FV_NO_L2_NORM 8u      /* skip the L2 normalisation */
#define FV_ASYNC 16u          /* return after enqueueing on the stream, without waiting */
#define FV_THRESHOLD 32u      /* the paper's posterior threshold (see above) */
#define FV_THRESHOLD_TAU 1e-6 /* its value: terms with gamma <= 1e-6 are left out */

typedef struct fv_gmm fv_gmm;

/* Size limits of this build: K <= max_K, D <= max_D (any K >= 1, D >= 1 below them). */
void fv_limits(int* max_K, int* max_D);

/*
 * Load a diagonal GMM onto device `device` (Algorithm 1 precomputes the inverse standard
 * deviation once per model; here the whole per-model constant set is evaluated once, in double precision, on the host:
 * 1/sigma, 1/sigma^2, the E-step operand [mu/sigma^2 ; -1/(2 sigma^2)] and offsets
 * ln w_k - 1/2 sum_d ln sigma^2_kd - 1/2 sum_d mu_kd^2/sigma^2_kd, and the block scales
 * 1/sqrt(w_k), 1/sqrt(2 w_k)).
 *   priors    [K]     host float32, every entry finite and > 0; used as given (no
 *                     renormalisation to sum 1)
 *   means     [K x D] host float32 row-major (component-major), finite
 *   variances [K x D] host float32 row-major, finite and > 0 (variances, not std devs)
 *   out       receives an opaque, immutable handle; share it freely between threads
 * The caller keeps ownership of its arrays and may free them on return.
 * Errors: FV_E_INVAL (null pointer, K < 1, D < 1, a bad value), FV_E_UNSUPPORTED (K or D over
 * the limits), FV_E_NOMEM, FV_E_DEVICE.  On error *out is set to NULL.
 */
int fv_gmm_load(int K, int D, const float* priors, const float* means, const float* variances,
                int device, fv_gmm** out);

/* Release a handle (NULL is accepted).  No call using it may still be in flight. */
int fv_gmm_free(fv_gmm* gmm);

/* K, D and device of a handle (any pointer may be NULL). */
int fv_gmm_info(const fv_gmm* gmm, int* K, int* D, int* device);

/*
 * Encode one frame: X [N x D] float32 row-major -> out [2*K*D] float32, laid out as above.
 *   flags      FV_X_DEVICE / FV_OUT_DEVICE say where X and out live (host otherwise);
 *              FV_NO_POWER_NORM / FV_NO_L2_NORM drop the normalisation steps;
 *              FV_THRESHOLD leaves out terms with gamma <= FV_THRESHOLD_TAU;
 *              FV_ASYNC returns once the work is enqueued on `hip_stream` -- the caller then
 *              keeps X and out alive (host buffers too) until that stream is synchronised.
 *   hip_stream a hipStream_t (NULL = the default stream) on the handle's device.
 * The caller owns X and out.  N = 0 writes zeros.  Device X must be 4-byte aligned; a
 * 16-byte aligned X with D % 4 == 0 takes the vector-load path.
 * Errors: FV_E_INVAL (null pointers, N < 0, bad precision or flags), FV_E_UNSUPPORTED (the
 * fp16 split for a model outside its range, see above), FV_E_NOMEM, FV_E_DEVICE.
 */
int fv_encode(const fv_gmm* gmm, const float* X, int64_t N, float* out, int precision,
              unsigned flags, void* hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): fv_encode with every intermediate in one fixed
 * scratch array per GPU of FV_NOALLOC_SCRATCH_BYTES bytes, which the library's code object
 * holds on each GPU it runs on from load until the process ends.  X and out must be device
 * memory (FV_X_DEVICE and FV_OUT_DEVICE set, else FV_E_INVAL).  The call allocates nothing,
 * captures no graph and records no event.  A frame whose intermediates do not fit fails with
 * FV_E_UNSUPPORTED before anything is launched.  The per-chunk partial statistics are
 * bounded (at most one chunk per resident workgroup: about 34 MB at K = 256, D = 64 and 22 MB at
 * K = 512, D = 80); beyond them the intermediates grow with N only through the two-pass path's
 * per-row normalisers (8 bytes per row and group of 256 components), so frames up to about 2.8
 * million rows fit at K = 512, D = 80, and any N at K <= 256, D <= 64.  Within the limit the result is the one of fv_encode with the same kernels (the
 * two-pass path and the E-step recompute stand in where the preferred plan would not fit).
 * Every call on a GPU uses the same scratch: calls that overlap in time on one GPU (other
 * streams, other threads) race and give wrong results, so serialise them; FV_ASYNC calls on
 * one stream are ordered and safe.  The scratch keeps the last call's contents; no part of it
 * needs to start at zero (every intermediate is written before it is read).
 */
#define FV_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int fv_encode_noalloc(const fv_gmm* gmm, const float* X, int64_t N, float* out, int precision,
                      unsigned flags, void* hip_stream);

/*
 * Encode B frames in one launch sequence.  Frame b is rows [offsets[b], offsets[b+1]) of
 * X [offsets[B] x D]; out is [B x 2*K*D].  `offsets` is a HOST array of B+1 int64 values
 * with offsets[0] == 0 and offsets non-decreasing (else FV_E_INVAL).  Frames are split into
 * chunks relative to their own first row, so a frame's result does not depend on the other
 * frames in the batch (bitwise).  Other arguments as fv_encode.
 */
int fv_encode_batch(const fv_gmm* gmm, const float* X, const int64_t* offsets, int B, float* out,
                    int precision, unsigned flags, void* hip_stream);

/*
 * Launch tuning of one handle (set by an autotuner; the defaults are automatic choices).
 *   batch_chunk         rows per frame-relative chunk in fv_encode_batch (rounded down to a
 *                       multiple of 128; 0 = 1024).  Changing it changes the summation order
 *                       of the batched path (results agree within rounding, not bitwise).
 *   batch_path          0 = automatic (fused single pass when K <= 256), 1 = fused, 2 = two-pass
 *   single_split_below  fv_encode takes the two-pass path for N below this (0 = automatic:
 *                       four 32-row tiles per resident workgroup)
 *   batch_grid          workgroups of fv_encode_batch's statistics launch (the fused kernel or
 *                       the first pass; 0 = automatic: the resident workgroup count); the
 *                       kernels loop over the work items, so results do not depend on it
 *   fused16_variant     fused 16-bit kernel at 256 components, DP <= 64: 0 = automatic (the
 *                       pipelined kernel), 1 = wave-specialised with two barriers per tile,
 *                       2 = single-role (transposed E-step), 3 = wave-specialised and
 *                       pipelined (one barrier per tile); 1 and 3 give the same bits, 2 agrees
 *                       within rounding
 * Not synchronised with encodes running concurrently on the same handle.  Errors: FV_E_INVAL.
 */
typedef struct fv_tuning {
  int batch_chunk;
  int batch_path;
  int64_t single_split_below;
  int batch_grid;
  int fused16_variant;
} fv_tuning;

int fv_gmm_set_tuning(fv_gmm* gmm, const fv_tuning* tuning); /* NULL restores the defaults */
int fv_gmm_get_tuning(const fv_gmm* gmm, fv_tuning* tuning);

/*
 * Environment switches read at each call (for tests and measurements; results stay within the
 * gates either way):
 *   FV_PATH=fused|split   force the single-pass or two-pass path where both exist
 *   FV_BATCH_CHUNK=n      rows per frame-relative chunk of fv_encode_batch (multiple of 128)
 *   FV_GRAPH=0            never capture or replay graphs
 *   FV_SPLIT_GAMMA=0      FP32 two-pass frames recompute the E-step in the second pass instead
 *                         of reading the posterior factors the first pass wrote
 *   FV_MAX_GRID=n         cap the first grid dimension of every statistics launch at n
 *   FV_FUSED16=w|t|p      the fused 16-bit kernel variant at 256 components: wave-specialised,
 *                         single-role or pipelined (fused16_variant 1, 2, 3), over the tuning
 */

/*
 * Kernel timing (instrumentation for benchmarks and profilers).  fv_kernel_timing(1) resets
 * the counters and starts bracketing every launch of libfv's kernels with HIP events on the
 * stream the kernel is launched on; fv_kernel_timing(0) stops.  fv_kernel_timing_read waits
 * for the recorded events and returns the summed device duration (ms) and the launch count
 * of kernel class `which` (0 = statistics kernels, 1 = finalize kernels, 2 = projection
 * kernel) since the reset.
 * Errors: FV_E_INVAL (bad `which`), FV_E_DEVICE.
 */
int fv_kernel_timing(int enable);
int fv_kernel_timing_read(int which, double* total_ms, int64_t* launches);

/* ---- projection prologue ------------------------------------------------------------- */
/*
 * Dimension reduction of the raw descriptors before encoding (Sec. 3.1: the 128 dense-SIFT
 * values are reduced to m dimensions by PCA and the normalised image coordinates appended,
 * giving the D = m + 2 the GMM is trained on).  The prologue computes, per descriptor,
 *   y = A (x - m),   A [D x Din] row-major, m [Din]
 * so appended coordinates are identity rows of A (with m = 0 in their columns).  One MFMA
 * contraction per 32-descriptor tile: FP32 MFMA for the FP32 encoder form, the bf16 hi/lo
 * split (three products, FP32 accumulation) for the 16-bit forms; y is FP32 in every form.
 *
 * fv_pca_load copies A and m (host pointers) to `device` and precomputes -A m in FP64.
 * Requires 1 <= Din <= 256 (FV_E_UNSUPPORTED above), 1 <= D <= the fv_limits maximum, and
 * finite values, else FV_E_INVAL.  The handle is immutable and may be shared across threads;
 * fv_pca_free releases it.
 */
typedef struct fv_pca fv_pca;
int fv_pca_load(int Din, int D, const float* A, const float* mean, int device, fv_pca** out);
int fv_pca_free(fv_pca* pca);
int fv_pca_info(const fv_pca* pca, int* Din, int* D, int* device);

/*
 * Projection alone: X [N x Din] -> Y [N x D], both row-major float32; FV_X_DEVICE and
 * FV_OUT_DEVICE say where X and Y live, FV_ASYNC as for fv_encode; FV_PROJ_SPLIT16 selects
 * the split-bf16 contraction the 16-bit encoder forms use (the same bits as their prologue).
 * Errors: FV_E_INVAL (null pointers, N < 0, other flags), FV_E_NOMEM, FV_E_DEVICE.
 */
#define FV_PROJ_SPLIT16 64u
int fv_project(const fv_pca* pca, const float* X, int64_t N, float* Y, unsigned flags,
               void* hip_stream);

/*
 * fv_encode / fv_encode_batch of the projected descriptors: X holds raw descriptors of Din
 * values per row (host or device, per FV_X_DEVICE); the projection runs on the device into
 * the library's scratch and feeds the encoder, within the same stream order (and the same
 * captured graph).  Requires pca's D == gmm's D and the same device, else FV_E_INVAL.
 * Otherwise as fv_encode / fv_encode_batch.
 */
int fv_encode_projected(const fv_gmm* gmm, const fv_pca* pca, const float* X, int64_t N,
                        float* out, int precision, unsigned flags, void* hip_stream);
int fv_encode_batch_projected(const fv_gmm* gmm, const fv_pca* pca, const float* X,
                              const int64_t* offsets, int B, float* out, int precision,
                              unsigned flags, void* hip_stream);

/* ---- dense-SIFT front end ----------------------------------------------------------------
 * Flat-window dense SIFT on the GPU (Sec. 3.1: per scale of the image, the gradient of every
 * pixel falls into 8 orientation bins, a triangular convolution follows, and each descriptor
 * holds the 8 values of 4 x 4 spatial bins, taken at a stride; Sec. 3.2: the triangular filter
 * is applied once along each image dimension, and the second convolution only where a
 * descriptor reads it; Sec. 4: stride 4 and scales from 2 (or sqrt 2) down to 1/8).  The paper
 * leaves the resampling, gradient, binning, window and normalisation unstated; this library
 * computes, per scale s of an H x W grayscale image (float32, row-major):
 *   resize       Hs = round(s H), Ws = round(s W) (ties to even; the image itself at s = 1),
 *                bilinear at the source point ((x + 1/2) / s - 1/2, (y + 1/2) / s - 1/2)
 *                clamped to the image
 *   gradient     central differences (I[x+1] - I[x-1]) / 2, one-sided at the first and last
 *                column (row)
 *   binning      t = 8 atan2(gy, gx) / (2 pi) in [0, 8); magnitude shared by bins floor(t)
 *                (weight 1 - frac t) and floor(t) + 1 mod 8 (weight frac t)
 *   window       w(d) = (B - |d|) / B^2 for |d| < B (B = `bin`), zero outside the image,
 *                along y, then along x
 *   sampling     descriptor (x0, y0) = (a step, b step), x0 + 3B <= Ws - 1, y0 + 3B <= Hs - 1;
 *                spatial bin (i, j) reads the filtered maps at (x0 + i B, y0 + j B); value
 *                (4 j + i) * 8 + o
 *   normalise    L2, clamp at 0.2, L2 (a zero vector stays zero)
 *   row          the 128 values, then ((x0 + 1.5 B + 1/2) / Ws - 1/2, (y0 + 1.5 B + 1/2) / Hs
 *                - 1/2): FV_DSIFT_DIM = 130 floats, rows of scale 0 first, then scale 1, ...
 * Arithmetic is float32 (resampling coordinates in double); results agree with a float64
 * evaluation to rounding.
 *   scales       n_scales factors (1..16, finite and > 0), or NULL for the n_scales (1..9)
 *                smallest of 2, sqrt 2, 1, ..., 1/8 (8: the paper's 8-scale setting)
 *   bin, step    1 <= bin <= 16, step >= 1
 * Limits: H, W <= 16384, scaled sides <= 32768 (FV_E_UNSUPPORTED beyond).
 */
#define FV_DSIFT_DIM 130

/* Descriptors one image yields (*n_rows; 0 when no scale fits a descriptor).  Errors:
 * FV_E_INVAL (bad sizes, scales, bin or step), FV_E_UNSUPPORTED. */
int fv_dsift_rows(int H, int W, int n_scales, const double* scales, int bin, int step,
                  int64_t* n_rows);

/* Extract the descriptors of n_images images [n_images x H x W] (FV_X_DEVICE: device memory,
 * else host) into rows [n_images x n_rows x FV_DSIFT_DIM] (FV_OUT_DEVICE: device memory, 8-byte
 * aligned, else host) on `device`, stream `hip_stream`; FV_ASYNC as for fv_encode.  The caller
 * owns both arrays.  Errors: FV_E_INVAL (null pointers, bad sizes or flags),
 * FV_E_UNSUPPORTED (n_images > 65535 or the limits above), FV_E_NOMEM, FV_E_DEVICE. */
int fv_dsift(const float* images, int n_images, int H, int W, int n_scales,
             const double* scales, int bin, int step, float* rows, unsigned flags, int device,
             void* hip_stream);

/* Fisher vector of each image: fv_dsift (into the library's scratch), the projection `pca`
 * (Din = FV_DSIFT_DIM, D = the GMM's D), then the batched encode with image n as frame n, or,
 * when the images have too few rows to fill the GPU's resident workgroups in batch chunks, an
 * fv_encode of each image (the same vectors within rounding); out [n_images x 2KD].  Images on the host (copied in) or device (FV_X_DEVICE); out per
 * FV_OUT_DEVICE; other flags and errors as fv_encode_batch and fv_dsift. */
int fv_encode_images(const fv_gmm* gmm, const fv_pca* pca, const float* images, int n_images,
                     int H, int W, int n_scales, const double* scales, int bin, int step,
                     float* out, int precision, unsigned flags, void* hip_stream);

/* ---- training step -------------------------------------------------------------------- */
/*
 * One EM iteration for the GMM (the model the encoder uses is trained beforehand, Sec. 3.1).
 * The E-step and the sums are the encoder's own kernels (first pass: per-row normalisers;
 * statistics pass: S0 = sum_t gamma_tk, S1 = gamma^T X, S2 = gamma^T X^2, precision as for
 * fv_encode); then, in double on the device:
 *   w_k = S0_k / N,   mu_kd = S1_kd / S0_k,   var_kd = max(S2_kd / S0_k - mu_kd^2, var_floor)
 * (a component with S0_k = 0 gets w_k = 0, mu_k = 0, var_k = var_floor; such a model is not
 * loadable until the caller re-seeds it), and the log-likelihood of X under the current model,
 *   loglik = sum_t ln sum_k w_k N(x_t; mu_k, diag var_k).
 * X [N x D] float32 row-major, host or device (FV_X_DEVICE; no other flag).  Outputs are host
 * arrays: weights [K], means [K x D], variances [K x D] (float32), *loglik (double).  Returns
 * after the stream has finished.  Errors: FV_E_INVAL (null pointers, N < 1, bad precision,
 * flags, negative or non-finite var_floor), FV_E_UNSUPPORTED (the fp16 split out of range),
 * FV_E_NOMEM, FV_E_DEVICE.
 */
int fv_em_step(const fv_gmm* gmm, const float* X, int64_t N, int precision, float var_floor,
               unsigned flags, void* hip_stream, float* weights, float* means, float* variances,
               double* loglik);

/* ---- serving ------------------------------------------------------------------------------
 * A server keeps one GMM and its own HIP streams, accepts frames of any size from any thread,
 * and encodes them with continuous batching: a scheduler thread admits queued requests in
 * arrival order while their device-memory footprint fits the budget, groups them into one
 * batched launch (fv_encode_batch semantics, so each frame's result is bitwise the same alone
 * or in any mix), and runs up to n_streams launches concurrently; requests that arrive while
 * others are on the GPU are admitted as soon as a stream and budget are free.  The paper runs
 * one frame at a time for its real-time video applications (Sec. 4.2); serving is new here.
 */
typedef struct fv_server fv_server;

#define FV_EXEC_HIP 0   /* encode on the GPU */
#define FV_EXEC_FAKE 1  /* host-only test executor: no device use; a batch "completes" after
                           fake_us_per_krow microseconds per 1000 rows and yields zeros */

typedef struct fv_server_config {
  size_t hbm_budget_bytes;  /* device bytes in-flight batches may hold (0 = unlimited) */
  int precision;            /* FV_PREC_* */
  unsigned flags;           /* FV_NO_POWER_NORM / FV_NO_L2_NORM / FV_THRESHOLD only */
  int max_queue;            /* requests waiting for admission (<= 0: 4096) */
  int n_streams;            /* concurrent launches (<= 0: 2) */
  int max_batch_frames;     /* frames per launch (<= 0: 64) */
  int64_t max_batch_rows;   /* rows per launch (<= 0: 262144) */
  double deadline_ms;       /* a request not admitted within this time fails with
                               FV_E_TIMEOUT (<= 0: no deadline) */
  double batch_window_us;   /* a launch that is not yet full waits until its oldest request is
                               this old, to collect more frames (<= 0: launch at once) */
  int executor;             /* FV_EXEC_HIP or FV_EXEC_FAKE */
  int fake_K, fake_D;       /* FV_EXEC_FAKE only: output size 2*K*D when gmm is NULL */
  double fake_us_per_krow;  /* FV_EXEC_FAKE only */
  int fake_fail_every;      /* FV_EXEC_FAKE only: every n-th batch fails with FV_E_DEVICE */
  int copy_threads;         /* helper threads that share the submit-side copy of a host frame of
                               2 MiB or more into its pinned staging (0: the submitting thread
                               copies alone; default 3; at most 16) */
} fv_server_config;

typedef struct fv_req_stats {
  double t_submit_us, t_admit_us, t_start_us, t_done_us;  /* server clock (steady, microseconds
                                                              since fv_server_create) */
  int64_t rows;
  int batch_frames;  /* frames in the launch that carried this request */
  int status;        /* FV_OK or the failure code */
} fv_req_stats;

typedef struct fv_server_stats {
  int64_t submitted, completed, failed, rejected;
  int64_t launches;
  int64_t rows_done;
  int queued, in_flight;
  size_t admitted_bytes, peak_admitted_bytes;
  double p50_ms, p99_ms, max_ms;  /* submit-to-done latency of completed requests */
  double busy_s;                  /* wall time with at least one launch in flight */
  int64_t cancelled;              /* requests withdrawn by fv_server_cancel */
  int64_t graph_captures;         /* graphs captured on the server's streams (not reset) */
  int64_t graph_replays;          /* graph replays on the server's streams (not reset) */
} fv_server_stats;

/* Fill a config with the defaults above (budget unlimited, FP32, HIP executor). */
void fv_server_config_default(fv_server_config* cfg);

/* Create a server for `gmm` (may be NULL only with FV_EXEC_FAKE).  The handle must outlive the
 * server.  Errors: FV_E_INVAL, FV_E_UNSUPPORTED (the fp16 split out of range), FV_E_NOMEM,
 * FV_E_DEVICE. */
int fv_server_create(const fv_gmm* gmm, const fv_server_config* cfg, fv_server** out);

/* Stop the scheduler (waits for in-flight launches) and free everything; unpolled results are
 * discarded. */
int fv_server_destroy(fv_server* srv);

/* Enqueue one frame X [N x D] (host memory; copied before return, so the caller may reuse X).
 * Thread-safe and non-blocking.  Returns FV_OK and a ticket, FV_E_BUDGET if the frame can never
 * fit the budget, FV_E_AGAIN if the queue is full, FV_E_UNSUPPORTED for N above the encoder's
 * row limit (2^40 / D), FV_E_INVAL for bad arguments. */
int fv_server_submit(fv_server* srv, const float* X, int64_t N, uint64_t* ticket);

/* As fv_server_submit for a frame already in device memory: X [N x D] f32 row-major on the
 * server's GPU.  Nothing is copied at submit time; the launch gathers the frame with a
 * device-to-device copy, so the caller keeps X valid and unmodified until the ticket has
 * finished (fv_server_poll returned something other than FV_PENDING).  Same return codes. */
int fv_server_submit_device(fv_server* srv, const float* X, int64_t N, uint64_t* ticket);

/* Result of a ticket: FV_PENDING while queued or running; FV_OK with out (host, 2*K*D floats,
 * may be NULL) and st (may be NULL) filled -- the ticket is then consumed; a failure code
 * (FV_E_TIMEOUT, FV_E_DEVICE) also consumes it; FV_E_NOTFOUND for an unknown ticket. */
int fv_server_poll(fv_server* srv, uint64_t ticket, float* out, fv_req_stats* st);

/* Withdraw a request.  FV_OK: it was still queued (not yet admitted to a launch), or it had
 * finished and was not yet polled; it is removed with its staging and result, the ticket is
 * consumed and is never reported by fv_server_next_done.  FV_PENDING: it is already in a
 * launch, which cannot be stopped; it finishes and is polled as usual.  FV_E_NOTFOUND for an
 * unknown or consumed ticket.  A device frame (fv_server_submit_device) is no longer read once
 * FV_OK is returned.  Thread-safe. */
int fv_server_cancel(fv_server* srv, uint64_t ticket);

/* Wait up to timeout_ms (< 0: forever) for any request to finish and return its ticket
 * (each finished ticket is reported once).  FV_PENDING on timeout. */
int fv_server_next_done(fv_server* srv, double timeout_ms, uint64_t* ticket);

/* Aggregate counters and latency percentiles since creation (or the last reset). */
int fv_server_get_stats(fv_server* srv, fv_server_stats* st, int reset);

/* Graph captures and replays of libfv's launch sequences since the process started, over all
 * devices and streams (monitoring: a capture instantiates a new executable graph, which costs
 * far more than a replay).  Batches on one stream share two graphs (one per half of the
 * double-buffered table staging, used by alternate calls) while they fit its capacities
 * (frames, chunks, rows; doubled when exceeded); single frames are keyed by their size. */
int fv_graph_counters(int64_t* captures, int64_t* replays);

/* Static description of a status code. */
const char* fv_strerror(int code);

/* The last HIP error code seen by the calling thread inside libfv (0 if none). */
int fv_last_device_error(void);

/*
 * Release what the library caches for one (device, stream) pair: device scratch (partial
 * statistics, normalisers, staging), pinned host staging and captured graphs, all created on
 * first use of that stream and otherwise kept for the life of the process.  Call it before
 * destroying a stream that was passed to fv_encode* / fv_em_step; it waits for the stream,
 * and no call on that stream may be in flight or start concurrently.  A pair never used is a
 * no-op; later calls on the stream allocate again.  Servers release their own streams in
 * fv_server_destroy.  Errors: FV_E_DEVICE (the stream, a free, or the device failed).
 */
int fv_stream_release(int device, void* hip_stream);

#ifdef __cplusplus
}
#endif

#endif /* FV_H_ */
