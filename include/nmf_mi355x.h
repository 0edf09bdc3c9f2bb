/*
 * nmf_mi355x.h -- C ABI of the MI355X (gfx950) weighted multiplicative-update
 * NMF library: PSF-basis construction from a reference library, projection
 * of science frames onto the basis (target modelling) and model-PSF
 * subtraction, after arXiv:2309.04623 ("NMF-based GPU accelerated
 * coronagraphy pipeline").
 *
 * Notation.  The paper factorises its data X ~ W H under weights V (Eq. 1-2).
 * This library names the data V, the weights M:
 *     V  : n x p   reference library, one image per row          (float32)
 *     M  : n x p   per-pixel weight >= 0, 0 = missing / masked   (float32)
 *     W  : n x k   coefficients                                  (float32)
 *     H  : k x p   basis components                              (float32)
 * All matrices are row-major with the last index fastest and tightly
 * packed (leading dimension = number of columns).
 *
 * Pointers.  Every array argument is a DEVICE pointer on the handle's device
 * unless its comment says [host].  The caller allocates and owns every input
 * and output; the library never frees them.  Inputs are read-only.  Outputs
 * may not alias inputs, except W_init == W_out, H_init == H_out and
 * C_init == C_out (in-place update).
 *
 * Streams.  ``stream`` is a hipStream_t passed as void* (NULL = the default
 * stream).  All work is enqueued on it.  Unless NMF_F_ASYNC is set, calls
 * synchronise the stream before returning so that data checks and the
 * report are valid on return.
 *
 * Errors.  0 = success, > 0 = warning (outputs valid), < 0 = error (outputs
 * unspecified).  Argument and shape checks run on the host before anything
 * is enqueued.  nmf_last_error() returns a thread-local description of the
 * last failure.  No C++ exception crosses this interface.
 *
 * Threading.  A handle owns its device workspace and is not thread-safe; use
 * one handle per host thread.
 */
#ifndef NMF_MI355X_H
#define NMF_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nmf_handle_s* nmf_handle;

enum nmf_status {
  NMF_OK = 0,
  NMF_ERR_ARG = -1,          /* null pointer, bad value, forbidden aliasing   */
  NMF_ERR_SHAPE = -2,        /* non-positive or inconsistent dimensions       */
  NMF_ERR_NONFINITE = -3,    /* NaN/Inf data under positive weight           */
  NMF_ERR_NEGATIVE = -4,     /* negative data under positive weight, or a
                                negative / non-finite weight                 */
  NMF_ERR_DIVERGED = -5,     /* objective became non-finite                  */
  NMF_ERR_HIP = -6,          /* HIP runtime error (text in nmf_last_error)   */
  NMF_ERR_NOMEM = -7,        /* device workspace allocation failed           */
  NMF_ERR_UNSUPPORTED = -8,  /* valid request outside what this build runs   */
  NMF_WARN_NONMONOTONE = 1,  /* objective rose beyond rounding slack         */
  NMF_WARN_MAXITER = 2       /* tolerance set but not met by max_iter        */
};

enum nmf_precision {
  NMF_PREC_FP32 = 0,   /* FP32 operands on FP32 MFMA, FP32 accumulation     */
  NMF_PREC_BF16X3 = 1  /* split precision: x = x_hi + x_lo (bf16 each, RNE);
                          a*b ~ a_hi b_hi + a_hi b_lo + a_lo b_hi on bf16 MFMA,
                          FP32 accumulation                                 */
};

enum nmf_flags {
  NMF_F_VALIDATE_DATA = 1,   /* check data/weights, return NMF_ERR_* on bad */
  NMF_F_CLIP_NEGATIVE = 2,   /* negative data under weight: treat as masked */
  NMF_F_NORMALIZE_H = 4,     /* unit-L2 basis rows after the build          */
  NMF_F_BINARY_WEIGHTS = 8,  /* weights are a mask: every positive weight
                                counts as 1 (every call); the basis build and
                                the direct projection keep the staged
                                weights as one bit per element instead of an
                                FP32 copy                                    */
  NMF_F_MASKED_GRAM = 16,    /* projection through per-frame Gram matrices  */
  NMF_F_WARM_START = 32,     /* C_init is a warm start (e.g. from
                                nmf_warmstart_infer): masked-Gram projection
                                keeps it per frame only if its objective is
                                not above the seeded cold start's, else it
                                starts that frame cold (the fallback)        */
  NMF_F_ASYNC = 64,          /* do not synchronise; report filled later     */
  NMF_F_AUTOTUNE = 128       /* time candidate launch shapes of the fused
                                passes on first use of a shape and cache the
                                fastest in the handle (a different split
                                changes the summation order, so results may
                                differ in the last bits from the default);
                                for the masked-Gram projection, the depth of
                                its row gathers (same results), timed on the
                                call's own inputs (the call synchronises)  */
};

/* Iteration parameters.  Fill with nmf_params_default() first. */
typedef struct {
  uint32_t struct_size;  /* = sizeof(nmf_params)                              */
  int32_t k;             /* number of components, 1 <= k <= min(n, p); the
                            fused passes take k <= 224, the masked-Gram
                            projection k <= 200 (else NMF_ERR_UNSUPPORTED) */
  int32_t max_iter;      /* iterations of Eq. 3 (fixed count when tol == 0)   */
  int32_t check_every;   /* stop-rule test cadence c for tol (0 = never)      */
  double tol;            /* stop rule, on when tol > 0 and check_every > 0:
                            basis build: (J[t-c] - J[t]) / J[t-c] < tol;
                            masked-Gram projection: per frame, the model
                            change since the last test, relative (below) */
  uint64_t seed;         /* seed of the counter-based U(0,1) init             */
  int32_t precision;     /* enum nmf_precision                                */
  int32_t flags;         /* OR of enum nmf_flags                              */
  float floor_eps;       /* non-negativity floor applied after each update    */
  int32_t split;         /* row chunks of the split half-step; 0 = auto      */
  int32_t waves;         /* waves per workgroup of the fused passes (1, 2, 4;
                            k <= 64 only: from k = 65 on a workgroup of four
                            waves owns four column tiles); 0 = auto          */
  int32_t pipeline;      /* load pipelining of the fused passes: 1 = operands
                            per tile, 2 = operands and data one tile ahead,
                            3 = operands one and data two tiles ahead
                            (2 and 3 for k <= 64); 0 = auto                   */
} nmf_params;

/* Filled by the calls that iterate.  [host] */
typedef struct {
  uint32_t struct_size;  /* = sizeof(nmf_report)                              */
  int32_t iters_run;     /* iterations performed                              */
  int32_t status_flags;  /* warnings raised (NMF_WARN_* bit set as 1 << w)    */
  double objective;      /* final Eq. 2 cost, accumulated in FP64 on device   */
  double objective_rel;  /* objective / sum(M * V^2)                          */
  float elapsed_ms;      /* device time of the call's enqueued work           */
} nmf_report;

/* ---- handle ------------------------------------------------------------ */

/* Create a handle bound to HIP device ``hip_device``. */
int nmf_create(int hip_device, nmf_handle* out);
/* Release the handle and its device workspace.  NULL is accepted. */
int nmf_destroy(nmf_handle h);
/* Static text for a status code. */
const char* nmf_status_string(int status);
/* Thread-local text of the last error raised by this thread. */
const char* nmf_last_error(void);
/* Default parameters: floor 1e-30, FP32, 200 iterations, seed 0. [host] */
void nmf_params_default(nmf_params* prm);
/* Bytes of device workspace currently held by the handle. */
size_t nmf_workspace_bytes(nmf_handle h);

/* ---- initialisation ------------------------------------------------------
 * Random start of W and H (Sec. 2: W and H are initialised randomly).
 * Fills out[r * cols + c] with the open-interval U(0,1) value of the
 * counter-based SplitMix64 stream:
 *   key = mix(seed + (matrix_id + 1) * G),  u = mix(key + (r*cols + c + 1) * G)
 *   value = ((u >> 41) + 0.5) * 2^-23,    G = 0x9E3779B97F4A7C15,
 * mix = the SplitMix64 output finaliser (Steele, Lea & Flood 2014).
 * matrix_id: 0 = W, 1 = H, 2 = projection coefficients.  out: rows x cols.  */
int nmf_init_uniform(nmf_handle h, uint64_t seed, int32_t matrix_id, int64_t rows,
                     int64_t cols, float* out, void* stream);

/* ---- objective ------------------------------------------------------------
 * Eq. 2 weighted Frobenius cost  J = sum_{i,j} M_ij (V_ij - (W H)_ij)^2,
 * with V_ij taken as 0 wherever M_ij == 0 (masked = missing, Sec. 4.1).
 * Products in FP32 (or bf16x3), residual squares summed in FP64 in a fixed
 * order (bitwise reproducible).  J_out: [host] one double.                 */
int nmf_objective(nmf_handle h, const float* V, const float* M, const float* W,
                  const float* H, int64_t n, int64_t p, int32_t k, int32_t precision,
                  double* J_out, void* stream);

/* ---- basis construction --------------------------------------------------
 * Iterates Eq. 3 (H-rule, then the W-rule with the new H) prm->max_iter
 * times from (W_init, H_init), or from the seeded U(0,1) init when those are
 * NULL.  NMF_F_WARM_START (W_init and H_init required: a warm start of the
 * component initialisation, e.g. a prior basis and the coefficients
 * nmf_warmstart_infer predicts on it for each library image): the supplied
 * start is kept only if its Eq. 2 cost is not above the seeded cold start's
 * (one synchronisation before the first iteration); otherwise the build
 * starts cold, rep->status_flags gets NMF_RS_WARM_FALLBACK and
 * nmf_warm_fallbacks() returns 1.  After each update x := max(x, floor_eps); a zero denominator keeps
 * the factor.  Data under zero weight are ignored whatever their value.
 * Stop rule (Sec. 2: iterate until the change reaches a set value or the
 * cap), on when tol > 0 and check_every = c > 0: J[t] is the Eq. 2 cost of
 * the iterate entering iteration t (known during that iteration's H-rule
 * pass); at t = c, 2c, ... the device tests (J[t-c] - J[t]) / J[t-c] < tol
 * and, when it passes, iteration t is the last one (rep->iters_run = t + 1).
 * The test runs on the device; no host round trip decides it.  Without it
 * by max_iter the call returns NMF_WARN_MAXITER.  With NMF_F_ASYNC and a
 * stop rule, rep->iters_run is -1 (only the device knows it).
 *   V, M            : n x p inputs
 *   W_init, H_init  : nullable n x k and k x p starts
 *   W_out, H_out    : n x k and k x p results
 *   obj_hist        : [host] nullable, max_iter + 1 doubles: J before each
 *                     iteration and after the last one
 *   rep             : [host] nullable report
 * Errors: NMF_ERR_ARG/SHAPE before any work; with NMF_F_VALIDATE_DATA,
 * NMF_ERR_NONFINITE / NMF_ERR_NEGATIVE for bad data under weight;
 * NMF_ERR_DIVERGED if J turns non-finite.                                  */
int nmf_build_basis(nmf_handle h, const float* V, const float* M, int64_t n, int64_t p,
                    const nmf_params* prm, const float* W_init, const float* H_init,
                    float* W_out, float* H_out, double* obj_hist, nmf_report* rep,
                    void* stream);

/* ---- projection (target modelling) ---------------------------------------
 * Sec. 4.1: the basis models each target frame individually.  With H fixed,
 * each frame's coefficient row c_f (1 x k) follows Eq. 3's W-rule:
 *   c_f <- max(c_f o [(m_f o t_f) H^T] / [(m_f o (c_f H)) H^T], floor_eps)
 * for prm->max_iter iterations, from C_init (nullable: seeded U(0,1) with
 * matrix_id 2).  With NMF_F_MASKED_GRAM the denominator is formed as
 * c_f G_f, G_f = H diag(m_f) H^T (same value in exact arithmetic).
 *   H       : k x p basis;  T, M_T : f x p frames and weights
 *   C_out   : f x k coefficients
 *   obj_out : nullable f doubles (device): final per-frame Eq. 2 cost
 * NMF_F_WARM_START (masked-Gram form only, C_init required): per frame, the
 * start with the lower objective of C_init and the seeded cold start is
 * used; rep->status_flags gets bit NMF_RS_WARM_FALLBACK when any frame fell
 * back, and nmf_warm_fallbacks() returns how many did.
 * Per-frame stop rule (masked-Gram form; Sec. 2 leaves the test open), on
 * when tol > 0 and check_every = c > 0: before iteration t + 1, t = c, 2c,
 * ..., a frame stops after t iterations when d G_f d^T <= tol^2 c_f G_f
 * c_f^T, d = c_f - (c_f at the previous test, or the start at t = c), the
 * weighted squared norm of the model change against that of the model.  A
 * kept warm start that has not stopped by max_iter restarts from the cold
 * start with the same cap (it then counts as fallen back).  Iterations per
 * frame: nmf_frame_iters(); rep->iters_run is their maximum; a frame that
 * never met the rule makes the call return NMF_WARN_MAXITER.              */
int nmf_project(nmf_handle h, const float* H, int64_t k, int64_t p, const float* T,
                const float* M_T, int64_t f, const nmf_params* prm, const float* C_init,
                float* C_out, double* obj_out, nmf_report* rep, void* stream);

/* Same iteration for frames stored as CSR rows, always through the masked
 * Gram form: frame i owns entries offsets[i] .. offsets[i+1]-1 of pix (int32
 * pixel index in [0, p)), val (float32 data) and wt (float32 weight; NULL =
 * all ones, as is NMF_F_BINARY_WEIGHTS); pixels absent from a frame carry
 * weight 0.  Pixel indices
 * within a frame must be distinct.  offsets: f + 1 int64 (device) with
 * 0 <= offsets[i] <= offsets[i+1] <= nnz; entries that break this, or a
 * pixel index outside [0, p), are skipped and reported as NMF_ERR_ARG.
 * All frames run in one persistent launch that takes frames from a device
 * work queue, longest first.
 *   frame_ticks : nullable, 2 * f uint64 (device): device clock at which
 *                 each frame was taken from the queue and finished (see
 *                 nmf_device_clock_khz).                                  */
int nmf_project_ragged(nmf_handle h, const float* H, int64_t k, int64_t p, int64_t f,
                       const int64_t* offsets, int64_t nnz, const int32_t* pix,
                       const float* val, const float* wt, const nmf_params* prm,
                       const float* C_init, float* C_out, uint64_t* frame_ticks,
                       nmf_report* rep, void* stream);

/* Bit of nmf_report.status_flags: a warm-started projection fell back to
 * the cold start for at least one frame. */
#define NMF_RS_WARM_FALLBACK (1 << 8)

/* Frames of the last synchronous warm-started projection on h that fell back
 * to the cold start, or 1/0 after a warm-started basis build (-1 if none
 * ran). */
int64_t nmf_warm_fallbacks(nmf_handle h);

/* Iterations each frame ran in the last synchronous masked-Gram projection
 * on h that had a stop rule.  iters_out: [host] room for f int32, or NULL to
 * ask for the count only.  Returns that call's frame count (written unless
 * iters_out is NULL), 0 when the last projection had no stop rule (or none
 * ran), NMF_ERR_ARG when f is smaller than the count. */
int64_t nmf_frame_iters(nmf_handle h, int32_t* iters_out, int64_t f);

/* How many times the persistent launch of the last synchronous masked-Gram
 * projection on h took each frame from its work queue (1 for every frame
 * when the queue is sound; a check of the batched form, Sec. 4.1 target
 * modelling frame by frame).  visits_out: [host] room for f int32, or NULL
 * to ask for the count only.  Returns that call's frame count (written
 * unless visits_out is NULL), 0 when no masked-Gram projection ran on h,
 * NMF_ERR_ARG when f is smaller than the count. */
int64_t nmf_frame_visits(nmf_handle h, int32_t* visits_out, int64_t f);

/* Frequency (kHz) of the device clock used by frame_ticks. */
double nmf_device_clock_khz(nmf_handle h);

/* ---- subtraction -----------------------------------------------------------
 * Sec. 1 and Sec. 4.1: the model PSF c_f H is removed from each frame:
 *   model_out[f, j] = sum_k C[f, k] H[k, j]          (every pixel)
 *   resid_out[f, j] = T[f, j] - s_f * model[f, j]     where M_T[f, j] > 0,
 *                     NaN                              where M_T[f, j] == 0,
 * s_f = scale[f] (NULL: 1).  The sum is accumulated in FP64.
 *   H: k x p; C: f x k; T, M_T: f x p; scale: nullable f; model_out:
 *   nullable f x p; resid_out: f x p.                                      */
int nmf_subtract(nmf_handle h, const float* H, const float* C, const float* T,
                 const float* M_T, int64_t f, int64_t k, int64_t p, const float* scale,
                 float* model_out, float* resid_out, void* stream);

/* ---- reference selection ---------------------------------------------------
 * Sec. 4.1: the target frames are compared with the reference library and
 * the closest frames, by the Euclidean norm (the cost the factorisation
 * minimises), build the basis; Sec. 5.3 finds this the largest SNR gain.
 *   dist[f, n] = sum over pixels j with M_T[f, j] > 0 and M[n, j] > 0 of
 *                (T[f, j] - V[n, j])^2     (data under zero weight ignored)
 * summed in FP32 over 64-pixel chunks and in FP64 across chunks.
 *   idx_out[f, r] (r < n_sel) = the reference of rank r for target f, by
 *   increasing distance, equal distances by increasing reference index.
 *   V, M: n x p library and weights; T, M_T: f x p targets and weights
 *   dist_out: nullable f x n doubles (device); idx_out: f x n_sel int32
 *   (device).  n < 2^31, f <= 65535, 1 <= n_sel <= n.
 * Synchronous.  Errors: NMF_ERR_ARG / NMF_ERR_SHAPE before any work;
 * NMF_ERR_NONFINITE when data under positive weight are not finite.      */
int nmf_closest_frames(nmf_handle h, const float* V, const float* M, int64_t n, int64_t p,
                       const float* T, const float* M_T, int64_t f, int64_t n_sel,
                       double* dist_out, int32_t* idx_out, void* stream);

/* ---- reference selection without allocation ---------------------------------
 * For callers that cannot allocate device memory during the call (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * nmf_closest_frames without the distance output, with every intermediate
 * in a fixed per-device scratch array of 16 MiB that the library holds from
 * the first nmf_create on the device until the process ends.  The call
 * allocates nothing (no hipMalloc / hipFree, no workspace growth).
 *   idx_out: f x n_sel int32 (device), as nmf_closest_frames.
 * Limit: f * n <= 2,097,120 distances, else NMF_ERR_UNSUPPORTED (checked on
 * the host before any work).  All calls on one GPU share that GPU's array,
 * which keeps the last call's contents: calls that overlap on one GPU (other
 * streams, other threads) race and must be serialised by the caller.
 * Synchronous.  Errors as nmf_closest_frames.                              */
int nmf_closest_frames_noalloc(nmf_handle h, const float* V, const float* M, int64_t n,
                               int64_t p, const float* T, const float* M_T, int64_t f,
                               int64_t n_sel, int32_t* idx_out, void* stream);

/* ---- best factor -------------------------------------------------------------
 * Sec. 2 and Sec. 4.1 (best factor finding, after Ren et al. 2018, which
 * the paper cites without restating): the per-frame scale s_f of the model
 * PSF m = c_f H applied before subtraction.  Read here as the s minimising
 * the variance of t - s m over the pixels with M_T > 0 (and region > 0 when
 * a region is given, to keep the circumstellar signal out of the fit):
 *   s_f = cov(t, m) / var(m), clamped to [s_lo, s_hi];
 *   s_f = 1 with fewer than two such pixels or var(m) <= 1e-12 mean(m^2).
 * Moments accumulated in FP64.  Feed scale_out to nmf_subtract.
 *   H: k x p; C: f x k; T, M_T: f x p; region: nullable p; scale_out: f
 *   floats (device).  Synchronous.  Errors: NMF_ERR_ARG (null, s_lo > s_hi). */
int nmf_best_factor(nmf_handle h, const float* H, const float* C, const float* T,
                    const float* M_T, const float* region, int64_t f, int64_t k, int64_t p,
                    float s_lo, float s_hi, float* scale_out, void* stream);

/* ---- component-by-component basis construction ------------------------------
 * The basis-build variant of the package the paper modifies (Sec. 2): stage
 * j = 1..k runs nmf_build_basis with j components from the j - 1 components
 * of stage j - 1 plus one new component, W column j - 1 = U(0,1) of matrix 3
 * at index r * k + j - 1 and H row j - 1 = U(0,1) of matrix 4 at index
 * (j - 1) * p + c (their places in n x k and k x p matrices; the stream of
 * nmf_init_uniform).  prm->max_iter (and the stop rule) apply per stage.
 *   W_out, H_out: n x k and k x p results of the last stage
 *   obj_stages: [host] nullable, k doubles: the Eq. 2 cost after each stage
 *   rep: iters_run = iterations over all stages, objective of the last one
 * Errors and warnings as nmf_build_basis (the first failing stage's).     */
int nmf_build_basis_sequential(nmf_handle h, const float* V, const float* M, int64_t n, int64_t p,
                               const nmf_params* prm, float* W_out, float* H_out,
                               double* obj_stages, nmf_report* rep, void* stream);

/* ---- learned warm start of the projection ---------------------------------
 * Not part of the paper's method: a small network predicts each frame's
 * coefficients so that the Eq. 3 W-rule iteration (target modelling,
 * Sec. 4.1) starts near its limit; cold start stays the fallback.
 *   x = masked-mean-pool(t) / s  (32 x 32 grid over the frame padded with
 *       weight 0 to a multiple of 32 per axis; s = masked mean of t)
 *   a1 = x W1 + b1, h1 = gelu(a1)    1024 -> 512
 *   a2 = h1 W2 + b2, h2 = gelu(a2)   512 -> 512
 *   z = h2 W3 + b3                   512 -> k
 *   c = max(s softplus(z), 1e-6 s)
 * The model state is one device float array: parameters in the order
 * W1 (1024 x 512), b1 (512), W2 (512 x 512), b2 (512), W3 (512 x k), b3 (k),
 * row-major, followed by the two Adam moment arrays of the same length.
 * GEMMs run on bf16 MFMA with FP32 accumulation; precision NMF_PREC_FP32
 * selects the split (bf16x3) products, NMF_PREC_BF16X3 is accepted as the
 * same, any other value rounds operands to bf16 (use 2).                   */
#define NMF_WS_IN 1024
#define NMF_WS_HIDDEN 512
#define NMF_PREC_BF16 2
/* Parameter count of the network for k outputs (the state holds 3x this). */
int64_t nmf_warmstart_param_count(int32_t k);
/* He-normal weights, zero biases and moments from the seeded generator. */
int nmf_warmstart_init(nmf_handle h, float* state, int32_t k, uint64_t seed, void* stream);
/* Pool f dense frames (f x ny*nx) into X_out (f x 1024) and s_out (f). */
int nmf_warmstart_pool(nmf_handle h, const float* T, const float* M_T, int64_t f, int32_t ny,
                       int32_t nx, float* X_out, float* s_out, void* stream);
/* One step on a batch of b rows: forward, loss
 *   L = mean_f (c_f - c*_f) G (c_f - c*_f)^T / (c*_f G c*_f^T),  G = H H^T,
 * backward, and an Adam update (lr > 0; step_index counts from 1).
 * grads_out: nullable parameter-sized gradient; loss_out: [host].        */
int nmf_warmstart_step(nmf_handle h, float* state, const float* X, const float* s,
                       const float* c_star, const float* G, int32_t b, int32_t k,
                       int32_t precision, float lr, int32_t step_index, float* grads_out,
                       double* loss_out, void* stream);
/* Epochs of shuffled minibatches over m rows (X: m x 1024, s: m, c_star:
 * m x k).  loss_hist: [host] nullable, one mean training loss per epoch.  */
int nmf_warmstart_train(nmf_handle h, float* state, const float* X, const float* s,
                        const float* c_star, const float* G, int64_t m, int32_t k,
                        int32_t precision, int32_t epochs, int32_t batch, float lr,
                        uint64_t seed, double* loss_hist, void* stream);
/* Predicted coefficients C_out (f x k) for pooled frames X, s. */
int nmf_warmstart_infer(nmf_handle h, const float* state, const float* X, const float* s,
                        int64_t f, int32_t k, int32_t precision, float* C_out, void* stream);

/* Launch shapes chosen so far by NMF_F_AUTOTUNE: writes up to cap lines of
 * "pass n p k precision: waves pipeline splits time_us" into buf [host]
 * (masked-Gram entries, keyed "gram.*": pipeline = chunks of rows gathered
 * ahead, time of the whole projection).  Returns the number of cached
 * entries.                                                                  */
int nmf_autotune_report(nmf_handle h, char* buf, size_t cap);

/* ---- live kernel timing ----------------------------------------------------
 * Opt-in instrumentation for measurement: while enabled, every kernel the
 * handle launches is bracketed by two HIP events recorded on the call's
 * stream, and the elapsed time is summed per kernel class.  Adds two event
 * records per launch; off by default.                                        */
enum nmf_kernel_class {
  NMF_K_HRULE = 0,      /* fused H-rule half-step over V (also yields J)      */
  NMF_K_WRULE = 1,      /* fused W-rule half-step over V^T (split partials)   */
  NMF_K_WFINISH = 2,    /* W-rule finish: partial sums + update               */
  NMF_K_OBJECTIVE = 3,  /* objective-only pass                                */
  NMF_K_PROJECT = 4,    /* projection iteration kernels                       */
  NMF_K_SUBTRACT = 5,   /* model-PSF subtraction                              */
  NMF_K_OTHER = 6,      /* staging, layouts, reductions, init                 */
  NMF_K_COUNT = 7
};
/* Turn timing on (1) or off (0); turning it on clears the counters. */
int nmf_profile_enable(nmf_handle h, int on);
/* Launch count and summed device milliseconds of one kernel class
 * (waits for the recorded events).  count, total_ms: [host].               */
int nmf_profile_get(nmf_handle h, int32_t kernel_class, int64_t* count, double* total_ms);

#ifdef __cplusplus
}
#endif
#endif /* NMF_MI355X_H */
