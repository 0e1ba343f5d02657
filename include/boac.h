/*
 * boac.h — C ABI of libboac, the MI355X (gfx950) library that evaluates BOAC candidate attenuation
 * maps: rasterise the Legendre head model, build the attenuated Radon projector, run MLEM, score the
 * reconstruction with the Poisson negative log-likelihood, and differentiate that score.
 *
 * Paper: "A Bayesian Optimization Approach for Attenuation Correction in SPECT Brain Imaging"
 * (Koutsantonis et al.). Eq. (1) attenuated Radon transform; Eq. (2) S = A^mu F; Eq. (3) Legendre
 * head outline; Eq. (4) piecewise attenuation map; Eq. (5) Poisson log-likelihood; BOAC steps 2-3
 * (per-candidate system matrix, fixed number of MLEM iterations, goodness of fit).
 *
 * Discretisation (the paper leaves it open; these are the library's conventions):
 *   image n x n, pixel (i, l) centre ((l - (n-1)/2) dx, (i - (n-1)/2) dx), arrays [i][l] row-major;
 *   angle a: phi_a = 2 pi a / n_angles over 360 deg; bin b offset s_b = (b - (n_bins-1)/2) n dx / n_bins;
 *   ray sample k at t_k = (k - (n_samples-1)/2) dx, point s_b (cos, sin) + t_k (-sin, cos); photons
 *   travel toward +t (detector at k = n_samples-1);
 *   images are read at sample points by bilinear interpolation, zero outside the grid (matrix W);
 *   L_abk = dx (m_abk / 2 + sum_{k'>k} m_abk'), m = W mu;  att = exp(-L);
 *   (A^mu f)_ab = dx sum_k att_abk (W f)_abk;  the backprojector is its exact transpose;
 *   R(theta) = sum_{k=0}^{5} c_k P_k(cos theta); partial-volume fractions from 4 x 4 sub-samples with
 *   a C^1 smoothstep edge of width dx/4; mu = mu_b fb + mu_c (fo - fb);
 *   MLEM: F^0 = 1, r = S / (A F) where A F > 0 else 0, F <- F * (A^T r) / s with s = A^T 1;
 *   objective J = sum_i [y_i - S_i ln y_i + ln Gamma(S_i + 1)] at y = A F^K, evaluated as
 *   sum_i [y_i - S_i - S_i ln(y_i / S_i)] (FP32, compensated) + sum_i [ln Gamma(S_i + 1) - S_i ln S_i + S_i]
 *   (FP64), both over S_i > 0 (bins with S_i = 0 add y_i), so that J keeps its precision at high counts.
 *
 * Conventions for every entry point:
 *   - Pointers named d_* are caller-owned DEVICE buffers (e.g. a contiguous float32 torch tensor's
 *     data_ptr()), 16-byte aligned, on the context's device. The library never frees or keeps them.
 *     Pointers named h_* are host memory read during the call only.
 *   - Calls are asynchronous on `stream` (a hipStream_t; NULL = the device's null stream). Scratch
 *     (attenuation tensors, iterates, partial sums) lives in the context and grows on demand; calls on
 *     one context must be serialised by the caller (one stream at a time).
 *   - Arguments are validated before any launch: geometry sizes >= 2, n <= 1024, n_bins <= 4096,
 *     n_bins <= 2 n, n_samples <= 1024, pixel_cm > 0 and finite, 1 <= C <= 2^20, n_iter >= 0, finite candidates,
 *     non-null and 16-byte-aligned pointers where required. Nothing aborts or throws across the ABI.
 *   - On failure the return value is non-zero and boac_last_error() holds a message (thread-local).
 *     HIP failures map to BOAC_EDEVICE with the HIP error text.
 *   - The reconstruction's GPU arithmetic is FP32 (the likelihood's measurement-only constant is FP64;
 *     the surrogate's kernels are FP64); ray sums, angle sums, scans and the likelihood are accumulated
 *     with compensated (error-free transformation) summation.
 *   - With an even n_angles, ray (a, b) and ray (a + n_angles/2, n_bins-1-b) share their samples in
 *     reverse order, and under the half-self rule their attenuations multiply to exp(-T), T the ray's
 *     total. Where the backprojection runs on its column-group kernel, the library then stores the
 *     attenuation of the first n_angles/2 angles plus exp(-T) per ray and derives the rest ("opposed-
 *     ray pairing"). Results equal those of holding every angle up to FP32 rounding for optical path
 *     lengths below ~87 (attenuations above the smallest normal float). Setting the environment
 *     variable BOAC_OPPOSED_RAYS=0 holds every angle.
 */
#ifndef BOAC_H
#define BOAC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BOAC_OK = 0,
    BOAC_EINVAL = 1,   /* null / misaligned pointer, bad count, non-finite parameter */
    BOAC_ESHAPE = 2,   /* geometry out of the supported range */
    BOAC_ENOMEM = 3,   /* device scratch allocation failed */
    BOAC_EDEVICE = 4,  /* a HIP call failed (message in boac_last_error) */
    BOAC_ETIMEOUT = 5, /* a bounded device wait expired (persistent batch execution) */
    BOAC_ENOTSUP = 6   /* device is not gfx950 / feature not built */
} boac_status;

/* Slice geometry. n x n image of square pixels pixel_cm wide; n_angles projections over 360 deg;
 * n_bins detector bins; n_samples samples per ray at spacing pixel_cm. */
typedef struct {
    int32_t n;
    int32_t n_angles;
    int32_t n_bins;
    int32_t n_samples;
    float pixel_cm;
} boac_geom;

/* One candidate head model (Eqs. 3-4): Legendre coefficients c_0..c_5 of R(cos theta) in cm, brain
 * and cranium attenuation coefficients in 1/cm. 32 bytes, stored as 8 consecutive floats. */
typedef struct {
    float c[6];
    float mu_b;
    float mu_c;
} boac_cand;

/* Per-candidate status bits written by boac_objective / boac_objective_grad / boac_evaluate_batch. */
#define BOAC_STATUS_ZERO_PROJECTION 1u /* some y_i <= 0 with S_i > 0: J = +inf */
#define BOAC_STATUS_NONFINITE 2u       /* J or a gradient entry is not finite */
#define BOAC_STATUS_NEGATIVE_RADIUS 4u /* R(theta) < 0 at some sub-sample (informational) */
#define BOAC_STATUS_NEGATIVE_COUNTS 8u /* the measured sinogram has S_i < 0 somewhere */

typedef struct boac_ctx boac_ctx;

/* Library version, (major << 16) | minor. */
int32_t boac_version(void);

/* Create a context on HIP device `device` (must be gfx950). `tune_cache_path` names a JSON file of
 * launch plans written by the autotuner (NULL: the library's defaults). *out receives the handle. */
boac_status boac_ctx_create(int32_t device, const char *tune_cache_path, boac_ctx **out);

/* Release the context and its device scratch. Waits for the context's outstanding work. NULL is a
 * no-op. */
void boac_ctx_destroy(boac_ctx *ctx);

/* Message for the calling thread's last non-OK return (static storage; "" if none). */
const char *boac_last_error(void);

/* Eqs. (3)-(4): attenuation maps of C candidates.
 * d_cand [C] candidates; delta_r_cm: cranium thickness dR (> 0); d_mu out [C][n][n] float, 1/cm. */
boac_status boac_rasterize_mu(boac_ctx *ctx, const boac_geom *geom, const boac_cand *d_cand, int32_t C,
                              float delta_r_cm, float *d_mu, void *stream);

/* Eqs. (1)-(2): y_c = A^{mu_c} f_c for C (attenuation map, image) pairs.
 * d_mu [C][n][n], d_img [C][n][n] in; d_sino [C][n_angles][n_bins] out. */
boac_status boac_project(boac_ctx *ctx, const boac_geom *geom, const float *d_mu, const float *d_img,
                         int32_t C, float *d_sino, void *stream);

/* Exact transpose of boac_project: x_c = (A^{mu_c})^T z_c.
 * d_mu [C][n][n], d_sino [C][n_angles][n_bins] in; d_img [C][n][n] out. */
boac_status boac_backproject(boac_ctx *ctx, const boac_geom *geom, const float *d_mu, const float *d_sino,
                             int32_t C, float *d_img, void *stream);

/* MLEM (BOAC step 3) for C attenuation maps against ONE measured sinogram.
 * d_mu [C][n][n]; d_meas [n_angles][n_bins] counts as float (>= 0); n_iter >= 0 iterations;
 * d_img_inout [C][n][n]: starting image in (pass ones for the standard start), F^K out. */
boac_status boac_mlem(boac_ctx *ctx, const boac_geom *geom, const float *d_mu, const float *d_meas,
                      int32_t C, int32_t n_iter, float *d_img_inout, void *stream);

/* Full candidate evaluation (BOAC steps 2-3): mu(theta) -> att -> n_iter MLEM iterations from F^0 = 1
 * -> J = -ln P(S | F^K, A^mu) (Eq. 5, negated).
 * d_obj [C] out; d_img_out [C][n][n] (F^K) or NULL; d_status [C] uint32 bits or NULL. */
boac_status boac_objective(boac_ctx *ctx, const boac_geom *geom, const float *d_meas, const boac_cand *d_cand,
                           int32_t C, float delta_r_cm, int32_t n_iter, float *d_obj, float *d_img_out,
                           uint32_t *d_status, void *stream);

/* boac_objective for callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc). Same arguments, results and validation as
 * boac_objective; every scratch buffer and table is carved from a fixed device array of
 * BOAC_NOALLOC_SCRATCH_BYTES that the library holds per device until the process ends, so the call makes
 * no hipMalloc / hipFree and allocates nothing on the device (the tables are copied in with
 * hipMemcpyAsync on `stream` from host copies the context keeps). Candidates are evaluated in chunks
 * that fit the array; BOAC_ENOMEM when even one candidate of the geometry does not fit (at 128 x 128,
 * 128 angles, about 4.6 MB per candidate). Every call on one device shares that device's array and
 * leaves its contents behind: calls that overlap on one device (other streams, other contexts, other
 * threads) race and must be serialised by the caller. */
#define BOAC_NOALLOC_SCRATCH_BYTES (64u << 20)
boac_status boac_objective_noalloc(boac_ctx *ctx, const boac_geom *geom, const float *d_meas,
                                   const boac_cand *d_cand, int32_t C, float delta_r_cm, int32_t n_iter,
                                   float *d_obj, float *d_img_out, uint32_t *d_status, void *stream);

/* Eq. (6) with the inner problem solved by the fixed number of MLEM iterations of BOAC step 3: the
 * objective and its exact gradient dJ/d(c_0..c_5, mu_b, mu_c) through the unrolled MLEM iterations
 * (reverse mode; the MLEM state is checkpointed every ckpt_every iterations and recomputed between
 * checkpoints; 1 <= ckpt_every, values above n_iter mean "only F^0").
 * d_obj [C], d_grad [C][8] out (order c_0..c_5, mu_b, mu_c); d_status [C] or NULL. */
boac_status boac_objective_grad(boac_ctx *ctx, const boac_geom *geom, const float *d_meas,
                                const boac_cand *d_cand, int32_t C, float delta_r_cm, int32_t n_iter,
                                int32_t ckpt_every, float *d_obj, float *d_grad, uint32_t *d_status,
                                void *stream);

/* Gradient variants of boac_objective_grad_ex. */
#define BOAC_GRAD_UNROLLED 0 /* exact derivative through the n_iter unrolled MLEM iterations */
#define BOAC_GRAD_ENVELOPE 1 /* derivative with the reconstruction F^K held fixed */

/* Objective and a gradient that also covers the cranium thickness dR (the last of 9 components).
 * grad_mode BOAC_GRAD_UNROLLED: the exact derivative, as boac_objective_grad (ckpt_every as there).
 * grad_mode BOAC_GRAD_ENVELOPE: the derivative of the joint objective of Eq. (6), -ln P(S | F, A^mu(theta)),
 *   in theta at F = F^K(theta), with F^K treated as a constant: the envelope-theorem gradient, exact when
 *   F^K maximises the likelihood for this attenuation map, an approximation of the unrolled gradient after
 *   finitely many iterations. It costs one projection adjoint after the objective (ckpt_every is
 *   validated but unused).
 * d_obj [C] out; d_grad [C][9] out (order c_0..c_5, mu_b, mu_c, dR); d_status [C] or NULL. Any other
 * grad_mode is BOAC_EINVAL. */
boac_status boac_objective_grad_ex(boac_ctx *ctx, const boac_geom *geom, const float *d_meas,
                                   const boac_cand *d_cand, int32_t C, float delta_r_cm, int32_t n_iter,
                                   int32_t ckpt_every, int32_t grad_mode, float *d_obj, float *d_grad,
                                   uint32_t *d_status, void *stream);

/* One slice of an uneven batch: its geometry, measured sinogram and candidates, and where results go
 * (all device pointers; d_grad NULL = objective only; d_status may be NULL). */
typedef struct {
    boac_geom geom;
    const float *d_meas;     /* [n_angles][n_bins] */
    const boac_cand *d_cand; /* [C] */
    int32_t C;
    float *d_obj;            /* [C] */
    float *d_grad;           /* [C][8] or NULL */
    uint32_t *d_status;      /* [C] or NULL */
} boac_slice;

/* Batched evaluation of many slices of uneven sizes (and their candidates) with one launch per phase
 * covering every slice; the launch sequence is captured once into a HIP graph per batch shape and
 * replayed on later calls with the same shape (same pointers, sizes, n_iter, ckpt_every, delta_r_cm,
 * stream, batch mode and the BOAC_BATCH_LANES / BOAC_BATCH_SPLIT / BOAC_PERSIST_LANES and plan-switch
 * environment settings). h_slices is host memory [n_slices]. Slices needing a gradient use ckpt_every
 * as in boac_objective_grad. The batch's scratch is the lanes' own, apart from the eager entry points';
 * calls on one context still must not overlap. */
boac_status boac_evaluate_batch(boac_ctx *ctx, const boac_slice *h_slices, int32_t n_slices, float delta_r_cm,
                                int32_t n_iter, int32_t ckpt_every, void *stream);

/* Execution of boac_evaluate_batch (BOAC step 3 for many candidate sets at once).
 * BOAC_BATCH_LANES (the default): the slices run on concurrent stream lanes and the launch sequence is
 *   captured into a HIP graph per batch shape.
 * BOAC_BATCH_PERSISTENT: the batch's launches are recorded as tasks and run by ONE persistent launch of
 *   one 1024-thread workgroup per CU that takes work items from a queue in device memory; each task waits
 *   for its predecessor on the same lane through completion counters (release / acquire at device scope).
 *   A wait is bounded: after spin_limit polls (spin_limit <= 0: 2^26) the executor stops every workgroup
 *   and the call returns BOAC_ETIMEOUT with incomplete results. In this mode boac_evaluate_batch waits for
 *   the launch before returning. Batches whose plans the executor cannot run (a backprojection outside the
 *   column-group gather, more than four candidates per gather workgroup) return BOAC_ENOTSUP.
 * The mode stays set on the context. */
#define BOAC_BATCH_LANES 0
#define BOAC_BATCH_PERSISTENT 1
boac_status boac_ctx_set_batch_mode(boac_ctx *ctx, int32_t mode, int64_t spin_limit);

/* ---- Surrogate model of the BOAC outer loop (Eqs. 7-10) ----
 * The negative log-likelihood J of a candidate is modelled as a Gaussian process (Eq. 7) over unit-box
 * coordinates u (the search box mapped affinely onto [0,1]^d) with the RBF kernel of Eq. (8) read as
 * k(u, u') = amp exp(-|u - u'|^2 / (2 length^2)) (the printed names of amplitude and length-scale are
 * swapped). Targets are standardised, z = (J - m0) / s (sample mean; sample standard deviation, 1 if
 * it is 0), amp = 1 in those units, and a nugget `noise` is added to the diagonal. Expected improvement
 * (Eqs. 9-10) is taken for minimisation: gamma = (J_best - mu - xi) / sigma. FP64 throughout. */
typedef struct {
    int32_t n, d;   /* observations, input dimension */
    double length;  /* selected RBF length-scale (unit-box units) */
    double amp;     /* kernel amplitude (1) */
    double noise;   /* nugget */
    double m0, s;   /* target standardisation */
    double lml;     /* log marginal likelihood of the final fit (all n observations) */
} boac_gp_info;

/* Host-only (no device work, no context): fit the surrogate to n observations.
 * h_u [n][d] unit-box inputs, h_y [n] objective values; h_lengths [n_lengths] candidate length-scales,
 * the selected one maximises the log marginal likelihood (first on ties) over the n_select observations
 * of smallest y (ties by index; n_select <= 0 or >= n: all); the final factor uses all n.
 * Outputs: h_linv [n][n] = L^-1 for K = L L^T (row-major, upper triangle zero), h_alpha [n] = K^-1 z,
 * *info. 1 <= n <= 8192, 1 <= d <= 64, noise >= 0. BOAC_EINVAL if no grid length gives a positive
 * definite covariance (raise noise). */
boac_status boac_gp_fit(const double *h_u, const double *h_y, int32_t n, int32_t d, const double *h_lengths,
                        int32_t n_lengths, int32_t n_select, double noise, double *h_linv, double *h_alpha,
                        boac_gp_info *info);

/* Device: posterior mean, standard deviation (of J, not z) and expected improvement at M queries.
 * *info as returned by boac_gp_fit; d_u [n][d], d_linv [n][n], d_alpha [n]: device copies of the fit;
 * d_q [M][d] queries in unit-box coordinates; best = J_best; xi >= 0 exploration margin.
 * d_mu [M], d_sigma [M] out or NULL; d_ei [M] out. 1 <= M <= 2^20. Scratch ((n rounded up to 64) + n/64)
 * x M doubles lives in the context. Asynchronous on stream. */
boac_status boac_gp_ei(boac_ctx *ctx, const boac_gp_info *info, const double *d_u, const double *d_linv,
                       const double *d_alpha, const double *d_q, int32_t M, double best, double xi, double *d_mu,
                       double *d_sigma, double *d_ei, void *stream);

/* Device: the local stage of the acquisition search (Bayesian Optimization, step 5: the chaotic search,
 * read as in the host search of the Python package), n_local rounds with no host round trip. The
 * chains are split evenly over the centres, per = P / n_centres chains each (the first per * n_centres
 * chains are used). Round t (r_0 = radius0, r_{t+1} = r_t * shrink):
 *   U[c * per + k] = clip(C[c] + r_t * (2 z[c * per + k] - 1), 0, 1)   (FP64, in that operation order)
 *   v = EI at U (as boac_gp_ei); centre c moves to its first chain of largest v when that v exceeds
 *   centre_ei[c]; then every chain steps z <- 4 z (1 - z).
 * d_z [P][d] chains in (0, 1), updated in place; d_centres [n_centres][d] and d_centre_ei [n_centres]
 * updated in place; d_pts [n_local][per * n_centres][d] and d_vals [n_local][per * n_centres] receive
 * every round's points and EI values. d = info->d; 1 <= n_centres <= P, 0 <= n_local <= 4096,
 * per * n_centres <= 2^20, radius0 and shrink finite and >= 0. EI values are taken to be finite (NaN
 * never wins a comparison). Scratch as boac_gp_ei. Asynchronous on stream. */
boac_status boac_gp_chaos_local(boac_ctx *ctx, const boac_gp_info *info, const double *d_u, const double *d_linv,
                                const double *d_alpha, double best, double xi, double *d_z, int32_t P,
                                double *d_centres, double *d_centre_ei, int32_t n_centres, double radius0,
                                double shrink, int32_t n_local, double *d_pts, double *d_vals, void *stream);

/* Device, synchronous: the whole acquisition search (Bayesian Optimization, step 5, read as above) for up
 * to q proposals. The chains start at d_z0 [P][d] (not modified). Global stage: n_global rounds whose
 * points are the chains themselves, then z <- 4 z (1 - z); their EI in one launch. Each round keeps a
 * pool of its min(M, per_step) best points (larger EI first, lower index on ties; M the round's
 * points). Centres: the greedy choice (below) over the global pools of min(max(centres, q), P) points,
 * no exclusion from earlier points; then the local stage of boac_gp_chaos_local with radius0, shrink,
 * n_local, the chains as left by the global stage, and P / (number of centres) chains per centre, its
 * rounds pooled the same way. Proposals: the greedy choice over all pools (global rounds first, in
 * round order) of up to q points, each at least `exclusion` from the d_taken [T][d] rows.
 * Greedy choice: repeatedly the pool entry of largest EI (lowest pool position on ties) among those
 * left, each entry nearer than `exclusion` (Euclidean, unit box) to a chosen one or to a taken row
 * dropped. d_props [q][d] receives the proposals in choice order; *h_count their number (< q when the
 * pool runs out), *h_max the largest EI of all pools (= of all points evaluated), *h_queries the number
 * of EI evaluations. 1 <= P <= 8192, 1 <= n_global <= 4096, 0 <= n_local <= 4096, n_global * P <= 2^20,
 * min(P, per_step) * (n_global + n_local) <= 32768; centres, q, per_step >= 1; radius0, shrink,
 * exclusion finite and >= 0; d_taken may be NULL when T = 0. EI values are taken to be finite.
 * Scratch lives in the context. The call waits for the stream (twice: the number of centres fixes the
 * local stage's launches, and the counts are returned on the host). */
boac_status boac_gp_chaos_search(boac_ctx *ctx, const boac_gp_info *info, const double *d_u, const double *d_linv,
                                 const double *d_alpha, double best, double xi, const double *d_z0, int32_t P,
                                 int32_t n_global, int32_t n_local, int32_t centres, int32_t q, double radius0,
                                 double shrink, double exclusion, int32_t per_step, const double *d_taken,
                                 int32_t T, double *d_props, int32_t *h_count, double *h_max, int64_t *h_queries,
                                 void *stream);

/* Kernel-time instrumentation: when enabled, every launch is bracketed by HIP events on its stream
 * and its duration is accumulated per kernel kind after the caller synchronises. */
typedef enum {
    BOAC_K_RASTER = 0,
    BOAC_K_ATT = 1,
    BOAC_K_FWD = 2,
    BOAC_K_BACK = 3,
    BOAC_K_REDUCE = 4,
    BOAC_K_ADJ_RAY = 5,
    BOAC_K_ADJ_PIX = 6,
    BOAC_K_OTHER = 7,
    BOAC_K_GP = 8, /* surrogate acquisition (boac_gp_ei) */
    BOAC_K_COUNT = 9
} boac_kernel_kind;

boac_status boac_ctx_set_profiling(boac_ctx *ctx, int32_t enable);
/* Synchronises the pending events and returns, for `kind`, the number of timed launches, their total
 * milliseconds and the sum of their algorithmic HBM bytes (the library's per-launch model). */
boac_status boac_ctx_kernel_stats(boac_ctx *ctx, int32_t kind, int64_t *count, double *total_ms,
                                  double *total_bytes);
boac_status boac_ctx_reset_stats(boac_ctx *ctx);

/* Graph cache of boac_evaluate_batch: the number of graphs held, the captures and replays so far, and
 * the scratch generation (bumped whenever a scratch buffer is reallocated; a graph captured under an
 * older generation is destroyed, never replayed). Any out pointer may be NULL. */
boac_status boac_ctx_graph_stats(boac_ctx *ctx, int64_t *graphs, int64_t *captures, int64_t *replays,
                                 int64_t *scratch_generation);

#ifdef __cplusplus
}
#endif

#endif /* BOAC_H */
