/*
 * lba.h -- C ABI of the MI355X (gfx950) Local Bundle Adjustment library (liblba.so).
 *
 * The operation (paper Section III-C "Local Bundle Adjustment", Section IV-E "Local
 * Bundle Adjustment"): refine the poses of a window of local keyframes and the 3-D
 * points they observe by nonlinear least squares on the reprojection residuals, solved
 * iteratively by Levenberg-Marquardt with the points eliminated by the Schur
 * complement (the reduced camera system is factorised, the points back-substituted).
 *
 * Formulation (the library's reading of that passage; every symbol below is fixed):
 *   residual   e = z - pi(T_k X_j): mono (u, v), stereo (u, v, uR) with
 *              pi = (fx x/z + cx, fy y/z + cy, fx x/z + cx - bf/z), X_c = R X + t;
 *   weight     s = |e|^2 / sigma2[octave];  robust cost rho(s) = s for s <= d2, else
 *              2 sqrt(d2 s) - d2 (Huber on s; d2 = huber2_mono / huber2_stereo);
 *   cost       F = sum over active observations of rho(s);
 *   step       (H + lambda I) d = b, H = sum w J^T Om J, b = sum w J^T Om e, w = rho'(s),
 *              Om = I / sigma2, J the Jacobian of pi; poses move on the left,
 *              T <- Exp(dxi) T with the twist ordered (rotation, translation);
 *   damping    lambda0 = tau * max diag(H) at the start of each round; gain ratio
 *              (F - F') / (d^T (lambda d + b)); accept iff > 0 and finite, then
 *              lambda *= max(1/3, 1 - (2 g - 1)^3); otherwise lambda *= nu, nu *= 2;
 *              max_trials consecutive rejections end a round;
 *   schedule   round 1 on all observations (iters_round1 iterations); an observation
 *              is an outlier if s > chi2(type) or its depth <= 0; round 2 on the
 *              inliers (iters_round2 iterations, lambda re-initialised); the returned
 *              flags are recomputed on all observations at the final state.
 *
 * Memory: every array is caller-owned.  Arrays marked DEVICE live in device memory of
 * the context's GPU (e.g. torch tensors); arrays marked HOST are small plan metadata in
 * host memory.  All device work is enqueued on the caller's HIP stream; the solve
 * synchronises that stream a few times to read per-window completion flags (see
 * lba_solve).  No entry point throws; every failure is a status code, and
 * lba_last_error() gives a message.  A context is not thread-safe: use one per thread.
 */
#ifndef LBA_H
#define LBA_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LBA_ABI_VERSION 4

typedef enum {
    LBA_OK = 0,
    LBA_ERR_INVALID_ARGUMENT = -1,   /* bad pointer, size, index, octave, flag, ...      */
    LBA_ERR_OUT_OF_MEMORY = -2,      /* a host allocation of the context failed          */
    LBA_ERR_HIP = -3,                /* a HIP runtime call failed (message has the text) */
    LBA_ERR_WORKSPACE_TOO_SMALL = -4,
    LBA_ERR_UNSUPPORTED = -5         /* a window exceeds the built limits (see below)    */
} lba_status;

typedef enum {
    LBA_PREC_FP64 = 0,   /* everything in FP64 */
    LBA_PREC_MIXED = 1   /* Jacobians, Hessian blocks and the Schur products in FP32; the
                            sums that form the Schur complement in FP64 (FP32 with
                            schur_fp32_accum); residuals, cost, gain ratio, damping, states,
                            the 3x3 point blocks and the reduced-camera-system Cholesky in
                            FP64 */
} lba_precision;

/* Solver options.  lba_default_options() fills the values noted in brackets. */
typedef struct {
    int32_t precision;       /* lba_precision [LBA_PREC_FP64] */
    int32_t iters_round1;    /* LM iterations before the outlier pass [5] */
    int32_t iters_round2;    /* LM iterations after it [10] */
    int32_t max_trials;      /* damped solves per iteration before the round ends [10] */
    int32_t round2_robust;   /* 1: keep the Huber kernel in round 2, 0: plain squares [1] */
    int32_t check_inputs;    /* cost layer: 1 = validate indices/octaves/order on the GPU first
                                [1]; the solver always validates */
    double huber2_mono;      /* Huber threshold on s, monocular [5.991] */
    double huber2_stereo;    /* Huber threshold on s, stereo [7.815] */
    double chi2_mono;        /* outlier threshold on s, monocular [5.991] */
    double chi2_stereo;      /* outlier threshold on s, stereo [7.815] */
    double tau;              /* initial damping factor [1e-5] */
    int32_t points_per_tile; /* 0: per window from lba_tune's table for this problem if it
                                was tuned, else from the total point count (cost layer:
                                tiles of about 448 observations); else fixed */
    int32_t use_graphs;      /* 1: each LM step (five kernels over every window) is captured
                                once into a HIP graph and replayed; kernels are launched one
                                by one while profiling is enabled [1] */
    int32_t trial_log;       /* records per window of the per-trial log kept in the workspace
                                and returned through lba_result.log, 0..4096 [0] */
    int32_t schur_fp32_accum; /* mixed precision only: 1 = sum the Schur complement and the
                                 per-camera terms in FP32 (the literal precision form), 0 = in
                                 FP64 from the FP32 products [0] */
    int32_t pair_cache;      /* 1: the linearisation keeps the pair structure of the Schur
                                complement (which observations of a point pair up on which
                                camera block) in the workspace for the rest of an LM round, so
                                that only the first step of a round forms it; 0: formed at
                                every step.  The results are the same [1] */
} lba_options;

typedef struct {
    double fx, fy, cx, cy;   /* pinhole intrinsics, pixels */
    double bf;               /* stereo baseline times fx (px*m); only read for stereo obs */
} lba_intrinsics;

/*
 * One window, or a batch of windows concatenated end to end (lba_solve_batch).
 * Observation indices are local to their window: obs_kf in [0, window's n_kf),
 * obs_pt in [0, window's n_pt), and within a window obs_pt must be non-decreasing
 * (observations grouped by point).  A point may have at most 64 observations.
 */
typedef struct {
    int32_t n_kf, n_pt, n_obs;   /* totals over the batch */
    int32_t n_levels;            /* entries of sigma2, 1..32 */
    const double *T_cw;          /* DEVICE n_kf x 12, row-major [R | t], world -> camera */
    const uint8_t *fixed;        /* HOST   n_kf, 1 = pose held fixed (decides the size of the
                                    reduced system, hence the launch plan) */
    const double *X_w;           /* DEVICE n_pt x 3 */
    const int32_t *obs_kf;       /* DEVICE n_obs */
    const int32_t *obs_pt;       /* DEVICE n_obs */
    const void *obs_z;           /* DEVICE 3 x n_obs planar: u[n_obs], v[n_obs], uR[n_obs] */
    int32_t obs_z_f32;           /* 0: obs_z is double, 1: float */
    int32_t reserved;
    const uint8_t *obs_type;     /* DEVICE n_obs, 0 mono / 1 stereo */
    const uint8_t *obs_oct;      /* DEVICE n_obs, octave < n_levels */
    const double *sigma2;        /* HOST   n_levels, measurement variance per octave (px^2) */
    lba_intrinsics cam;
} lba_problem;

/* Window boundaries of a batch: HOST arrays of n_windows + 1 offsets into the
 * concatenated keyframe / point / observation arrays (first 0, last the totals). */
typedef struct {
    int32_t n_windows;
    int32_t reserved;
    const int32_t *kf_off;
    const int32_t *pt_off;
    const int32_t *obs_off;
} lba_batch;

/* Per-window statistics row (doubles) written to lba_result.stats when it is not NULL */
enum {
    LBA_STAT_F_INITIAL = 0,   /* round-1 cost at the input state */
    LBA_STAT_F_FINAL = 1,     /* round-2 cost at the returned state */
    LBA_STAT_ITERS_R1 = 2,    /* accepted iterations, round 1 */
    LBA_STAT_ITERS_R2 = 3,    /* accepted iterations, round 2 */
    LBA_STAT_TRIALS = 4,      /* damped solves, both rounds */
    LBA_STAT_LAMBDA = 5,      /* damping at the end */
    LBA_STAT_TERM_R1 = 6,     /* 1 if round 1 ended on max_trials rejections */
    LBA_STAT_TERM_R2 = 7,
    LBA_STAT_N_OUTLIERS = 8,  /* returned flags set */
    LBA_STAT_F_END_R1 = 9,    /* round-1 cost at the end of round 1 */
    LBA_STAT_F_START_R2 = 10, /* round-2 cost at the start of round 2 */
    LBA_STAT_KOPT = 11,       /* optimisable keyframes */
    LBA_STATS_LEN = 12
};

/* One damped solve of the LM loop (a trial), as the per-window decision records it:
 * the round (1, 2), the iteration within the round (accepted steps so far), the trial
 * within the iteration, whether it was accepted, whether the reduced system and every
 * point block factorised, the damping it was solved with, the cost before it, the cost
 * at the trial state and the gain ratio (F_trial and gain are not meaningful when
 * solve_ok is 0). */
typedef struct {
    int32_t round, iter, trial, accepted, solve_ok, reserved;
    double lambda, F, F_trial, gain;
} lba_trial_record;

typedef struct {
    double *T_out;       /* DEVICE n_kf x 12; may alias lba_problem.T_cw */
    double *X_out;       /* DEVICE n_pt x 3;  may alias lba_problem.X_w */
    uint8_t *outlier;    /* DEVICE n_obs, 1 = outlier at the final state */
    double *stats;       /* HOST n_windows x LBA_STATS_LEN, or NULL */
    lba_trial_record *log;   /* HOST n_windows x options.trial_log records, or NULL: window w's
                                first min(trials, trial_log) trials in order, from record
                                w * trial_log on (trials = its LBA_STAT_TRIALS) */
} lba_result;

typedef struct lba_ctx lba_ctx;

int32_t lba_abi_version(void);
const char *lba_status_string(lba_status status);
void lba_default_options(lba_options *opt);

/* Create a context bound to HIP device `device`.  Options are copied. */
lba_status lba_create(const lba_options *opt, int32_t device, lba_ctx **out);
/* Destroy a context (NULL-safe).  Waits for nothing; the caller orders it after its
 * last solve on the stream. */
void lba_destroy(lba_ctx *ctx);
/* Message of the last failure on this context ("" if none). */
const char *lba_last_error(const lba_ctx *ctx);
/* Replace the options of a context. */
lba_status lba_set_options(lba_ctx *ctx, const lba_options *opt);

/* Bytes of DEVICE workspace lba_solve / lba_solve_batch need for this problem
 * (batch NULL: one window).  Limits: per window n_kf <= 128, optimisable keyframes
 * <= 60 (reduced systems of up to 360 unknowns; above 180 unknowns, or whenever one
 * window of a batch is that large, the systems are factorised in a copy in HBM rather than
 * in LDS, and the linearisation makes one pass per 476 camera blocks), at most 64
 * observations per point; beyond them the call returns LBA_ERR_UNSUPPORTED. */
lba_status lba_workspace_size(lba_ctx *ctx, const lba_problem *problem, const lba_batch *batch,
                              size_t *bytes);

/* Solve one window.  `workspace` is DEVICE memory of at least lba_workspace_size bytes,
 * aligned to 256 bytes; `stream` is a hipStream_t (NULL: the null stream).  The stream is
 * synchronised after input validation, about twice per LM round to read completion
 * flags, and at the end; the results are complete when the call returns LBA_OK. */
lba_status lba_solve(lba_ctx *ctx, const lba_problem *problem, lba_result *result,
                     void *workspace, size_t workspace_bytes, void *stream);

/* Solve many independent windows together: every kernel of an LM step covers all of
 * them in one launch, so windows of uneven size share the GPU.  Each window follows the
 * schedule lba_solve gives it alone; the results agree to rounding (the linearisation
 * sums its per-camera terms in no fixed order). */
lba_status lba_solve_batch(lba_ctx *ctx, const lba_problem *problem, const lba_batch *batch,
                           lba_result *result, void *workspace, size_t workspace_bytes,
                           void *stream);

/* ---- stereo-inertial form -------------------------------------------------------------
 * The same solve with inertial residuals between keyframes (Section III-C: in visual-
 * inertial systems the local bundle adjustment adds inertial residuals to the
 * reprojection errors; the paper's runs are stereo-inertial, Section V-A).  Reading: the
 * preintegrated IMU factor of Forster et al. (IEEE T-RO 2017) with a bias random walk.
 *
 *   states     per keyframe the pose T_cw and, in the world frame, the body velocity v,
 *              gyroscope bias bg and accelerometer bias ba (fixed keyframes hold all);
 *              the body pose is R = R_cw^T R_cb, p = R_cw^T (t_cb - t_cw) for the
 *              body-to-camera transform T_cb = [R_cb | t_cb];
 *   residual   of a measurement (dR, dv, dp over dt, integrated with biases bg_bar,
 *              ba_bar, bias Jacobians J_Rg, J_vg, J_va, J_pg, J_pa) from keyframe i to j,
 *              with dbg = bg_i - bg_bar and dba = ba_i - ba_bar:
 *                r_R = Log((dR Exp(J_Rg dbg))^T R_i^T R_j)
 *                r_v = R_i^T (v_j - v_i - g dt) - (dv + J_vg dbg + J_va dba)
 *                r_p = R_i^T (p_j - p_i - v_i dt - g dt^2 / 2) - (dp + J_pg dbg + J_pa dba)
 *                r_bg = bg_j - bg_i,  r_ba = ba_j - ba_i;
 *   cost       r9^T info r9 + info_bg |r_bg|^2 + info_ba |r_ba|^2 (r9 = (r_R, r_v, r_p)),
 *              added to the reprojection cost; no robust kernel;
 *   step       15 unknowns per optimisable keyframe (twist, dv, dbg, dba), lambda on
 *              every diagonal entry, the points eliminated as before; v, bg, ba move
 *              additively.  The outlier pass and the schedule are those of lba_solve.
 * The inertial terms are evaluated in FP64 in both precisions.  Limit: 15 Kopt <= 180
 * (at most 12 optimisable keyframes per window). */
typedef struct {
    int32_t n_edges;          /* measurements over the batch */
    int32_t reserved;
    const int32_t *edge_off;  /* HOST n_windows + 1 (NULL for one window): window w owns the
                                 measurements [edge_off[w], edge_off[w + 1]) */
    const int32_t *edge_i;    /* DEVICE n_edges, window-local keyframe the measurement starts at */
    const int32_t *edge_j;    /* DEVICE n_edges, window-local keyframe it ends at (!= edge_i) */
    const double *dt;         /* DEVICE n_edges, seconds (> 0) */
    const double *dR;         /* DEVICE n_edges x 9, row-major */
    const double *dv, *dp;    /* DEVICE n_edges x 3 */
    const double *J_Rg, *J_vg, *J_va, *J_pg, *J_pa;   /* DEVICE n_edges x 9 each, row-major */
    const double *bg_bar, *ba_bar;                    /* DEVICE n_edges x 3 */
    const double *info;       /* DEVICE n_edges x 81: information of (r_R, r_v, r_p), symmetric */
    const double *info_bg, *info_ba;                  /* DEVICE n_edges */
    const double *v, *bg, *ba;                        /* DEVICE n_kf x 3: initial states */
    double T_cb[12];          /* body -> camera, row-major [R | t] */
    double g[3];              /* gravity in the world frame */
} lba_inertial;

/* Bytes of DEVICE workspace lba_solve_inertial needs (batch NULL: one window). */
lba_status lba_inertial_workspace_size(lba_ctx *ctx, const lba_problem *problem, const lba_batch *batch,
                                       const lba_inertial *inertial, size_t *bytes);
/* Solve one window or a batch with inertial measurements.  v_out, bg_out, ba_out: DEVICE
 * n_kf x 3 each (may alias the inputs).  Everything else as lba_solve / lba_solve_batch;
 * the costs in the statistics and the trial log include the inertial terms. */
lba_status lba_solve_inertial(lba_ctx *ctx, const lba_problem *problem, const lba_batch *batch,
                              const lba_inertial *inertial, lba_result *result, double *v_out, double *bg_out,
                              double *ba_out, void *workspace, size_t workspace_bytes, void *stream);

/* Tile tuner of the batched form.  The linearisation kernel runs one block per tile of
 * a window's points (the update one block per part of a tile); the tile size trades
 * per-tile work (the partial reduced system each tile writes and the fixed-order sum over
 * tiles) against the number of blocks that fill the GPU.  lba_tune times short solves
 * (three LM steps on every window, on `stream`; the least of three runs after a first
 * that captures the step graph) of this problem with candidate tile sizes 64 ... 4096
 * points, one value per class of windows (LBA_TUNE_CLASSES classes: optimisable
 * keyframes <= 10, <= 20, > 20, times points < 2,000, < 8,000, >= 8,000; class index
 * 3 * keyframe class + point class), by coordinate descent, and keeps the fastest table
 * in the context: later solves of a problem with the same sizes and precision use it
 * when points_per_tile is 0.  The problem's inputs are only read.  It allocates and frees
 * its own device scratch (hipMalloc) and synchronises the stream; points_per_tile (HOST,
 * LBA_TUNE_CLASSES entries, or NULL) receives the table.
 * lba_tune_get copies the context's table (LBA_ERR_INVALID_ARGUMENT if it has none) so
 * that a caller can store it; lba_tune_set installs a stored table (entries 1..65536), which
 * then applies to every problem the context solves with points_per_tile 0 (NULL: forget
 * it). */
#define LBA_TUNE_CLASSES 9
lba_status lba_tune(lba_ctx *ctx, const lba_problem *problem, const lba_batch *batch, void *stream,
                    int32_t *points_per_tile);
lba_status lba_tune_get(const lba_ctx *ctx, int32_t *points_per_tile);
lba_status lba_tune_set(lba_ctx *ctx, const int32_t *points_per_tile);

/* ---- per-kernel timing ------------------------------------------------------------------
 * With profiling enabled, every kernel a solve launches is bracketed by two HIP events on
 * the caller's stream and, at the end of the solve, its duration is added to the counters
 * of its kernel class.  Enabling resets the counters.  Reading returns the number of
 * launches and their summed duration in milliseconds for one class. */
typedef enum {
    LBA_KCLASS_LINEARIZE = 0,    /* residual + Jacobian + Hessian blocks + Schur, per step */
    LBA_KCLASS_LINEARIZE_INIT,   /* cost and damping scale at the start of a round */
    LBA_KCLASS_REDUCE,           /* fixed-order sum of the per-tile partial systems */
    LBA_KCLASS_CHOLESKY,         /* FP64 factorisation and solve of the reduced system */
    LBA_KCLASS_UPDATE,           /* back-substitution, retraction and trial cost */
    LBA_KCLASS_DECIDE,           /* gain ratio, accept / reject, damping update */
    LBA_KCLASS_INIT_REDUCE,
    LBA_KCLASS_SETUP,
    LBA_KCLASS_VALIDATE,
    LBA_KCLASS_FLAGS,            /* chi-square outlier pass */
    LBA_KCLASS_FINALIZE,
    LBA_KCLASS_COST_FORWARD,     /* robust-cost layer, forward */
    LBA_KCLASS_COST_BACKWARD,    /* robust-cost layer, backward */
    LBA_KCLASS_ORDER,            /* once per solve: point order of the linearisation */
    LBA_KCLASS_INERTIAL,         /* inertial measurements: residuals, blocks, joint system */
    LBA_KCLASS_COUNT
} lba_kernel_class;

lba_status lba_profile_enable(lba_ctx *ctx, int32_t enable);
lba_status lba_profile_read(const lba_ctx *ctx, int32_t kernel_class, int64_t *launches, double *total_ms);

/* ---- differentiation form: the robust reprojection cost as a layer ----------------------
 * The same cost the solver minimises (Section III-C: reprojection residuals of the local
 * keyframes and their points), as a differentiable function of the poses, points and
 * measurements of every window of a batch:
 *
 *   cost[w] = sum over the observations i of window w not masked out of rho(s_i),
 *   s_i = |z_i - pi(Exp(xi_k) T_k X_j)|^2 / sigma2[octave_i],
 *
 * with rho the Huber function on s (huber2_mono / huber2_stereo of the context's
 * options), pi the mono or stereo projection and Exp(xi) the SE(3) exponential of a
 * left perturbation xi = (rotation, translation) of the base pose T_k (xi NULL: zero).
 * The backward pass returns, for an upstream gradient grad_cost[w],
 *   g_xi[k] = dL/dxi_k      (all keyframes, fixed or not: the fixed mask is not read),
 *   g_X[j]  = dL/dX_j,      g_z[i] = dL/dz_i   (zero for masked observations and for the
 *                                                uR row of monocular observations).
 * Per-observation arithmetic is FP32; the cost and the pose-gradient sums accumulate in
 * FP64 in a fixed order, so results are reproducible bit for bit.  The backward pass
 * recomputes the Jacobians from the inputs; nothing is kept between the two calls.
 *
 * Topology and constants come from `problem` (and `batch`, NULL: one window):
 * n_kf, n_pt, n_obs, n_levels, T_cw (DEVICE, FP64 base poses), obs_kf, obs_pt, obs_type,
 * obs_oct (DEVICE), sigma2 (HOST), cam.  problem->X_w, obs_z and fixed are not read: the
 * differentiable inputs are the separate FP32 arrays
 *   xi   DEVICE n_kf x 6 or NULL,   X   DEVICE n_pt x 3,   z   DEVICE 3 x n_obs planar
 *   mask DEVICE n_obs (1 = observation left out) or NULL.
 * Outputs (DEVICE, caller-owned): cost n_windows doubles; g_xi n_kf x 6, g_X n_pt x 3,
 * g_z 3 x n_obs floats, every entry written.  grad_cost is DEVICE n_windows doubles.
 * Limits: n_kf <= 128 per window, at most 64 observations per point.  With
 * check_inputs set (the default) the indices are validated on the GPU first and the
 * stream is synchronised once to read the verdict (LBA_ERR_INVALID_ARGUMENT on a bad
 * index, octave, type or order); with it off nothing synchronises, and invalid indices
 * are skipped by the kernels and leave the outputs undefined. */
lba_status lba_cost_workspace_size(lba_ctx *ctx, const lba_problem *problem, const lba_batch *batch,
                                   size_t *bytes);
lba_status lba_cost_forward(lba_ctx *ctx, const lba_problem *problem, const lba_batch *batch,
                            const float *xi, const float *X, const float *z, const uint8_t *mask,
                            double *cost, void *workspace, size_t workspace_bytes, void *stream);
lba_status lba_cost_backward(lba_ctx *ctx, const lba_problem *problem, const lba_batch *batch,
                             const float *xi, const float *X, const float *z, const uint8_t *mask,
                             const double *grad_cost, float *g_xi, float *g_X, float *g_z,
                             void *workspace, size_t workspace_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* LBA_H */
