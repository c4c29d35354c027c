/*
 * lbaref.c -- plain FP64 CPU oracle for Local Bundle Adjustment (LBA).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg load this library; the product path never does.  It shares no code,
 * header, table or helper with the GPU library.
 *
 * What it computes (paper: Section III-C "Local Bundle Adjustment" and Section IV-E
 * "Local Bundle Adjustment"): a nonlinear least-squares refinement of the local
 * keyframe poses and the 3-D points they observe, minimising reprojection residuals,
 * solved iteratively with Levenberg-Marquardt, with the point variables eliminated by
 * the Schur complement so that only the pose system is factorised, then the points
 * back-substituted.  The paper gives no equations for this stage beyond that; the GPU
 * solver it adopts keeps the formulation of the CPU g2o solver it replaces.  The
 * concrete formulation below is the reading used throughout this project:
 *
 *   residual     e = z - pi(T_k X_j)             (mono: u,v ; stereo: u,v,uR)
 *   pinhole      pi = (fx x/z + cx, fy y/z + cy [, fx x/z + cx - bf/z])
 *   weight       s = e^T e / sigma2[octave]      ("chi2" of the observation)
 *   robust cost  rho(s) = s                 if s <= d2
 *                       = 2 sqrt(d2 s) - d2   otherwise     (Huber on s)
 *                F = sum_active rho(s)        (no factor 1/2)
 *   IRLS         H = sum w J^T Om J,  b = sum w Jpi^T Om e,  w = rho'(s),  Om = I/sigma2
 *   damping      (H + lambda I) d = b on every variable; lambda0 = tau * max diag(H)
 *   Schur        S = Hpp + lI - sum_j sum_{a,b in obs(j)} W_a V_j^-1 W_b^T,
 *                r = bp - sum_j sum_a W_a V_j^-1 bl_j,  V_j = Hll_j + lI,
 *                dense Cholesky of S; dl_j = V_j^-1 (bl_j - sum_a W_a^T dp_k(a))
 *   retraction   T_k <- Exp(dp_k) T_k (left, twist = (rotation, translation)),
 *                X_j <- X_j + dl_j
 *   gain ratio   rho_g = (F - F') / (d^T (lambda d + b)); accept iff rho_g > 0 and
 *                finite: lambda *= max(1/3, 1 - (2 rho_g - 1)^3), nu = 2; otherwise
 *                lambda *= nu, nu *= 2 (Nielsen's rule); max_trials rejections end
 *                the round.
 *   schedule     round 1: all observations, robust, iters_round1 iterations;
 *                outlier flags s > chi2(type) or depth <= 0; round 2 on the unflagged
 *                observations, lambda re-initialised, iters_round2 iterations; final
 *                flags recomputed on all observations at the final state.
 *
 * Everything is FP64, single-threaded, written for readability, compiled without
 * fast-math.  Observation order is arbitrary (no sorting is assumed).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ------------------------------------------------------------------------------------ */
/* public structs (mirrored by the ctypes wrapper in lbaref.py)                           */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    int32_t n_kf, n_pt, n_obs, n_levels;
    const double *T_cw;           /* n_kf x 12, row-major [R | t], world -> camera */
    const uint8_t *fixed;         /* n_kf, 1 = pose held fixed */
    const double *X_w;            /* n_pt x 3 */
    const int32_t *obs_kf;        /* n_obs */
    const int32_t *obs_pt;        /* n_obs */
    const double *obs_z;          /* 3 x n_obs planar: u[], v[], uR[] */
    const uint8_t *obs_type;      /* 0 mono, 1 stereo */
    const uint8_t *obs_oct;       /* octave < n_levels */
    const double *sigma2;         /* n_levels */
    double fx, fy, cx, cy, bf;
} ref_problem;

typedef struct {
    int32_t iters_round1, iters_round2, max_trials, round2_robust;
    double huber2_mono, huber2_stereo, chi2_mono, chi2_stereo, tau;
} ref_options;

typedef struct {                  /* one record per LM trial */
    int32_t round, iter, trial, accepted, solve_ok, pad;
    double lambda, F, F_trial, gain;
} ref_logrec;

/* ------------------------------------------------------------------------------------ */
/* small linear algebra                                                                 */
/* ------------------------------------------------------------------------------------ */
static void hat(const double w[3], double W[9]) {
    W[0] = 0.0;   W[1] = -w[2]; W[2] = w[1];
    W[3] = w[2];  W[4] = 0.0;   W[5] = -w[0];
    W[6] = -w[1]; W[7] = w[0];  W[8] = 0.0;
}

static void matmul(const double *A, const double *B, double *C, int n, int m, int p) {
    /* C (n x p) = A (n x m) * B (m x p), all row-major */
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < p; ++j) {
            double acc = 0.0;
            for (int k = 0; k < m; ++k) acc += A[i * m + k] * B[k * p + j];
            C[i * p + j] = acc;
        }
}

/* SE(3) exponential of the twist xi = (w, v): R = I + A W + B W^2,
 * t = (I + B W + C W^2) v with A = sin t / t, B = (1 - cos t)/t^2, C = (t - sin t)/t^3.
 * Series are used below theta = 1e-2 where the closed forms lose digits. */
static void so3_coeffs(double th, double *A, double *B, double *C) {
    if (th < 1e-2) {
        double t2 = th * th, t4 = t2 * t2, t6 = t4 * t2;
        *A = 1.0 - t2 / 6.0 + t4 / 120.0 - t6 / 5040.0;
        *B = 0.5 - t2 / 24.0 + t4 / 720.0 - t6 / 40320.0;
        *C = 1.0 / 6.0 - t2 / 120.0 + t4 / 5040.0 - t6 / 362880.0;
    } else {
        double s = sin(th), h = sin(0.5 * th);
        *A = s / th;
        *B = 2.0 * h * h / (th * th);
        *C = (th - s) / (th * th * th);
    }
}

void lbaref_se3_exp(const double xi[6], double R[9], double t[3]) {
    const double *w = xi, *v = xi + 3;
    double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double A, B, C, W[9], W2[9], V[9];
    so3_coeffs(th, &A, &B, &C);
    hat(w, W);
    matmul(W, W, W2, 3, 3, 3);
    for (int i = 0; i < 9; ++i) {
        double I = (i % 4 == 0) ? 1.0 : 0.0;
        R[i] = I + A * W[i] + B * W2[i];
        V[i] = I + B * W[i] + C * W2[i];
    }
    matmul(V, v, t, 3, 3, 1);
}

/* Left Jacobian of SE(3) for the twist ordering (rotation, translation):
 * Exp(xi + d) ~= Exp(Jl d) Exp(xi),  Jl = [[J, 0], [Q, J]] with J the SO(3) left
 * Jacobian and Q the coupling block (Barfoot, "State Estimation for Robotics", 7.1.5). */
void lbaref_se3_left_jacobian(const double xi[6], double Jl[36]) {
    const double *w = xi, *v = xi + 3;
    double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double A, B, C, W[9], W2[9], J[9], U[9];
    so3_coeffs(th, &A, &B, &C);
    hat(w, W);
    hat(v, U);
    matmul(W, W, W2, 3, 3, 3);
    for (int i = 0; i < 9; ++i) J[i] = ((i % 4 == 0) ? 1.0 : 0.0) + B * W[i] + C * W2[i];
    double c1, c2, c3;
    if (th < 1e-2) {
        double t2 = th * th, t4 = t2 * t2;
        c1 = 1.0 / 6.0 - t2 / 120.0 + t4 / 5040.0;
        c2 = 1.0 / 24.0 - t2 / 720.0 + t4 / 40320.0;
        c3 = 1.0 / 120.0 - t2 / 2520.0 + t4 / 120960.0;
    } else {
        double s = sin(th), c = cos(th);
        c1 = (th - s) / (th * th * th);
        c2 = (th * th + 2.0 * c - 2.0) / (2.0 * th * th * th * th);
        c3 = (2.0 * th - 3.0 * s + th * c) / (2.0 * th * th * th * th * th);
    }
    double WU[9], UW[9], WUW[9], WWU[9], UWW[9], WUWW[9], WWUW[9];
    matmul(W, U, WU, 3, 3, 3);
    matmul(U, W, UW, 3, 3, 3);
    matmul(WU, W, WUW, 3, 3, 3);
    matmul(W2, U, WWU, 3, 3, 3);
    matmul(UW, W, UWW, 3, 3, 3);
    matmul(WUW, W, WUWW, 3, 3, 3);
    matmul(W2, UW, WWUW, 3, 3, 3);
    double Q[9];
    for (int i = 0; i < 9; ++i)
        Q[i] = 0.5 * U[i] + c1 * (WU[i] + UW[i] + WUW[i]) +
               c2 * (WWU[i] + UWW[i] - 3.0 * WUW[i]) + c3 * (WUWW[i] + WWUW[i]);
    memset(Jl, 0, 36 * sizeof(double));
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            Jl[r * 6 + c] = J[r * 3 + c];
            Jl[(r + 3) * 6 + (c + 3)] = J[r * 3 + c];
            Jl[(r + 3) * 6 + c] = Q[r * 3 + c];
        }
}

/* In-place dense Cholesky A = L L^T (row-major n x n, lower triangle used and
 * overwritten with L; the strict upper triangle is zeroed).  Returns 0 on success,
 * 1 if a pivot is not positive or not finite. */
int lbaref_cholesky(int n, double *A) {
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= i; ++j) {
            double sum = A[i * n + j];
            for (int k = 0; k < j; ++k) sum -= A[i * n + k] * A[j * n + k];
            if (i == j) {
                if (!(sum > 0.0) || !isfinite(sum)) return 1;
                A[i * n + i] = sqrt(sum);
            } else {
                A[i * n + j] = sum / A[j * n + j];
            }
        }
        for (int j = i + 1; j < n; ++j) A[i * n + j] = 0.0;
    }
    return 0;
}

/* Solve L L^T x = b given the factor from lbaref_cholesky (b overwritten with x). */
static void chol_solve(int n, const double *L, double *b) {
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * n + k] * b[k];
        b[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = b[i];
        for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * b[k];
        b[i] = s / L[i * n + i];
    }
}

/* Inverse of a 3x3 matrix by the adjugate; returns 1 if det <= 0 or not finite
 * (the matrices inverted here are symmetric positive definite when valid). */
static int inv3_spd(const double *V, double *Vi) {
    double c00 = V[4] * V[8] - V[5] * V[7];
    double c01 = V[5] * V[6] - V[3] * V[8];
    double c02 = V[3] * V[7] - V[4] * V[6];
    double det = V[0] * c00 + V[1] * c01 + V[2] * c02;
    if (!(det > 0.0) || !isfinite(det)) return 1;
    double id = 1.0 / det;
    Vi[0] = c00 * id;
    Vi[1] = (V[2] * V[7] - V[1] * V[8]) * id;
    Vi[2] = (V[1] * V[5] - V[2] * V[4]) * id;
    Vi[3] = c01 * id;
    Vi[4] = (V[0] * V[8] - V[2] * V[6]) * id;
    Vi[5] = (V[2] * V[3] - V[0] * V[5]) * id;
    Vi[6] = c02 * id;
    Vi[7] = (V[1] * V[6] - V[0] * V[7]) * id;
    Vi[8] = (V[0] * V[4] - V[1] * V[3]) * id;
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* observation model                                                                    */
/* ------------------------------------------------------------------------------------ */

/* Camera-frame point and projection of X through pose T (3x4 row-major).  Returns the
 * residual dimension (2 mono, 3 stereo). */
static int project(const ref_problem *P, const double *T, const double *X, int stereo,
                   double pi[3], double Xc[3]) {
    for (int r = 0; r < 3; ++r)
        Xc[r] = T[r * 4 + 0] * X[0] + T[r * 4 + 1] * X[1] + T[r * 4 + 2] * X[2] + T[r * 4 + 3];
    double iz = 1.0 / Xc[2];
    pi[0] = P->fx * Xc[0] * iz + P->cx;
    pi[1] = P->fy * Xc[1] * iz + P->cy;
    pi[2] = stereo ? pi[0] - P->bf * iz : 0.0;
    return stereo ? 3 : 2;
}

/* Jacobians of pi (not of e) w.r.t. the left pose twist (r x 6) and the point (r x 3):
 * dpi/dXc (r x 3) times dXc/dxi = [-[Xc]x | I] and dXc/dX = R. */
static void jacobians(const ref_problem *P, const double *T, const double Xc[3], int stereo,
                      double Jp[18], double Jx[9]) {
    double z = Xc[2], iz = 1.0 / z, iz2 = iz * iz;
    double D[9] = {P->fx * iz, 0.0, -P->fx * Xc[0] * iz2,
                   0.0, P->fy * iz, -P->fy * Xc[1] * iz2,
                   P->fx * iz, 0.0, -(P->fx * Xc[0] - P->bf) * iz2};
    int r = stereo ? 3 : 2;
    double A[18], Xh[9], R[9];
    hat(Xc, Xh);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            A[i * 6 + j] = -Xh[i * 3 + j];
            A[i * 6 + 3 + j] = (i == j) ? 1.0 : 0.0;
            R[i * 3 + j] = T[i * 4 + j];
        }
    matmul(D, A, Jp, r, 3, 6);
    matmul(D, R, Jx, r, 3, 3);
}

static void huber(double s, double d2, double *rho, double *w) {
    if (s <= d2) {
        *rho = s;
        *w = 1.0;
    } else {
        double d = sqrt(d2), rs = sqrt(s);
        *rho = 2.0 * d * rs - d2;
        *w = d / rs;
    }
}

/* exported scalar helpers for pinning */
int lbaref_project(const ref_problem *P, const double T[12], const double X[3], int stereo,
                   double pi[3], double Xc[3]) {
    return project(P, T, X, stereo, pi, Xc);
}

void lbaref_jacobians(const ref_problem *P, const double T[12], const double X[3], int stereo,
                      double Jpose[18], double Jpoint[9]) {
    double pi[3], Xc[3];
    project(P, T, X, stereo, pi, Xc);
    jacobians(P, T, Xc, stereo, Jpose, Jpoint);
}

void lbaref_huber(double s, double d2, double *rho, double *w) { huber(s, d2, rho, w); }

/* squared weighted error s, residual and depth of observation i at (T, X) */
static int obs_eval(const ref_problem *P, const double *T, const double *X, int i, double e[3],
                    double Xc[3], double *s) {
    int k = P->obs_kf[i], j = P->obs_pt[i];
    int stereo = P->obs_type[i] != 0;
    double pi[3];
    int r = project(P, T + 12 * k, X + 3 * j, stereo, pi, Xc);
    e[0] = P->obs_z[i] - pi[0];
    e[1] = P->obs_z[P->n_obs + i] - pi[1];
    e[2] = stereo ? P->obs_z[2 * P->n_obs + i] - pi[2] : 0.0;
    double ss = 0.0;
    for (int q = 0; q < r; ++q) ss += e[q] * e[q];
    *s = ss / P->sigma2[P->obs_oct[i]];
    return r;
}

/* Robust (or plain) cost over the active set (active == NULL: all observations). */
double lbaref_cost(const ref_problem *P, const ref_options *O, const double *T, const double *X,
                   const uint8_t *active, int robust) {
    double F = 0.0;
    for (int i = 0; i < P->n_obs; ++i) {
        if (active && !active[i]) continue;
        double e[3], Xc[3], s, rho, w;
        obs_eval(P, T, X, i, e, Xc, &s);
        if (robust) huber(s, P->obs_type[i] ? O->huber2_stereo : O->huber2_mono, &rho, &w);
        else rho = s;
        F += rho;
    }
    return F;
}

/* ------------------------------------------------------------------------------------ */
/* normal equations in block form                                                       */
/* ------------------------------------------------------------------------------------ */
typedef struct {
    int K, M, N, Kopt;
    int *opt;              /* kf -> optimisable index or -1 */
    double *Hpp, *bp;      /* Kopt x 36, Kopt x 6 */
    double *Hll, *bl;      /* M x 9, M x 3 */
    double *W;             /* N x 18 (6x3), only for active obs on optimisable kfs */
    int *pt_first, *pt_next;   /* per-point linked list of observations */
    double F, maxdiag;
} blocks_t;

static void blocks_alloc(blocks_t *B, const ref_problem *P) {
    B->K = P->n_kf; B->M = P->n_pt; B->N = P->n_obs;
    B->opt = (int *)malloc(sizeof(int) * (B->K + 1));
    B->Kopt = 0;
    for (int k = 0; k < B->K; ++k) B->opt[k] = P->fixed[k] ? -1 : B->Kopt++;
    B->Hpp = (double *)calloc((size_t)B->Kopt * 36 + 1, sizeof(double));
    B->bp = (double *)calloc((size_t)B->Kopt * 6 + 1, sizeof(double));
    B->Hll = (double *)calloc((size_t)B->M * 9 + 1, sizeof(double));
    B->bl = (double *)calloc((size_t)B->M * 3 + 1, sizeof(double));
    B->W = (double *)calloc((size_t)B->N * 18 + 1, sizeof(double));
    B->pt_first = (int *)malloc(sizeof(int) * (B->M + 1));
    B->pt_next = (int *)malloc(sizeof(int) * (B->N + 1));
    for (int j = 0; j < B->M; ++j) B->pt_first[j] = -1;
    for (int i = B->N - 1; i >= 0; --i) {
        int j = P->obs_pt[i];
        B->pt_next[i] = B->pt_first[j];
        B->pt_first[j] = i;
    }
}

static void blocks_free(blocks_t *B) {
    free(B->opt); free(B->Hpp); free(B->bp); free(B->Hll); free(B->bl); free(B->W);
    free(B->pt_first); free(B->pt_next);
}

/* Gauss-Newton blocks at (T, X): H = sum w J^T Om J, b = sum w Jpi^T Om e. */
static void linearize(const ref_problem *P, const ref_options *O, const double *T, const double *X,
                      const uint8_t *active, int robust, blocks_t *B) {
    memset(B->Hpp, 0, sizeof(double) * B->Kopt * 36);
    memset(B->bp, 0, sizeof(double) * B->Kopt * 6);
    memset(B->Hll, 0, sizeof(double) * B->M * 9);
    memset(B->bl, 0, sizeof(double) * B->M * 3);
    B->F = 0.0;
    for (int i = 0; i < P->n_obs; ++i) {
        if (active && !active[i]) continue;
        int k = P->obs_kf[i], j = P->obs_pt[i], stereo = P->obs_type[i] != 0;
        double e[3], Xc[3], s, rho, w;
        int r = obs_eval(P, T, X, i, e, Xc, &s);
        if (robust) huber(s, stereo ? O->huber2_stereo : O->huber2_mono, &rho, &w);
        else { rho = s; w = 1.0; }
        B->F += rho;
        double Jp[18], Jx[9];
        jacobians(P, T + 12 * k, Xc, stereo, Jp, Jx);
        double om = w / P->sigma2[P->obs_oct[i]];
        for (int a = 0; a < 3; ++a) {
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int q = 0; q < r; ++q) acc += Jx[q * 3 + a] * Jx[q * 3 + c];
                B->Hll[j * 9 + a * 3 + c] += om * acc;
            }
            double g = 0.0;
            for (int q = 0; q < r; ++q) g += Jx[q * 3 + a] * e[q];
            B->bl[j * 3 + a] += om * g;
        }
        int ok = B->opt[k];
        if (ok < 0) continue;
        for (int a = 0; a < 6; ++a) {
            for (int c = 0; c < 6; ++c) {
                double acc = 0.0;
                for (int q = 0; q < r; ++q) acc += Jp[q * 6 + a] * Jp[q * 6 + c];
                B->Hpp[ok * 36 + a * 6 + c] += om * acc;
            }
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int q = 0; q < r; ++q) acc += Jp[q * 6 + a] * Jx[q * 3 + c];
                B->W[i * 18 + a * 3 + c] = om * acc;
            }
            double g = 0.0;
            for (int q = 0; q < r; ++q) g += Jp[q * 6 + a] * e[q];
            B->bp[ok * 6 + a] += om * g;
        }
    }
    double md = 0.0;
    for (int k = 0; k < B->Kopt; ++k)
        for (int a = 0; a < 6; ++a) md = fmax(md, B->Hpp[k * 36 + a * 7]);
    for (int j = 0; j < B->M; ++j)
        for (int a = 0; a < 3; ++a) md = fmax(md, B->Hll[j * 9 + a * 4]);
    B->maxdiag = md;
}

static int obs_in_schur(const ref_problem *P, const blocks_t *B, const uint8_t *active, int i) {
    return (!active || active[i]) && B->opt[P->obs_kf[i]] >= 0;
}

/* Reduced camera system S dp = r for damping lambda.  S is n x n (n = 6 Kopt), full. */
static int reduced_system(const ref_problem *P, const blocks_t *B, const uint8_t *active,
                          double lambda, double *S, double *r) {
    int n = 6 * B->Kopt;
    memset(S, 0, sizeof(double) * n * n);
    for (int k = 0; k < B->Kopt; ++k)
        for (int a = 0; a < 6; ++a) {
            r[k * 6 + a] = B->bp[k * 6 + a];
            for (int c = 0; c < 6; ++c)
                S[(k * 6 + a) * n + k * 6 + c] = B->Hpp[k * 36 + a * 6 + c] + (a == c ? lambda : 0.0);
        }
    for (int j = 0; j < B->M; ++j) {
        double V[9], Vi[9];
        for (int q = 0; q < 9; ++q) V[q] = B->Hll[j * 9 + q] + ((q % 4 == 0) ? lambda : 0.0);
        if (inv3_spd(V, Vi)) return 1;
        for (int ia = B->pt_first[j]; ia >= 0; ia = B->pt_next[ia]) {
            if (!obs_in_schur(P, B, active, ia)) continue;
            int ka = B->opt[P->obs_kf[ia]];
            double Y[18];                       /* W_a V^-1 */
            matmul(B->W + ia * 18, Vi, Y, 6, 3, 3);
            for (int a = 0; a < 6; ++a) {
                double acc = 0.0;
                for (int c = 0; c < 3; ++c) acc += Y[a * 3 + c] * B->bl[j * 3 + c];
                r[ka * 6 + a] -= acc;
            }
            for (int ib = B->pt_first[j]; ib >= 0; ib = B->pt_next[ib]) {
                if (!obs_in_schur(P, B, active, ib)) continue;
                int kb = B->opt[P->obs_kf[ib]];
                for (int a = 0; a < 6; ++a)
                    for (int c = 0; c < 6; ++c) {
                        double acc = 0.0;
                        for (int q = 0; q < 3; ++q) acc += Y[a * 3 + q] * B->W[ib * 18 + c * 3 + q];
                        S[(ka * 6 + a) * n + kb * 6 + c] -= acc;
                    }
            }
        }
    }
    return 0;
}

/* Point back-substitution for a pose step: dl_j = V_j^-1 (bl_j - sum_a W_a^T dp_k(a)).
 * Returns 0, or 1 if a point block is not positive definite. */
static int back_substitute(const ref_problem *P, const blocks_t *B, const uint8_t *active, double lambda,
                           const double *dp, double *dl) {
    for (int j = 0; j < B->M; ++j) {
        double V[9], Vi[9], rhs[3];
        for (int q = 0; q < 9; ++q) V[q] = B->Hll[j * 9 + q] + ((q % 4 == 0) ? lambda : 0.0);
        if (inv3_spd(V, Vi)) return 1;
        for (int c = 0; c < 3; ++c) rhs[c] = B->bl[j * 3 + c];
        for (int ia = B->pt_first[j]; ia >= 0; ia = B->pt_next[ia]) {
            if (!obs_in_schur(P, B, active, ia)) continue;
            int ka = B->opt[P->obs_kf[ia]];
            for (int c = 0; c < 3; ++c)
                for (int a = 0; a < 6; ++a) rhs[c] -= B->W[ia * 18 + a * 3 + c] * dp[ka * 6 + a];
        }
        matmul(Vi, rhs, dl + 3 * j, 3, 3, 1);
    }
    return 0;
}

/* Full damped step: Schur-reduced pose solve by dense Cholesky, then back-substitution.
 * Returns 0 on success, 1 if a point block or S is not positive definite. */
static int schur_step(const ref_problem *P, const blocks_t *B, const uint8_t *active, double lambda,
                      double *dp, double *dl) {
    int n = 6 * B->Kopt;
    double *S = (double *)malloc(sizeof(double) * ((size_t)n * n + 1));
    int fail = reduced_system(P, B, active, lambda, S, dp);
    if (!fail && n > 0) {
        fail = lbaref_cholesky(n, S);
        if (!fail) chol_solve(n, S, dp);
    }
    free(S);
    if (fail) return 1;
    return back_substitute(P, B, active, lambda, dp, dl);
}

static void retract(const blocks_t *B, const double *T, const double *X, const double *dp,
                    const double *dl, double *T2, double *X2) {
    for (int k = 0; k < B->K; ++k) {
        int ok = B->opt[k];
        if (ok < 0) {
            memcpy(T2 + 12 * k, T + 12 * k, 12 * sizeof(double));
            continue;
        }
        double R[9], t[3];
        lbaref_se3_exp(dp + 6 * ok, R, t);
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 3; ++c)
                T2[12 * k + r * 4 + c] = R[r * 3 + 0] * T[12 * k + 0 * 4 + c] +
                                         R[r * 3 + 1] * T[12 * k + 1 * 4 + c] +
                                         R[r * 3 + 2] * T[12 * k + 2 * 4 + c];
            T2[12 * k + r * 4 + 3] = R[r * 3 + 0] * T[12 * k + 3] + R[r * 3 + 1] * T[12 * k + 7] +
                                     R[r * 3 + 2] * T[12 * k + 11] + t[r];
        }
    }
    for (int q = 0; q < 3 * B->M; ++q) X2[q] = X[q] + dl[q];
}

/* Outlier test at (T, X) on every observation: s > chi2(type) or depth <= 0. */
void lbaref_flags(const ref_problem *P, const ref_options *O, const double *T, const double *X,
                  uint8_t *flags) {
    for (int i = 0; i < P->n_obs; ++i) {
        double e[3], Xc[3], s;
        obs_eval(P, T, X, i, e, Xc, &s);
        double th = P->obs_type[i] ? O->chi2_stereo : O->chi2_mono;
        flags[i] = (s > th || Xc[2] <= 0.0) ? 1 : 0;
    }
}

/* Damping at the start of a round: tau times the largest diagonal entry of the
 * undamped Gauss-Newton matrix H over every variable, pose and point blocks alike
 * (Madsen, Nielsen & Tingleff, "Methods for Non-Linear Least Squares Problems", 2004,
 * Section 3.2, the initial mu of the Levenberg-Marquardt method). */
double lbaref_initial_damping(double tau, double max_diag_H) { return tau * max_diag_H; }

/* Nielsen's damping update after one trial (same reference, Section 3.2): an accepted
 * step with gain ratio g scales lambda by max(1/3, 1 - (2g - 1)^3) and resets nu to 2;
 * a rejected one multiplies lambda by nu and doubles nu. */
void lbaref_damping_update(double gain, int accepted, double *lambda, double *nu) {
    if (accepted) {
        double f = 2.0 * gain - 1.0;
        *lambda *= fmax(1.0 / 3.0, 1.0 - f * f * f);
        *nu = 2.0;
    } else {
        *lambda *= *nu;
        *nu *= 2.0;
    }
}

/* one LM round; returns the number of completed (accepted) iterations; *terminated set
 * when max_trials consecutive rejections ended the round early */
static int lm_round(const ref_problem *P, const ref_options *O, int round, int iters,
                    const uint8_t *active, int robust, double *T, double *X, blocks_t *B,
                    double *F_out, double *lambda_out, int *trials_total, int *terminated,
                    ref_logrec *log, int log_cap, int *log_n) {
    int n = 6 * B->Kopt;
    double *dp = (double *)malloc(sizeof(double) * (n + 1));
    double *dl = (double *)malloc(sizeof(double) * (3 * B->M + 1));
    double *T2 = (double *)malloc(sizeof(double) * (12 * B->K + 1));
    double *X2 = (double *)malloc(sizeof(double) * (3 * B->M + 1));
    linearize(P, O, T, X, active, robust, B);
    double F = B->F;
    double lambda = lbaref_initial_damping(O->tau, B->maxdiag), nu = 2.0;
    int done = 0;
    *terminated = 0;
    for (int it = 0; it < iters; ++it) {
        int accepted = 0;
        for (int trial = 0; trial < O->max_trials; ++trial) {
            ++*trials_total;
            int fail = schur_step(P, B, active, lambda, dp, dl);
            double F2 = NAN, gain = NAN;
            if (!fail) {
                retract(B, T, X, dp, dl, T2, X2);
                F2 = lbaref_cost(P, O, T2, X2, active, robust);
                double den = 0.0;
                for (int q = 0; q < n; ++q) den += dp[q] * (lambda * dp[q] + B->bp[q]);
                for (int q = 0; q < 3 * B->M; ++q) den += dl[q] * (lambda * dl[q] + B->bl[q]);
                gain = (F - F2) / den;
            }
            int acc = !fail && isfinite(F2) && isfinite(gain) && gain > 0.0;
            if (log && *log_n < log_cap) {
                ref_logrec *L = &log[(*log_n)++];
                L->round = round; L->iter = it; L->trial = trial; L->accepted = acc;
                L->solve_ok = !fail; L->pad = 0;
                L->lambda = lambda; L->F = F; L->F_trial = F2; L->gain = gain;
            }
            lbaref_damping_update(gain, acc, &lambda, &nu);
            if (acc) {
                memcpy(T, T2, sizeof(double) * 12 * B->K);
                memcpy(X, X2, sizeof(double) * 3 * B->M);
                F = F2;
                accepted = 1;
                break;
            }
        }
        if (!accepted) {
            *terminated = 1;
            break;
        }
        ++done;
        if (it + 1 < iters) linearize(P, O, T, X, active, robust, B);
    }
    *F_out = F;
    *lambda_out = lambda;
    free(dp); free(dl); free(T2); free(X2);
    return done;
}

/*
 * Full solve.  stats[0..11]: initial cost (round-1 objective at the input state),
 * final cost (round-2 objective at the final state), iterations round 1, iterations
 * round 2, trials, final lambda, round-1 terminated early, round-2 terminated early,
 * final outlier count, cost at the end of round 1, round-2 initial cost, Kopt.
 * Returns 0, or -1 for invalid input.
 */
int lbaref_solve(const ref_problem *P, const ref_options *O, double *T_out, double *X_out,
                 uint8_t *outlier_out, double *stats, ref_logrec *log, int log_cap, int *log_n) {
    for (int i = 0; i < P->n_obs; ++i) {
        if (P->obs_kf[i] < 0 || P->obs_kf[i] >= P->n_kf) return -1;
        if (P->obs_pt[i] < 0 || P->obs_pt[i] >= P->n_pt) return -1;
        if (P->obs_oct[i] >= P->n_levels) return -1;
    }
    int ln = 0;
    if (!log_n) log_n = &ln;
    *log_n = 0;
    memcpy(T_out, P->T_cw, sizeof(double) * 12 * P->n_kf);
    memcpy(X_out, P->X_w, sizeof(double) * 3 * P->n_pt);
    blocks_t B;
    blocks_alloc(&B, P);
    double F0 = lbaref_cost(P, O, T_out, X_out, NULL, 1);
    double F1 = F0, F2, lam1 = 0.0, lam2 = 0.0;
    int trials = 0, term1 = 0, term2 = 0;
    int it1 = lm_round(P, O, 1, O->iters_round1, NULL, 1, T_out, X_out, &B, &F1, &lam1, &trials,
                       &term1, log, log_cap, log_n);
    if (O->iters_round1 == 0) F1 = F0;
    uint8_t *active = (uint8_t *)malloc((size_t)P->n_obs + 1);
    lbaref_flags(P, O, T_out, X_out, outlier_out);
    for (int i = 0; i < P->n_obs; ++i) active[i] = !outlier_out[i];
    double F20 = lbaref_cost(P, O, T_out, X_out, active, O->round2_robust);
    F2 = F20;
    int it2 = lm_round(P, O, 2, O->iters_round2, active, O->round2_robust, T_out, X_out, &B, &F2,
                       &lam2, &trials, &term2, log, log_cap, log_n);
    if (O->iters_round2 == 0) F2 = F20;
    lbaref_flags(P, O, T_out, X_out, outlier_out);
    int nout = 0;
    for (int i = 0; i < P->n_obs; ++i) nout += outlier_out[i];
    if (stats) {
        stats[0] = F0; stats[1] = F2; stats[2] = it1; stats[3] = it2; stats[4] = trials;
        stats[5] = O->iters_round2 > 0 ? lam2 : lam1; stats[6] = term1; stats[7] = term2;
        stats[8] = nout; stats[9] = F1; stats[10] = F20; stats[11] = B.Kopt;
    }
    free(active);
    blocks_free(&B);
    return 0;
}

/* ------------------------------------------------------------------------------------ */
/* intermediates for pinning and kernel-level comparison                                */
/* ------------------------------------------------------------------------------------ */

/* Linearise at (T, X) and return the damped reduced system (S n x n full, r n), the
 * pose gradient bp (n), point blocks Hll (M x 9) / bl (M x 3), the cost and max diag,
 * and the step (dp n, dl M x 3).  Returns 0 or 1 (a factorisation failed). */
int lbaref_system(const ref_problem *P, const ref_options *O, const double *T, const double *X,
                  const uint8_t *active, int robust, double lambda, double *S, double *r, double *bp,
                  double *Hll, double *bl, double *Fmd, double *dp, double *dl) {
    blocks_t B;
    blocks_alloc(&B, P);
    linearize(P, O, T, X, active, robust, &B);
    int n = 6 * B.Kopt;
    int fail = reduced_system(P, &B, active, lambda, S, r);
    memcpy(bp, B.bp, sizeof(double) * n);
    memcpy(Hll, B.Hll, sizeof(double) * 9 * B.M);
    memcpy(bl, B.bl, sizeof(double) * 3 * B.M);
    Fmd[0] = B.F;
    Fmd[1] = B.maxdiag;
    if (!fail) fail = schur_step(P, &B, active, lambda, dp, dl);
    blocks_free(&B);
    return fail;
}

/* Dense (undamped) normal equations over all variables, for tiny windows: variable
 * order = optimisable poses (6 each, in keyframe order) then points (3 each).
 * H is D x D, b is D, D = 6 Kopt + 3 M. */
void lbaref_dense_system(const ref_problem *P, const ref_options *O, const double *T,
                         const double *X, const uint8_t *active, int robust, double *H, double *b) {
    int Kopt = 0;
    int *opt = (int *)malloc(sizeof(int) * (P->n_kf + 1));
    for (int k = 0; k < P->n_kf; ++k) opt[k] = P->fixed[k] ? -1 : Kopt++;
    int D = 6 * Kopt + 3 * P->n_pt;
    memset(H, 0, sizeof(double) * D * D);
    memset(b, 0, sizeof(double) * D);
    double *J = (double *)malloc(sizeof(double) * 3 * D);
    for (int i = 0; i < P->n_obs; ++i) {
        if (active && !active[i]) continue;
        int k = P->obs_kf[i], j = P->obs_pt[i], stereo = P->obs_type[i] != 0;
        double e[3], Xc[3], s, rho, w;
        int r = obs_eval(P, T, X, i, e, Xc, &s);
        if (robust) huber(s, stereo ? O->huber2_stereo : O->huber2_mono, &rho, &w);
        else w = 1.0;
        double Jp[18], Jx[9];
        jacobians(P, T + 12 * k, Xc, stereo, Jp, Jx);
        memset(J, 0, sizeof(double) * 3 * D);          /* full-width Jacobian row block */
        for (int q = 0; q < r; ++q) {
            if (opt[k] >= 0)
                for (int a = 0; a < 6; ++a) J[q * D + 6 * opt[k] + a] = Jp[q * 6 + a];
            for (int a = 0; a < 3; ++a) J[q * D + 6 * Kopt + 3 * j + a] = Jx[q * 3 + a];
        }
        double om = w / P->sigma2[P->obs_oct[i]];
        for (int a = 0; a < D; ++a) {
            for (int q = 0; q < r; ++q) b[a] += om * J[q * D + a] * e[q];
            for (int c = 0; c < D; ++c) {
                double acc = 0.0;
                for (int q = 0; q < r; ++q) acc += J[q * D + a] * J[q * D + c];
                H[a * D + c] += om * acc;
            }
        }
    }
    free(J);
    free(opt);
}

/*
 * Differentiable robust cost: F = sum over all observations of rho(s) evaluated at
 * poses Exp(xi_k) T_k (xi may be NULL for zero) and points X.  Gradients:
 * g_xi (n_kf x 6) = dF/dxi including the SE(3) left Jacobian, g_X (n_pt x 3),
 * g_z (3 x n_obs planar; the uR row is zero for mono).  Fixed flags are ignored.
 */
double lbaref_cost_grad(const ref_problem *P, const ref_options *O, const double *xi, double *g_xi,
                        double *g_X, double *g_z) {
    int K = P->n_kf;
    double *T = (double *)malloc(sizeof(double) * 12 * (K + 1));
    double *gl = (double *)calloc(6 * (K + 1), sizeof(double));
    for (int k = 0; k < K; ++k) {
        const double *T0 = P->T_cw + 12 * k;
        if (!xi) {
            memcpy(T + 12 * k, T0, 12 * sizeof(double));
            continue;
        }
        double R[9], t[3];
        lbaref_se3_exp(xi + 6 * k, R, t);
        for (int r = 0; r < 3; ++r) {
            for (int c = 0; c < 4; ++c) {
                double acc = 0.0;
                for (int q = 0; q < 3; ++q) acc += R[r * 3 + q] * T0[q * 4 + c];
                T[12 * k + r * 4 + c] = acc + (c == 3 ? t[r] : 0.0);
            }
        }
    }
    if (g_X) memset(g_X, 0, sizeof(double) * 3 * P->n_pt);
    double F = 0.0;
    for (int i = 0; i < P->n_obs; ++i) {
        int k = P->obs_kf[i], j = P->obs_pt[i], stereo = P->obs_type[i] != 0;
        double e[3], Xc[3], s, rho, w;
        int r = obs_eval(P, T, P->X_w, i, e, Xc, &s);
        huber(s, stereo ? O->huber2_stereo : O->huber2_mono, &rho, &w);
        F += rho;
        double om = w / P->sigma2[P->obs_oct[i]];
        /* dF/dz = 2 w Om e ; dF/dparam = -2 w Jpi^T Om e */
        if (g_z)
            for (int q = 0; q < 3; ++q) g_z[q * P->n_obs + i] = q < r ? 2.0 * om * e[q] : 0.0;
        double Jp[18], Jx[9];
        jacobians(P, T + 12 * k, Xc, stereo, Jp, Jx);
        for (int a = 0; a < 6; ++a) {
            double g = 0.0;
            for (int q = 0; q < r; ++q) g += Jp[q * 6 + a] * e[q];
            gl[6 * k + a] -= 2.0 * om * g;
        }
        if (g_X)
            for (int a = 0; a < 3; ++a) {
                double g = 0.0;
                for (int q = 0; q < r; ++q) g += Jx[q * 3 + a] * e[q];
                g_X[3 * j + a] -= 2.0 * om * g;
            }
    }
    if (g_xi)
        for (int k = 0; k < K; ++k) {
            if (!xi) {
                memcpy(g_xi + 6 * k, gl + 6 * k, 6 * sizeof(double));
                continue;
            }
            double Jl[36];
            lbaref_se3_left_jacobian(xi + 6 * k, Jl);
            for (int a = 0; a < 6; ++a) {
                double acc = 0.0;
                for (int q = 0; q < 6; ++q) acc += Jl[q * 6 + a] * gl[6 * k + q];
                g_xi[6 * k + a] = acc;
            }
        }
    free(T);
    free(gl);
    return F;
}

/* ==================================================================================== */
/* Stereo-inertial local bundle adjustment                                              */
/*                                                                                      */
/* The paper's local bundle adjustment minimises reprojection errors, and in visual-    */
/* inertial systems inertial residuals as well (Section III-C); its experiments run     */
/* stereo-inertial (Section V-A).  It gives no equations for the inertial terms; the     */
/* reading here is the preintegrated-IMU factor of Forster, Carlone, Dellaert and         */
/* Scaramuzza, "On-Manifold Preintegration for Real-Time Visual-Inertial Odometry"       */
/* (IEEE T-RO 2017), Section VI, with a bias random-walk factor:                          */
/*                                                                                      */
/*   states     per keyframe the camera pose T_cw (as above), the body velocity v in    */
/*              the world frame, gyroscope bias bg and accelerometer bias ba; fixed      */
/*              keyframes hold all of them;                                               */
/*   body pose  R = R_cw^T R_cb, p = R_cw^T (t_cb - t_cw) for the body-to-camera         */
/*              transform T_cb = [R_cb | t_cb];                                           */
/*   residual   for a measurement (dR, dv, dp, dt, biases bg_bar / ba_bar it was          */
/*              integrated with, bias Jacobians J_Rg, J_vg, J_va, J_pg, J_pa) between    */
/*              keyframes i and j, with dbg = bg_i - bg_bar, dba = ba_i - ba_bar:          */
/*                r_R = Log((dR Exp(J_Rg dbg))^T R_i^T R_j)                              */
/*                r_v = R_i^T (v_j - v_i - g dt) - (dv + J_vg dbg + J_va dba)             */
/*                r_p = R_i^T (p_j - p_i - v_i dt - g dt^2 / 2) - (dp + J_pg dbg + J_pa dba)*/
/*                r_bg = bg_j - bg_i,  r_ba = ba_j - ba_i                                 */
/*   cost       r9^T Info r9 + info_bg |r_bg|^2 + info_ba |r_ba|^2 per measurement       */
/*              (r9 = (r_R, r_v, r_p); no robust kernel, no factor 1/2, like the          */
/*              reprojection terms), added to the reprojection cost;                      */
/*   step       the normal equations gain the inertial blocks on 15 unknowns per          */
/*              optimisable keyframe (twist, dv, dbg, dba); the points are eliminated     */
/*              as before, so the reduced system has 15 Kopt unknowns; lambda is added    */
/*              to every diagonal entry; v, bg, ba move additively.                        */
/* ==================================================================================== */

typedef struct {
    int32_t n_edges, pad;
    const int32_t *edge_i, *edge_j;   /* keyframes of each measurement */
    const double *dt;                 /* n_edges */
    const double *dR;                 /* n_edges x 9 */
    const double *dv, *dp;            /* n_edges x 3 */
    const double *J_Rg, *J_vg, *J_va, *J_pg, *J_pa;   /* n_edges x 9 each */
    const double *bg_bar, *ba_bar;    /* n_edges x 3 */
    const double *info;               /* n_edges x 81, information of (r_R, r_v, r_p) */
    const double *info_bg, *info_ba;  /* n_edges */
    const double *T_cb;               /* 12 */
    double g[3];                      /* gravity, world frame */
} ref_inertial;

/* SO(3) exponential R = I + A W + B W^2 (coefficients as for SE(3) above). */
static void so3_exp(const double w[3], double R[9]) {
    double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double A, B, C, W[9], W2[9];
    so3_coeffs(th, &A, &B, &C);
    hat(w, W);
    matmul(W, W, W2, 3, 3, 3);
    for (int i = 0; i < 9; ++i) R[i] = ((i % 4 == 0) ? 1.0 : 0.0) + A * W[i] + B * W2[i];
}

/* SO(3) logarithm: the angle from atan2(|sin|, cos), so that small angles keep their
 * digits; near pi the axis comes from the symmetric part R + I. */
void lbaref_so3_log(const double R[9], double w[3]) {
    double vx = 0.5 * (R[7] - R[5]), vy = 0.5 * (R[2] - R[6]), vz = 0.5 * (R[3] - R[1]);
    double s = sqrt(vx * vx + vy * vy + vz * vz);
    double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    double th = atan2(s, c);
    if (th < 1e-4) {
        double f = 1.0 + th * th / 6.0;           /* th / sin th */
        w[0] = f * vx; w[1] = f * vy; w[2] = f * vz;
    } else if (M_PI - th > 1e-4) {
        double f = th / s;
        w[0] = f * vx; w[1] = f * vy; w[2] = f * vz;
    } else {
        /* near pi: the symmetric part gives (R + R^T) / 2 - cos(t) I = (1 - cos t) a a^T;
         * its column of largest diagonal entry is parallel to the axis a, and the
         * antisymmetric part fixes the sign */
        double Bm[9];
        for (int r = 0; r < 3; ++r)
            for (int q = 0; q < 3; ++q) Bm[r * 3 + q] = 0.5 * (R[r * 3 + q] + R[q * 3 + r]) - (r == q ? c : 0.0);
        int k = 0;
        for (int q = 1; q < 3; ++q) if (Bm[q * 4] > Bm[k * 4]) k = q;
        double a[3];
        for (int q = 0; q < 3; ++q) a[q] = Bm[q * 3 + k];
        double na = sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        double sg = (a[0] * vx + a[1] * vy + a[2] * vz) < 0.0 ? -1.0 : 1.0;
        for (int q = 0; q < 3; ++q) w[q] = sg * th * a[q] / na;
    }
}

/* Right Jacobian of SO(3): Jr(w) = I - B W + C W^2 (Exp(w + d) ~= Exp(w) Exp(Jr d)). */
void lbaref_so3_jr(const double w[3], double Jr[9]) {
    double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double A, B, C, W[9], W2[9];
    so3_coeffs(th, &A, &B, &C);
    hat(w, W);
    matmul(W, W, W2, 3, 3, 3);
    for (int i = 0; i < 9; ++i) Jr[i] = ((i % 4 == 0) ? 1.0 : 0.0) - B * W[i] + C * W2[i];
}

/* Its inverse: Jr^-1(w) = I + W / 2 + D W^2, D = 1/t^2 - (1 + cos t) / (2 t sin t). */
void lbaref_so3_jr_inv(const double w[3], double Jri[9]) {
    double th = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    double D, W[9], W2[9];
    if (th < 1e-2) {
        double t2 = th * th;
        D = 1.0 / 12.0 + t2 / 720.0 + t2 * t2 / 30240.0;
    } else {
        D = 1.0 / (th * th) - (1.0 + cos(th)) / (2.0 * th * sin(th));
    }
    hat(w, W);
    matmul(W, W, W2, 3, 3, 3);
    for (int i = 0; i < 9; ++i) Jri[i] = ((i % 4 == 0) ? 1.0 : 0.0) + 0.5 * W[i] + D * W2[i];
}

static void transpose3(const double *A, double *At) {
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) At[c * 3 + r] = A[r * 3 + c];
}

/* body rotation and position of a keyframe from its camera pose */
static void body_pose(const double *T, const double *T_cb, double Rb[9], double pb[3]) {
    double Rcw[9], RcwT[9], Rcb[9], d[3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            Rcw[r * 3 + c] = T[r * 4 + c];
            Rcb[r * 3 + c] = T_cb[r * 4 + c];
        }
    transpose3(Rcw, RcwT);
    matmul(RcwT, Rcb, Rb, 3, 3, 3);
    for (int q = 0; q < 3; ++q) d[q] = T_cb[q * 4 + 3] - T[q * 4 + 3];
    matmul(RcwT, d, pb, 3, 3, 1);
}

/* intermediate quantities of measurement e at the states */
typedef struct {
    double Ri[9], Rj[9], pi[3], pj[3];
    double dbg[3], dba[3], E[9], u[3], w[3], r[15];
} vi_eval_t;

static void vi_eval(const ref_inertial *I, int e, const double *T, const double *V, const double *BG,
                    const double *BA, vi_eval_t *q) {
    int i = I->edge_i[e], j = I->edge_j[e];
    double dt = I->dt[e];
    body_pose(T + 12 * i, I->T_cb, q->Ri, q->pi);
    body_pose(T + 12 * j, I->T_cb, q->Rj, q->pj);
    for (int a = 0; a < 3; ++a) {
        q->dbg[a] = BG[3 * i + a] - I->bg_bar[3 * e + a];
        q->dba[a] = BA[3 * i + a] - I->ba_bar[3 * e + a];
    }
    /* rotation: E = (dR Exp(J_Rg dbg))^T R_i^T R_j */
    double phi[3], Eb[9], dRc[9], dRcT[9], RiT[9], RiTRj[9];
    matmul(I->J_Rg + 9 * e, q->dbg, phi, 3, 3, 1);
    so3_exp(phi, Eb);
    matmul(I->dR + 9 * e, Eb, dRc, 3, 3, 3);
    transpose3(dRc, dRcT);
    transpose3(q->Ri, RiT);
    matmul(RiT, q->Rj, RiTRj, 3, 3, 3);
    matmul(dRcT, RiTRj, q->E, 3, 3, 3);
    lbaref_so3_log(q->E, q->r);
    /* velocity and position */
    double Ru[3], Rw[3], a1[3], a2[3], b1[3], b2[3];
    for (int a = 0; a < 3; ++a) {
        q->u[a] = V[3 * j + a] - V[3 * i + a] - I->g[a] * dt;
        q->w[a] = q->pj[a] - q->pi[a] - V[3 * i + a] * dt - 0.5 * I->g[a] * dt * dt;
    }
    matmul(RiT, q->u, Ru, 3, 3, 1);
    matmul(RiT, q->w, Rw, 3, 3, 1);
    matmul(I->J_vg + 9 * e, q->dbg, a1, 3, 3, 1);
    matmul(I->J_va + 9 * e, q->dba, a2, 3, 3, 1);
    matmul(I->J_pg + 9 * e, q->dbg, b1, 3, 3, 1);
    matmul(I->J_pa + 9 * e, q->dba, b2, 3, 3, 1);
    for (int a = 0; a < 3; ++a) {
        q->r[3 + a] = Ru[a] - (I->dv[3 * e + a] + a1[a] + a2[a]);
        q->r[6 + a] = Rw[a] - (I->dp[3 * e + a] + b1[a] + b2[a]);
        q->r[9 + a] = BG[3 * j + a] - BG[3 * i + a];
        q->r[12 + a] = BA[3 * j + a] - BA[3 * i + a];
    }
}

static double vi_edge_cost(const ref_inertial *I, int e, const double r[15]) {
    double c = 0.0;
    for (int a = 0; a < 9; ++a) {
        double acc = 0.0;
        for (int b = 0; b < 9; ++b) acc += I->info[81 * e + a * 9 + b] * r[b];
        c += r[a] * acc;
    }
    double g2 = 0.0, a2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        g2 += r[9 + a] * r[9 + a];
        a2 += r[12 + a] * r[12 + a];
    }
    return c + I->info_bg[e] * g2 + I->info_ba[e] * a2;
}

void lbaref_vi_residual(const ref_inertial *I, int e, const double *T, const double *V, const double *BG,
                        const double *BA, double r[15]) {
    vi_eval_t q;
    vi_eval(I, e, T, V, BG, BA, &q);
    memcpy(r, q.r, sizeof(q.r));
}

double lbaref_vi_cost(const ref_inertial *I, const double *T, const double *V, const double *BG,
                      const double *BA) {
    double F = 0.0;
    for (int e = 0; e < I->n_edges; ++e) {
        vi_eval_t q;
        vi_eval(I, e, T, V, BG, BA, &q);
        F += vi_edge_cost(I, e, q.r);
    }
    return F;
}

/* Jacobian (15 x 30, row-major) of the residual of measurement e with respect to the
 * perturbations (twist, dv, dbg, dba) of keyframe i (columns 0-14) and keyframe j
 * (columns 15-29).  Body-frame perturbations first: the left twist (w, u) of T_cw turns
 * the body rotation by -R_cb^T w (on the right) and moves the body position by
 * R_cw^T ([t_cb]x w - u); then the standard preintegration derivatives. */
void lbaref_vi_jacobian(const ref_inertial *I, int e, const double *T, const double *V, const double *BG,
                        const double *BA, double J[450]) {
    vi_eval_t q;
    vi_eval(I, e, T, V, BG, BA, &q);
    double dt = I->dt[e];
    /* blocks per residual row group and body variable: th_i, p_i, v_i, bg_i, ba_i,
     * th_j, p_j, v_j, bg_j, ba_j (15 x 3 each) */
    double Bk[10][45];
    memset(Bk, 0, sizeof(Bk));
#define SETB(blk, row, M9) do { for (int rr = 0; rr < 3; ++rr) for (int cc = 0; cc < 3; ++cc) \
        Bk[blk][((row) + rr) * 3 + cc] = (M9)[rr * 3 + cc]; } while (0)
    double Jri[9], RjT[9], RjTRi[9], tmp[9], RiT[9], mRiT[9], I3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, mI3[9];
    lbaref_so3_jr_inv(q.r, Jri);
    transpose3(q.Rj, RjT);
    transpose3(q.Ri, RiT);
    for (int a = 0; a < 9; ++a) {
        mRiT[a] = -RiT[a];
        mI3[a] = -I3[a];
    }
    /* r_R */
    matmul(RjT, q.Ri, RjTRi, 3, 3, 3);
    matmul(Jri, RjTRi, tmp, 3, 3, 3);
    for (int a = 0; a < 9; ++a) tmp[a] = -tmp[a];
    SETB(0, 0, tmp);
    SETB(5, 0, Jri);
    {
        double phi[3], Jr[9], ET[9], M1[9], M2[9], M3[9];
        matmul(I->J_Rg + 9 * e, q.dbg, phi, 3, 3, 1);
        lbaref_so3_jr(phi, Jr);
        transpose3(q.E, ET);
        matmul(Jri, ET, M1, 3, 3, 3);
        matmul(M1, Jr, M2, 3, 3, 3);
        matmul(M2, I->J_Rg + 9 * e, M3, 3, 3, 3);
        for (int a = 0; a < 9; ++a) M3[a] = -M3[a];
        SETB(3, 0, M3);
    }
    /* r_v */
    {
        double Ru[3], H[9], M[9];
        matmul(RiT, q.u, Ru, 3, 3, 1);
        hat(Ru, H);
        SETB(0, 3, H);
        SETB(2, 3, mRiT);
        SETB(7, 3, RiT);
        for (int a = 0; a < 9; ++a) M[a] = -I->J_vg[9 * e + a];
        SETB(3, 3, M);
        for (int a = 0; a < 9; ++a) M[a] = -I->J_va[9 * e + a];
        SETB(4, 3, M);
    }
    /* r_p */
    {
        double Rw[3], H[9], M[9];
        matmul(RiT, q.w, Rw, 3, 3, 1);
        hat(Rw, H);
        SETB(0, 6, H);
        SETB(1, 6, mRiT);
        SETB(6, 6, RiT);
        for (int a = 0; a < 9; ++a) M[a] = -RiT[a] * dt;
        SETB(2, 6, M);
        for (int a = 0; a < 9; ++a) M[a] = -I->J_pg[9 * e + a];
        SETB(3, 6, M);
        for (int a = 0; a < 9; ++a) M[a] = -I->J_pa[9 * e + a];
        SETB(4, 6, M);
    }
    /* bias random walks */
    SETB(3, 9, mI3);
    SETB(8, 9, I3);
    SETB(4, 12, mI3);
    SETB(9, 12, I3);
#undef SETB
    /* chain to the camera twist of each keyframe, assemble 15 x 30 */
    memset(J, 0, sizeof(double) * 450);
    double RcbT[9], Rcb[9], tcb[3], tx[9];
    for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) Rcb[r * 3 + c] = I->T_cb[r * 4 + c];
        tcb[r] = I->T_cb[r * 4 + 3];
    }
    transpose3(Rcb, RcbT);
    hat(tcb, tx);
    for (int side = 0; side < 2; ++side) {
        int k = side == 0 ? I->edge_i[e] : I->edge_j[e];
        const double *Tk = T + 12 * k;
        double Rcw[9], RcwT[9], Ptw[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) Rcw[r * 3 + c] = Tk[r * 4 + c];
        transpose3(Rcw, RcwT);
        matmul(RcwT, tx, Ptw, 3, 3, 3);                 /* d p / d w = R_cw^T [t_cb]x */
        const double *Bth = Bk[5 * side + 0], *Bp = Bk[5 * side + 1];
        for (int row = 0; row < 15; ++row) {
            double *Jr = J + row * 30 + 15 * side;
            for (int c = 0; c < 3; ++c) {
                double aw = 0.0, au = 0.0;
                for (int m = 0; m < 3; ++m) {
                    aw += Bth[row * 3 + m] * (-RcbT[m * 3 + c]) + Bp[row * 3 + m] * Ptw[m * 3 + c];
                    au += Bp[row * 3 + m] * (-RcwT[m * 3 + c]);
                }
                Jr[c] = aw;
                Jr[3 + c] = au;
            }
            for (int blk = 2; blk < 5; ++blk)
                for (int c = 0; c < 3; ++c) Jr[6 + 3 * (blk - 2) + c] = Bk[5 * side + blk][row * 3 + c];
        }
    }
}

/* inertial normal equations over the 15 Kopt unknowns: H (n x n, added), b (added),
 * b = -J^T Info r; returns the inertial cost */
static double vi_linearize(const ref_inertial *I, const int *opt, int n, const double *T, const double *V,
                           const double *BG, const double *BA, double *H, double *b) {
    double F = 0.0;
    for (int e = 0; e < I->n_edges; ++e) {
        vi_eval_t q;
        vi_eval(I, e, T, V, BG, BA, &q);
        F += vi_edge_cost(I, e, q.r);
        double J[450], Om[225];
        lbaref_vi_jacobian(I, e, T, V, BG, BA, J);
        memset(Om, 0, sizeof(Om));
        for (int a = 0; a < 9; ++a)
            for (int c = 0; c < 9; ++c) Om[a * 15 + c] = I->info[81 * e + a * 9 + c];
        for (int a = 9; a < 12; ++a) Om[a * 15 + a] = I->info_bg[e];
        for (int a = 12; a < 15; ++a) Om[a * 15 + a] = I->info_ba[e];
        double OJ[450], Or[15];
        matmul(Om, J, OJ, 15, 15, 30);
        matmul(Om, q.r, Or, 15, 15, 1);
        int col0[2] = {opt[I->edge_i[e]], opt[I->edge_j[e]]};
        for (int sa = 0; sa < 2; ++sa) {
            if (col0[sa] < 0) continue;
            for (int a = 0; a < 15; ++a) {
                int ga = 15 * col0[sa] + a, ca = 15 * sa + a;
                double g = 0.0;
                for (int m = 0; m < 15; ++m) g += J[m * 30 + ca] * Or[m];
                b[ga] -= g;
                for (int sc = 0; sc < 2; ++sc) {
                    if (col0[sc] < 0) continue;
                    for (int c = 0; c < 15; ++c) {
                        int gc = 15 * col0[sc] + c, cc = 15 * sc + c;
                        double acc = 0.0;
                        for (int m = 0; m < 15; ++m) acc += J[m * 30 + ca] * OJ[m * 30 + cc];
                        H[ga * n + gc] += acc;
                    }
                }
            }
        }
    }
    return F;
}

/* Damped step of the visual-inertial system: the visual reduced system (6 Kopt) placed in
 * the pose rows of the 15 Kopt system, the inertial blocks and lambda on the velocity and
 * bias diagonal added, dense Cholesky, then the points back-substituted with the pose
 * part.  d: 15 Kopt, dl: 3 M.  Returns 0, or 1 if a factorisation failed. */
static int vi_step(const ref_problem *P, const blocks_t *B, const uint8_t *active, double lambda,
                   const double *Hi, const double *bi, double *d, double *dl) {
    int nv = 6 * B->Kopt, n = 15 * B->Kopt;
    double *Sv = (double *)malloc(sizeof(double) * ((size_t)nv * nv + 1));
    double *rv = (double *)malloc(sizeof(double) * (nv + 1));
    double *S = (double *)malloc(sizeof(double) * ((size_t)n * n + 1));
    double *dp = (double *)malloc(sizeof(double) * (nv + 1));
    int fail = reduced_system(P, B, active, lambda, Sv, rv);
    if (!fail) {
        for (int a = 0; a < n; ++a) {
            d[a] = bi[a];
            for (int c = 0; c < n; ++c) S[a * n + c] = Hi[a * n + c];
            if (a % 15 >= 6) S[a * n + a] += lambda;
        }
        for (int ka = 0; ka < B->Kopt; ++ka)
            for (int a = 0; a < 6; ++a) {
                d[15 * ka + a] += rv[6 * ka + a];
                for (int kc = 0; kc < B->Kopt; ++kc)
                    for (int c = 0; c < 6; ++c) S[(15 * ka + a) * n + 15 * kc + c] += Sv[(6 * ka + a) * nv + 6 * kc + c];
            }
        if (n > 0) {
            fail = lbaref_cholesky(n, S);
            if (!fail) chol_solve(n, S, d);
        }
    }
    if (!fail) {
        for (int ka = 0; ka < B->Kopt; ++ka)
            for (int a = 0; a < 6; ++a) dp[6 * ka + a] = d[15 * ka + a];
        fail = back_substitute(P, B, active, lambda, dp, dl);
    }
    free(Sv); free(rv); free(S); free(dp);
    return fail;
}

typedef struct {
    double *V, *BG, *BA;
} vi_states_t;

static int vi_lm_round(const ref_problem *P, const ref_options *O, const ref_inertial *I, int round, int iters,
                       const uint8_t *active, int robust, double *T, double *X, vi_states_t *S, blocks_t *B,
                       double *F_out, double *lambda_out, int *trials_total, int *terminated, ref_logrec *log,
                       int log_cap, int *log_n) {
    int n = 15 * B->Kopt, K = B->K;
    double *Hi = (double *)malloc(sizeof(double) * ((size_t)n * n + 1));
    double *bi = (double *)malloc(sizeof(double) * (n + 1));
    double *d = (double *)malloc(sizeof(double) * (n + 1));
    double *dl = (double *)malloc(sizeof(double) * (3 * B->M + 1));
    double *T2 = (double *)malloc(sizeof(double) * (12 * K + 1));
    double *X2 = (double *)malloc(sizeof(double) * (3 * B->M + 1));
    double *dp = (double *)malloc(sizeof(double) * (6 * B->Kopt + 1));
    double *V2 = (double *)malloc(sizeof(double) * (3 * K + 1));
    double *G2 = (double *)malloc(sizeof(double) * (3 * K + 1));
    double *A2 = (double *)malloc(sizeof(double) * (3 * K + 1));
    double F = 0.0, lambda = 0.0, nu = 2.0;
    int done = 0;
    *terminated = 0;
    for (int it = 0; it < iters; ++it) {
        /* linearise both parts at the current state */
        linearize(P, O, T, X, active, robust, B);
        memset(Hi, 0, sizeof(double) * n * n);
        memset(bi, 0, sizeof(double) * n);
        double Fi = vi_linearize(I, B->opt, n, T, S->V, S->BG, S->BA, Hi, bi);
        if (it == 0) {
            F = B->F + Fi;
            /* largest diagonal entry of the whole Gauss-Newton matrix */
            double md = 0.0;
            for (int k = 0; k < B->Kopt; ++k)
                for (int a = 0; a < 15; ++a) {
                    double v = Hi[(15 * k + a) * n + 15 * k + a];
                    if (a < 6) v += B->Hpp[k * 36 + a * 7];
                    md = fmax(md, v);
                }
            for (int j = 0; j < 3 * B->M; ++j) md = fmax(md, B->Hll[(j / 3) * 9 + (j % 3) * 4]);
            lambda = lbaref_initial_damping(O->tau, md);
            nu = 2.0;
        }
        int accepted = 0;
        for (int tr = 0; tr < O->max_trials; ++tr) {
            ++*trials_total;
            int fail = vi_step(P, B, active, lambda, Hi, bi, d, dl);
            double F2 = NAN, gain = NAN;
            if (!fail) {
                for (int k = 0; k < B->Kopt; ++k)
                    for (int a = 0; a < 6; ++a) dp[6 * k + a] = d[15 * k + a];
                retract(B, T, X, dp, dl, T2, X2);
                for (int k = 0; k < K; ++k) {
                    int ok = B->opt[k];
                    for (int a = 0; a < 3; ++a) {
                        V2[3 * k + a] = S->V[3 * k + a] + (ok >= 0 ? d[15 * ok + 6 + a] : 0.0);
                        G2[3 * k + a] = S->BG[3 * k + a] + (ok >= 0 ? d[15 * ok + 9 + a] : 0.0);
                        A2[3 * k + a] = S->BA[3 * k + a] + (ok >= 0 ? d[15 * ok + 12 + a] : 0.0);
                    }
                }
                F2 = lbaref_cost(P, O, T2, X2, active, robust) + lbaref_vi_cost(I, T2, V2, G2, A2);
                /* predicted decrease d^T (lambda d + b), b = visual + inertial gradient */
                double den = 0.0;
                for (int k = 0; k < B->Kopt; ++k)
                    for (int a = 0; a < 15; ++a) {
                        double g = bi[15 * k + a] + (a < 6 ? B->bp[6 * k + a] : 0.0);
                        double x = d[15 * k + a];
                        den += x * (lambda * x + g);
                    }
                for (int q = 0; q < 3 * B->M; ++q) den += dl[q] * (lambda * dl[q] + B->bl[q]);
                gain = (F - F2) / den;
            }
            int acc = !fail && isfinite(F2) && isfinite(gain) && gain > 0.0;
            if (log && *log_n < log_cap) {
                ref_logrec *L = &log[(*log_n)++];
                L->round = round; L->iter = it; L->trial = tr; L->accepted = acc;
                L->solve_ok = !fail; L->pad = 0;
                L->lambda = lambda; L->F = F; L->F_trial = F2; L->gain = gain;
            }
            lbaref_damping_update(gain, acc, &lambda, &nu);
            if (acc) {
                memcpy(T, T2, sizeof(double) * 12 * K);
                memcpy(X, X2, sizeof(double) * 3 * B->M);
                memcpy(S->V, V2, sizeof(double) * 3 * K);
                memcpy(S->BG, G2, sizeof(double) * 3 * K);
                memcpy(S->BA, A2, sizeof(double) * 3 * K);
                F = F2;
                accepted = 1;
                break;
            }
        }
        if (!accepted) {
            *terminated = 1;
            break;
        }
        ++done;
    }
    if (iters == 0) F = lbaref_cost(P, O, T, X, active, robust) + lbaref_vi_cost(I, T, S->V, S->BG, S->BA);
    *F_out = F;
    lambda_out[0] = lambda;
    free(Hi); free(bi); free(d); free(dl); free(T2); free(X2); free(dp); free(V2); free(G2); free(A2);
    return done;
}

/* Full stereo-inertial solve: the schedule of lbaref_solve (round 1, outlier pass on the
 * reprojection terms, round 2, final flags) on the joint cost.  V/BG/BA in: n_kf x 3
 * each, overwritten with the result.  stats as lbaref_solve (costs include the inertial
 * terms).  Returns 0, or -1 for invalid input. */
int lbaref_solve_vi(const ref_problem *P, const ref_options *O, const ref_inertial *I, double *T_out,
                    double *X_out, double *V, double *BG, double *BA, uint8_t *outlier_out, double *stats,
                    ref_logrec *log, int log_cap, int *log_n) {
    for (int i = 0; i < P->n_obs; ++i) {
        if (P->obs_kf[i] < 0 || P->obs_kf[i] >= P->n_kf) return -1;
        if (P->obs_pt[i] < 0 || P->obs_pt[i] >= P->n_pt) return -1;
        if (P->obs_oct[i] >= P->n_levels) return -1;
    }
    for (int e = 0; e < I->n_edges; ++e)
        if (I->edge_i[e] < 0 || I->edge_i[e] >= P->n_kf || I->edge_j[e] < 0 || I->edge_j[e] >= P->n_kf ||
            I->edge_i[e] == I->edge_j[e])
            return -1;
    int ln = 0;
    if (!log_n) log_n = &ln;
    *log_n = 0;
    memcpy(T_out, P->T_cw, sizeof(double) * 12 * P->n_kf);
    memcpy(X_out, P->X_w, sizeof(double) * 3 * P->n_pt);
    vi_states_t S = {V, BG, BA};
    blocks_t B;
    blocks_alloc(&B, P);
    double F0 = lbaref_cost(P, O, T_out, X_out, NULL, 1) + lbaref_vi_cost(I, T_out, V, BG, BA);
    double F1 = F0, F2, lam1 = 0.0, lam2 = 0.0;
    int trials = 0, term1 = 0, term2 = 0;
    int it1 = vi_lm_round(P, O, I, 1, O->iters_round1, NULL, 1, T_out, X_out, &S, &B, &F1, &lam1, &trials, &term1,
                          log, log_cap, log_n);
    uint8_t *active = (uint8_t *)malloc((size_t)P->n_obs + 1);
    lbaref_flags(P, O, T_out, X_out, outlier_out);
    for (int i = 0; i < P->n_obs; ++i) active[i] = !outlier_out[i];
    double F20 = lbaref_cost(P, O, T_out, X_out, active, O->round2_robust) + lbaref_vi_cost(I, T_out, V, BG, BA);
    int it2 = vi_lm_round(P, O, I, 2, O->iters_round2, active, O->round2_robust, T_out, X_out, &S, &B, &F2, &lam2,
                          &trials, &term2, log, log_cap, log_n);
    lbaref_flags(P, O, T_out, X_out, outlier_out);
    int nout = 0;
    for (int i = 0; i < P->n_obs; ++i) nout += outlier_out[i];
    if (stats) {
        stats[0] = F0; stats[1] = F2; stats[2] = it1; stats[3] = it2; stats[4] = trials;
        stats[5] = O->iters_round2 > 0 ? lam2 : lam1; stats[6] = term1; stats[7] = term2;
        stats[8] = nout; stats[9] = F1; stats[10] = F20; stats[11] = B.Kopt;
    }
    free(active);
    blocks_free(&B);
    return 0;
}

/* The damped visual-inertial step at a state, for pinning (d: 15 Kopt, dl: 3 M; cost and
 * largest diagonal entry in Fmd[0], Fmd[1]).  Returns 0 or 1 (factorisation failed). */
int lbaref_vi_system_step(const ref_problem *P, const ref_options *O, const ref_inertial *I, const double *T,
                          const double *X, const double *V, const double *BG, const double *BA, double lambda,
                          double *d, double *dl, double *Fmd) {
    blocks_t B;
    blocks_alloc(&B, P);
    linearize(P, O, T, X, NULL, 1, &B);
    int n = 15 * B.Kopt;
    double *Hi = (double *)calloc((size_t)n * n + 1, sizeof(double));
    double *bi = (double *)calloc(n + 1, sizeof(double));
    double Fi = vi_linearize(I, B.opt, n, T, V, BG, BA, Hi, bi);
    Fmd[0] = B.F + Fi;
    int fail = vi_step(P, &B, NULL, lambda, Hi, bi, d, dl);
    free(Hi); free(bi);
    blocks_free(&B);
    return fail;
}
