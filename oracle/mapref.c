/*
 * mapref.c -- plain CPU oracle for the data-parallel local-mapping stages around local
 * bundle adjustment: the keypoint correspondence search of map-point creation (paper
 * Section III-A "Map-point Creation", Section IV-C "Keypoint Correspondence Search"), the
 * candidate search of map-point fusion (Section III-B "Map-point Fusion", Section IV-D
 * "Map-point Fusion") and the per-scale observation counters of keyframe culling
 * (Section III-D "Local Keyframe Culling", Section IV-F).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite and the benchmark's CPU-baseline leg load
 * this library; the product path never does.  It shares no code, header, table or helper
 * with the GPU library.
 *
 * The paper describes these stages in words only; the concrete tests are this project's
 * reading, written after the ORB-SLAM local-mapping conventions the paper builds on:
 *
 *   descriptor distance   Hamming distance of two 256-bit binary descriptors
 *   correspondence        for keypoint i of the current keyframe c (no map point yet) and a
 *                         neighbour keyframe n, the keypoint j of n (no map point yet) with
 *                         the smallest distance d <= th_low whose position passes
 *                           - the epipolar test: squared distance of x_j to the line F x_i
 *                             below epi_chi2 * sigma2[octave_j] (F: x_n^T F x_c = 0);
 *                           - the epipole test (both keypoints monocular): squared distance
 *                             of x_j to the epipole (centre of c seen from n) at least
 *                             epipole_min * scale[octave_j];
 *                         ties go to the smaller j.  Deferred resolution: a keypoint j chosen
 *                         by several i keeps the i of smallest distance (ties: smaller i).
 *   fusion candidate      for map point p and neighbour keyframe n: project p into n (depth
 *                         > 0, inside the image), require its distance to n's centre within
 *                         [dmin, dmax] and the angle between the viewing ray and the point's
 *                         mean viewing direction below 60 degrees, predict the octave l as
 *                         the smallest with scale[l]^2 dist^2 >= dmax^2 (at most the last),
 *                         and take, among n's keypoints within th * scale[l] pixels in u and
 *                         in v with octave l - 1 or l whose reprojection error passes
 *                         e^2 <= chi2 * sigma2[octave] (stereo keypoints with their right
 *                         coordinate), the one with the smallest descriptor distance <=
 *                         th_low (ties: smaller index).  The fuse itself is sequential and
 *                         deferred.
 *   culling counters      per map point the number of (active) observations at each
 *                         octave; an observation (k, j, o) is redundant when at least
 *                         min_obs other observations of j have an octave <= o + slack;
 *                         keyframe k is culled (unless protected) when it has observations
 *                         and den * redundant >= num * observations (at least num/den).
 *
 * Geometric decisions are taken in FP64 with the operations in a fixed order, compiled
 * without floating-point contraction.  Everything is single-threaded and written for
 * readability.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n_kf, n_kp, n_levels, width, height, pad;
    const int32_t *kp_off;      /* n_kf + 1 */
    const double *T_cw;         /* n_kf x 12, row-major [R | t], world -> camera */
    const float *kp_u, *kp_v;   /* n_kp */
    const float *kp_ur;         /* n_kp, right-image u, negative: monocular */
    const uint8_t *kp_oct;      /* n_kp */
    const uint8_t *kp_free;     /* n_kp, 1: no map point yet */
    const uint32_t *kp_desc;    /* n_kp x 8 */
    const double *sigma2;       /* n_levels */
    const double *scale;        /* n_levels */
    double fx, fy, cx, cy, bf;
} ref_store;

typedef struct {
    int32_t th_low;             /* largest accepted descriptor distance [50] */
    int32_t resolve;            /* 1: deferred resolution of keypoints chosen twice */
    double epi_chi2;            /* epipolar test [3.84] */
    double epipole_min;         /* epipole test [100] */
} ref_corr_params;

typedef struct {
    int32_t th_low;             /* [50] */
    int32_t pad;
    double radius_th;           /* search radius factor [3.0] */
    double chi2_mono, chi2_stereo;   /* [5.991, 7.815] */
} ref_fuse_params;

/* Hamming distance of two 256-bit descriptors, bit by bit. */
int mapref_hamming(const uint32_t *a, const uint32_t *b) {
    int d = 0;
    for (int w = 0; w < 8; ++w) {
        uint32_t x = a[w] ^ b[w];
        for (int bit = 0; bit < 32; ++bit) d += (x >> bit) & 1u;
    }
    return d;
}

/* C = A B for 3x3 row-major matrices, each entry summed over k = 0, 1, 2 in order. */
static void mul33(const double *A, const double *B, double *C) {
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double s = A[i * 3 + 0] * B[0 * 3 + j];
            s = s + A[i * 3 + 1] * B[1 * 3 + j];
            s = s + A[i * 3 + 2] * B[2 * 3 + j];
            C[i * 3 + j] = s;
        }
}

/* Fundamental matrix from keyframe a to keyframe b: x_b^T F x_a = 0 for the two pixels of
 * one 3-D point.  With the pose of b relative to a, R = R_b R_a^T and t = t_b - R t_a,
 * the essential matrix is E = [t]x R and F = K^-T E K^-1 (Hartley & Zisserman, "Multiple
 * View Geometry", 2nd ed., Section 9.6). */
void mapref_fundamental(const ref_store *S, int a, int b, double F[9]) {
    const double *Ta = S->T_cw + 12 * a, *Tb = S->T_cw + 12 * b;
    double Rb[9], RaT[9], R[9], t[3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            Rb[i * 3 + j] = Tb[i * 4 + j];
            RaT[j * 3 + i] = Ta[i * 4 + j];
        }
    mul33(Rb, RaT, R);
    for (int i = 0; i < 3; ++i) {
        double s = R[i * 3 + 0] * Ta[3];
        s = s + R[i * 3 + 1] * Ta[7];
        s = s + R[i * 3 + 2] * Ta[11];
        t[i] = Tb[i * 4 + 3] - s;
    }
    const double tx[9] = {0.0, -t[2], t[1], t[2], 0.0, -t[0], -t[1], t[0], 0.0};
    double E[9], KiT[9], Ki[9], KE[9];
    const double ifx = 1.0 / S->fx, ify = 1.0 / S->fy;
    const double k02 = -S->cx / S->fx, k12 = -S->cy / S->fy;
    const double Kinv[9] = {ifx, 0.0, k02, 0.0, ify, k12, 0.0, 0.0, 1.0};
    for (int i = 0; i < 9; ++i) Ki[i] = Kinv[i];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) KiT[i * 3 + j] = Kinv[j * 3 + i];
    mul33(tx, R, E);
    mul33(KiT, E, KE);
    mul33(KE, Ki, F);
}

/* Epipole of keyframe a in keyframe b: the projection of a's camera centre. */
void mapref_epipole(const ref_store *S, int a, int b, double e[2]) {
    const double *Ta = S->T_cw + 12 * a, *Tb = S->T_cw + 12 * b;
    double C[3], X[3];
    for (int i = 0; i < 3; ++i) {   /* C = -R_a^T t_a */
        double s = Ta[0 * 4 + i] * Ta[3];
        s = s + Ta[1 * 4 + i] * Ta[7];
        s = s + Ta[2 * 4 + i] * Ta[11];
        C[i] = -s;
    }
    for (int i = 0; i < 3; ++i) {
        double s = Tb[i * 4 + 0] * C[0];
        s = s + Tb[i * 4 + 1] * C[1];
        s = s + Tb[i * 4 + 2] * C[2];
        X[i] = s + Tb[i * 4 + 3];
    }
    e[0] = S->fx * X[0] / X[2] + S->cx;
    e[1] = S->fy * X[1] / X[2] + S->cy;
}

/* Squared distance of pixel (ub, vb) of keyframe b to the epipolar line F (ua, va, 1);
 * returns -1 when the line is degenerate (both direction coefficients zero). */
double mapref_epipolar_dist2(const double F[9], double ua, double va, double ub, double vb) {
    const double l0 = (F[0] * ua + F[1] * va) + F[2];
    const double l1 = (F[3] * ua + F[4] * va) + F[5];
    const double l2 = (F[6] * ua + F[7] * va) + F[8];
    const double num = (l0 * ub + l1 * vb) + l2;
    const double den = l0 * l0 + l1 * l1;
    if (den == 0.0) return -1.0;
    return num * num / den;
}

/*
 * Correspondence search for n_q queries (cur[q], nbr[q]).  Outputs for query q start at
 * out_off[q] and hold one entry per keypoint of cur[q] (in keypoint order): match = index
 * of the chosen keypoint within nbr[q], or -1; dist = its descriptor distance, or -1.
 */
void mapref_correspondence(const ref_store *S, const ref_corr_params *P, int n_q, const int32_t *cur,
                           const int32_t *nbr, const int64_t *out_off, int32_t *match, int32_t *dist) {
    for (int q = 0; q < n_q; ++q) {
        const int c = cur[q], n = nbr[q];
        double F[9], ep[2];
        mapref_fundamental(S, c, n, F);
        mapref_epipole(S, c, n, ep);
        const int i0 = S->kp_off[c], i1 = S->kp_off[c + 1];
        const int j0 = S->kp_off[n], j1 = S->kp_off[n + 1];
        int32_t *mo = match + out_off[q], *dout = dist + out_off[q];
        for (int i = i0; i < i1; ++i) {
            int best = -1, bd = P->th_low + 1;
            if (S->kp_free[i]) {
                const double ua = S->kp_u[i], va = S->kp_v[i];
                const int mono_a = S->kp_ur[i] < 0.0f;
                for (int j = j0; j < j1; ++j) {
                    if (!S->kp_free[j]) continue;
                    const int d = mapref_hamming(S->kp_desc + 8 * (size_t)i, S->kp_desc + 8 * (size_t)j);
                    if (d > P->th_low || d >= bd) continue;
                    const int o = S->kp_oct[j];
                    const double ub = S->kp_u[j], vb = S->kp_v[j];
                    if (mono_a && S->kp_ur[j] < 0.0f) {
                        const double dx = ep[0] - ub, dy = ep[1] - vb;
                        if (dx * dx + dy * dy < P->epipole_min * S->scale[o]) continue;
                    }
                    const double e2 = mapref_epipolar_dist2(F, ua, va, ub, vb);
                    if (e2 < 0.0 || !(e2 < P->epi_chi2 * S->sigma2[o])) continue;
                    best = j;
                    bd = d;
                }
            }
            mo[i - i0] = best < 0 ? -1 : best - j0;
            dout[i - i0] = best < 0 ? -1 : bd;
        }
        if (!P->resolve) continue;
        /* deferred resolution: each keypoint of n keeps the closest of the keypoints of c
         * that chose it (ties: the smaller index) */
        uint8_t *lose = (uint8_t *)calloc((size_t)(i1 - i0) + 1, 1);
        for (int i = 0; i < i1 - i0; ++i) {
            if (mo[i] < 0) continue;
            for (int k = 0; k < i1 - i0; ++k) {
                if (k == i || mo[k] != mo[i]) continue;
                if (dout[k] < dout[i] || (dout[k] == dout[i] && k < i)) {
                    lose[i] = 1;
                    break;
                }
            }
        }
        for (int i = 0; i < i1 - i0; ++i)
            if (lose[i]) {
                mo[i] = -1;
                dout[i] = -1;
            }
        free(lose);
    }
}

/*
 * Fusion candidate search for n_q queries (points [p0[q], p1[q]) against keyframe
 * nbr[q]).  Outputs for query q start at out_off[q], one entry per point of its range:
 * match = index of the chosen keypoint within nbr[q] or -1, dist = its distance or -1.
 * skip (or NULL): per output entry, 1 = the point already has an observation in nbr[q].
 */
void mapref_fusion(const ref_store *S, const ref_fuse_params *P, const double *X, const double *normal,
                   const double *dmin, const double *dmax, const uint32_t *pdesc, int n_q, const int32_t *p0,
                   const int32_t *p1, const int32_t *nbr, const int64_t *out_off, const uint8_t *skip,
                   int32_t *match, int32_t *dist) {
    for (int q = 0; q < n_q; ++q) {
        const int n = nbr[q];
        const double *T = S->T_cw + 12 * n;
        double O[3];
        for (int i = 0; i < 3; ++i) {   /* camera centre -R^T t */
            double s = T[0 * 4 + i] * T[3];
            s = s + T[1 * 4 + i] * T[7];
            s = s + T[2 * 4 + i] * T[11];
            O[i] = -s;
        }
        const int j0 = S->kp_off[n], j1 = S->kp_off[n + 1];
        for (int p = p0[q]; p < p1[q]; ++p) {
            const int64_t o_idx = out_off[q] + (p - p0[q]);
            match[o_idx] = -1;
            dist[o_idx] = -1;
            if (skip && skip[o_idx]) continue;
            const double *Xp = X + 3 * (size_t)p;
            double Xc[3];
            for (int i = 0; i < 3; ++i) {
                double s = T[i * 4 + 0] * Xp[0];
                s = s + T[i * 4 + 1] * Xp[1];
                s = s + T[i * 4 + 2] * Xp[2];
                Xc[i] = s + T[i * 4 + 3];
            }
            if (!(Xc[2] > 0.0)) continue;
            const double iz = 1.0 / Xc[2];
            const double u = S->fx * Xc[0] * iz + S->cx;
            const double v = S->fy * Xc[1] * iz + S->cy;
            if (!(u >= 0.0 && u < (double)S->width && v >= 0.0 && v < (double)S->height)) continue;
            const double ur = u - S->bf * iz;
            const double PO[3] = {Xp[0] - O[0], Xp[1] - O[1], Xp[2] - O[2]};
            const double d2 = (PO[0] * PO[0] + PO[1] * PO[1]) + PO[2] * PO[2];
            if (d2 < dmin[p] * dmin[p] || d2 > dmax[p] * dmax[p]) continue;
            const double *nv = normal + 3 * (size_t)p;
            const double dot = (PO[0] * nv[0] + PO[1] * nv[1]) + PO[2] * nv[2];
            if (!(dot > 0.0) || dot * dot < 0.25 * d2) continue;
            int level = 0;
            while (level < S->n_levels - 1 && S->scale[level] * S->scale[level] * d2 < dmax[p] * dmax[p]) ++level;
            const double radius = P->radius_th * S->scale[level];
            int best = -1, bd = P->th_low + 1;
            for (int j = j0; j < j1; ++j) {
                const double ku = S->kp_u[j], kv = S->kp_v[j];
                if (!(fabs(ku - u) < radius && fabs(kv - v) < radius)) continue;
                const int o = S->kp_oct[j];
                if (o < level - 1 || o > level) continue;
                const double ex = u - ku, ey = v - kv;
                if (S->kp_ur[j] >= 0.0f) {
                    const double er = ur - (double)S->kp_ur[j];
                    const double e2 = (ex * ex + ey * ey) + er * er;
                    if (e2 > P->chi2_stereo * S->sigma2[o]) continue;
                } else {
                    const double e2 = ex * ex + ey * ey;
                    if (e2 > P->chi2_mono * S->sigma2[o]) continue;
                }
                const int d = mapref_hamming(pdesc + 8 * (size_t)p, S->kp_desc + 8 * (size_t)j);
                if (d > P->th_low || d >= bd) continue;
                best = j;
                bd = d;
            }
            match[o_idx] = best < 0 ? -1 : best - j0;
            dist[o_idx] = best < 0 ? -1 : bd;
        }
    }
}

/*
 * Keyframe-culling counts on one window's observations (window-local indices).  active
 * (or NULL): 0 = observation left out (an outlier).  counters: n_pt x n_levels
 * observations per point per octave; kf_obs / kf_red: observations and redundant
 * observations per keyframe; cull: 1 = keyframe redundant (never for protect[k] = 1).
 * Each observation's count of other observations is taken directly over the point's
 * observations (the definition); the per-octave counters are returned beside it.
 */
void mapref_culling(int n_kf, int n_pt, int n_obs, int n_levels, const int32_t *obs_kf, const int32_t *obs_pt,
                    const uint8_t *obs_oct, const uint8_t *active, const uint8_t *protect, int min_obs, int slack,
                    int num, int den, int32_t *counters, int32_t *kf_obs, int32_t *kf_red, uint8_t *cull) {
    memset(counters, 0, sizeof(int32_t) * (size_t)n_pt * n_levels);
    memset(kf_obs, 0, sizeof(int32_t) * (size_t)n_kf);
    memset(kf_red, 0, sizeof(int32_t) * (size_t)n_kf);
    for (int a = 0; a < n_obs; ++a)
        if (!active || active[a]) counters[(size_t)obs_pt[a] * n_levels + obs_oct[a]] += 1;
    for (int a = 0; a < n_obs; ++a) {
        if (active && !active[a]) continue;
        kf_obs[obs_kf[a]] += 1;
        int others = 0;
        for (int b = 0; b < n_obs; ++b) {
            if (b == a || obs_pt[b] != obs_pt[a] || (active && !active[b])) continue;
            if (obs_oct[b] <= obs_oct[a] + slack) ++others;
        }
        if (others >= min_obs) kf_red[obs_kf[a]] += 1;
    }
    for (int k = 0; k < n_kf; ++k)
        cull[k] = (!protect || !protect[k]) && kf_obs[k] > 0 && (int64_t)den * kf_red[k] >= (int64_t)num * kf_obs[k];
}
