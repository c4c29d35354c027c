/*
 * lmap.h -- C ABI of the local-mapping searches in liblba.so: the GPU-resident keyframe
 * store, the keypoint correspondence search of map-point creation, the candidate search
 * of map-point fusion, and the per-scale observation counters of keyframe culling.
 *
 * The operations (paper Section III "Local Mapping": A "Map-point Creation", B
 * "Map-point Fusion", D "Local Keyframe Culling"; Section IV-B "Keyframe Storage", IV-C
 * "Keypoint Correspondence Search", IV-D "Map-point Fusion", IV-F "Local Keyframe
 * Culling"):
 *
 *   keyframe store   the immutable per-keyframe data (pose, keypoints, octaves, 256-bit
 *                    binary descriptors) kept in device memory for as long as the
 *                    keyframe lives; the mutable data (which keypoints already carry a
 *                    map point) is passed per call.  lmap_index_build derives, once per
 *                    keyframe, what the searches read: the descriptors as 256 signed
 *                    bytes (+1 for a set bit, -1 for a clear one) and the keypoints
 *                    sorted into 16x16-pixel cells.
 *
 *   correspondence   for keypoint i of the current keyframe c that has no map point yet
 *                    and a neighbour keyframe n: the keypoint j of n, also without a map
 *                    point, of smallest descriptor distance d <= th_low whose position
 *                    passes the epipolar test (squared distance of x_j to the epipolar
 *                    line of x_i below epi_chi2 * sigma2[octave_j]) and, when both
 *                    keypoints are monocular (uR < 0), the epipole test (squared
 *                    distance of x_j to the epipole of c in n at least
 *                    epipole_min * scale[octave_j]); ties go to the smaller j.  With
 *                    resolve set, a keypoint j chosen by several i keeps only the i of
 *                    smallest d (ties: smaller i).  Triangulation is left to the caller.
 *
 *   fusion           for map point p and neighbour keyframe n: project p into n (depth
 *                    > 0, inside the image), require its distance to n's centre within
 *                    [dmin, dmax] and a viewing angle below 60 degrees to its mean
 *                    viewing direction (dot > 0 and dot^2 >= d2 / 4), predict the octave
 *                    l (the smallest with scale[l]^2 d2 >= dmax^2, at most the last),
 *                    and take, among n's keypoints within radius_th * scale[l] pixels
 *                    in u and in v with octave l - 1 or l whose reprojection error
 *                    passes e^2 <= chi2 * sigma2[octave] (stereo keypoints with their
 *                    right coordinate), the one of smallest descriptor distance
 *                    d <= th_low (ties: smaller index).  The fuse itself is left to the
 *                    caller, after the search.
 *
 *   culling          per map point the number of active observations at each octave; an
 *                    observation (k, j, o) is redundant when at least min_obs other
 *                    active observations of j have octave <= o + slack; keyframe k is
 *                    culled (unless protected) when it has active observations and
 *                    den * redundant >= num * observations.
 *
 * Every decision that floating point takes (the geometric tests) is taken in FP64 on
 * the FP32 keypoint coordinates converted exactly, with the operations in the order the
 * formulas above are written (products left to right, sums left to right, no fused
 * multiply-add), so results are reproducible bit for bit.  Descriptor distances are
 * exact integers.
 *
 * Memory: every array is caller-owned.  DEVICE arrays live in device memory of the
 * current HIP device (e.g. torch tensors); HOST arrays are small per-call constants.  All
 * work is enqueued on the caller's HIP stream.  With check set, the inputs are validated
 * on the GPU first and the stream is synchronised once to read the verdict
 * (LMAP_ERR_INVALID_ARGUMENT with a message); with check 0 nothing synchronises, and
 * the kernels skip queries and observations whose indices are out of range, leaving
 * their outputs undefined, without reading or writing outside the arrays; the store
 * itself (kp_off, octaves) must then be valid, as a checked lmap_index_build found it.  No entry point throws;
 * lmap_last_error() gives the message of the calling thread's last failure.
 */
#ifndef LMAP_H
#define LMAP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LMAP_ABI_VERSION 1
#define LMAP_CELL_PX 16          /* side of a keypoint cell of the index, pixels */
#define LMAP_MAX_CELLS 8192      /* cells per keyframe image */
#define LMAP_MAX_KP (1 << 22)    /* keypoints per keyframe */

typedef enum {
    LMAP_OK = 0,
    LMAP_ERR_INVALID_ARGUMENT = -1,
    LMAP_ERR_HIP = -3,
    LMAP_ERR_WORKSPACE_TOO_SMALL = -4,
    LMAP_ERR_UNSUPPORTED = -5
} lmap_status;

/* The keyframe store.  Keypoints of keyframe k are [kp_off[k], kp_off[k + 1]). */
typedef struct {
    int32_t n_kf;            /* keyframes */
    int32_t n_kp;            /* keypoints over all keyframes */
    int32_t max_kp;          /* most keypoints of one keyframe (sizes the launches), 1..LMAP_MAX_KP */
    int32_t n_levels;        /* octaves, 1..32 */
    int32_t width, height;   /* image size in pixels (the fusion projection must fall inside) */
    const int32_t *kp_off;   /* DEVICE n_kf + 1, non-decreasing, kp_off[0] = 0, kp_off[n_kf] = n_kp */
    const double *T_cw;      /* DEVICE n_kf x 12, row-major [R | t], world -> camera */
    const float *kp_u;       /* DEVICE n_kp, left-image column (finite) */
    const float *kp_v;       /* DEVICE n_kp, row (finite) */
    const float *kp_ur;      /* DEVICE n_kp, right-image column; negative: monocular keypoint */
    const uint8_t *kp_oct;   /* DEVICE n_kp, octave < n_levels */
    const uint32_t *kp_desc; /* DEVICE n_kp x 8, 256-bit descriptors (bit b of word w is bit 32w + b) */
    void *index;             /* DEVICE lmap_index_size bytes, 256-byte aligned: written by
                                lmap_index_build, read by the searches */
    const double *sigma2;    /* HOST n_levels, keypoint position variance per octave (px^2) */
    const double *scale;     /* HOST n_levels, scale factor per octave */
    double fx, fy, cx, cy;   /* pinhole intrinsics, pixels */
    double bf;               /* stereo baseline times fx (px * m) */
} lmap_store;

typedef struct {
    int32_t th_low;          /* largest accepted descriptor distance, 0..256 [50] */
    int32_t resolve;         /* 1: a keypoint of n chosen twice keeps the closest [1] */
    double epi_chi2;         /* epipolar test [3.84] */
    double epipole_min;      /* epipole test [100] */
} lmap_corr_params;

typedef struct {
    int32_t th_low;          /* [50] */
    int32_t reserved;
    double radius_th;        /* search radius factor [3.0] */
    double chi2_mono;        /* [5.991] */
    double chi2_stereo;      /* [7.815] */
} lmap_fuse_params;

/* Map points of the fusion search, all DEVICE, n_pt entries each. */
typedef struct {
    int32_t n_pt;
    int32_t reserved;
    const double *X;         /* n_pt x 3, world position */
    const double *normal;    /* n_pt x 3, mean viewing direction (unit) */
    const double *dmin;      /* n_pt, distance range of scale invariance */
    const double *dmax;
    const uint32_t *desc;    /* n_pt x 8, representative descriptor */
} lmap_points;

typedef struct {
    int32_t min_obs;         /* other observations needed at the same or finer scale [3] */
    int32_t slack;           /* octaves of slack [0] */
    int32_t num, den;        /* culling ratio num/den [9, 10] */
} lmap_cull_params;

int32_t lmap_abi_version(void);
const char *lmap_status_string(lmap_status status);
/* Message of the calling thread's last failure ("" if none). */
const char *lmap_last_error(void);
void lmap_default_corr_params(lmap_corr_params *p);
void lmap_default_fuse_params(lmap_fuse_params *p);
void lmap_default_cull_params(lmap_cull_params *p);

/* ---- keyframe store index (Section IV-B) ------------------------------------------------
 * Bytes of the store's index: n_kp x 256 (signed-byte descriptors) + n_kf x (cells + 1) x 4
 * (cell offsets) + n_kp x 4 (keypoints by cell) + 256 (validation verdict), each part
 * 256-byte aligned. */
lmap_status lmap_index_size(const lmap_store *store, size_t *bytes);
/* Build the index entries of keyframes [k0, k1) (their keypoints, descriptors and
 * kp_off entries must already be in place): a keyframe entering the store costs one
 * call over its own range.  Within a cell, keypoints are in increasing order. */
lmap_status lmap_index_build(const lmap_store *store, int32_t k0, int32_t k1, size_t index_bytes,
                             int32_t check, void *stream);

/* ---- keypoint correspondence search (Sections III-A, IV-C) -------------------------------
 * n_q queries (cur[q], nbr[q]), DEVICE arrays.  kp_free: DEVICE n_kp, 1 = the keypoint
 * has no map point yet.  Outputs of query q are the entries out_off[q] ..
 * out_off[q + 1] - 1 of match and dist (DEVICE, n_out entries each), one per keypoint of
 * cur[q] in order: match = index within nbr[q] of the chosen keypoint, or -1; dist = its
 * descriptor distance, or -1.  out_off (DEVICE n_q + 1) must be the running sum of the
 * keypoint counts of cur[q], starting at 0, with out_off[n_q] <= n_out.  The workspace
 * (DEVICE, 256-byte aligned) holds the per-query geometry, the free-keypoint lists and
 * the resolution keys; its size is lmap_corr_workspace_size. */
lmap_status lmap_corr_workspace_size(const lmap_store *store, int32_t n_q, size_t *bytes);
lmap_status lmap_correspondence(const lmap_store *store, const lmap_corr_params *params,
                                const uint8_t *kp_free, int32_t n_q, const int32_t *cur,
                                const int32_t *nbr, const int64_t *out_off, int64_t n_out,
                                int32_t *match, int32_t *dist, void *workspace,
                                size_t workspace_bytes, int32_t check, void *stream);

/* ---- correspondence search without allocation ---------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): lmap_correspondence with its workspace
 * in a static device array of LMAP_NOALLOC_SCRATCH_BYTES on each GPU, which the library
 * holds until the process ends; nothing is allocated or freed.  A problem whose
 * lmap_corr_workspace_size exceeds that size returns LMAP_ERR_WORKSPACE_TOO_SMALL.  Every
 * call on a GPU shares that GPU's array, and each call sets what must start cleared:
 * calls that overlap on one GPU (other streams or threads) race and must be ordered by
 * the caller.  The array's device address is looked up on the first call on each device,
 * which must then be the current device.  With check set the call synchronises the
 * stream once (under graph capture, pass 0). */
#define LMAP_NOALLOC_SCRATCH_BYTES (16u << 20)
lmap_status lmap_correspondence_noalloc(const lmap_store *store, const lmap_corr_params *params,
                                        const uint8_t *kp_free, int32_t n_q, const int32_t *cur,
                                        const int32_t *nbr, const int64_t *out_off, int64_t n_out,
                                        int32_t *match, int32_t *dist, int32_t check, void *stream);

/* ---- fusion candidate search (Sections III-B, IV-D) --------------------------------------
 * n_q queries: map points [p0[q], p1[q]) against keyframe nbr[q] (DEVICE arrays).  One
 * output entry per (query, point), from out_off[q] on (DEVICE n_q + 1, running sum of
 * p1 - p0 from 0, out_off[n_q] <= n_out): match = index within nbr[q] of the chosen
 * keypoint or -1, dist = its distance or -1.  skip: DEVICE n_out or NULL, 1 = the point
 * already has an observation in nbr[q] (entry left at -1).  max_len: HOST hint, the
 * longest point range of one query (sizes the launch; any value >= 1 is correct).
 * The workspace holds the validation verdict: lmap_fuse_workspace_size bytes. */
lmap_status lmap_fuse_workspace_size(size_t *bytes);
lmap_status lmap_fusion(const lmap_store *store, const lmap_fuse_params *params,
                        const lmap_points *points, int32_t n_q, const int32_t *p0,
                        const int32_t *p1, const int32_t *nbr, const int64_t *out_off,
                        int64_t n_out, int32_t max_len, const uint8_t *skip, int32_t *match,
                        int32_t *dist, void *workspace, size_t workspace_bytes,
                        int32_t check, void *stream);

/* ---- keyframe-culling counters (Sections III-D, IV-F) ------------------------------------
 * Observations (obs_kf[i], obs_pt[i], obs_oct[i]) in any order, with indices into
 * [0, n_kf) and [0, n_pt) (a batch of windows is one problem with global indices).
 * active: DEVICE n_obs or NULL (all active); protect: DEVICE n_kf or NULL.  Outputs
 * (DEVICE): counters n_pt x n_levels (observations per point per octave), kf_obs and
 * kf_red (n_kf: active and redundant observations per keyframe), cull (n_kf, 1 =
 * redundant keyframe).  Counts are integers summed with atomic adds, so they are exact
 * and independent of the order.  Workspace: lmap_cull_workspace_size bytes. */
lmap_status lmap_cull_workspace_size(size_t *bytes);
lmap_status lmap_culling(int32_t n_kf, int32_t n_pt, int32_t n_obs, int32_t n_levels,
                         const int32_t *obs_kf, const int32_t *obs_pt, const uint8_t *obs_oct,
                         const uint8_t *active, const uint8_t *protect,
                         const lmap_cull_params *params, int32_t *counters, int32_t *kf_obs,
                         int32_t *kf_red, uint8_t *cull, void *workspace, size_t workspace_bytes,
                         int32_t check, void *stream);

/* ---- per-kernel timing ------------------------------------------------------------------
 * With profiling enabled (process-wide), every kernel the searches launch is bracketed by
 * two HIP events on the caller's stream; at the end of each call the stream is
 * synchronised and the durations are added to the counters of the kernel's class.
 * Enabling resets the counters. */
typedef enum {
    LMAP_KCLASS_INDEX = 0,        /* index build: signed-byte descriptors and cells */
    LMAP_KCLASS_PREP,             /* output fills, per-query geometry, free-keypoint lists */
    LMAP_KCLASS_CORR_SEARCH,      /* correspondence search (matrix cores + validation) */
    LMAP_KCLASS_CORR_RESOLVE,     /* deferred resolution of the correspondence search */
    LMAP_KCLASS_FUSE,             /* fusion candidate search */
    LMAP_KCLASS_CULL_COUNT,       /* per-point per-octave counters */
    LMAP_KCLASS_CULL_REDUNDANT,   /* redundancy test and per-keyframe totals */
    LMAP_KCLASS_CULL_DECIDE,      /* per-keyframe decision */
    LMAP_KCLASS_CHECK,            /* input validation */
    LMAP_KCLASS_COUNT
} lmap_kernel_class;

lmap_status lmap_profile_enable(int32_t enable);
lmap_status lmap_profile_read(int32_t kernel_class, int64_t *launches, double *total_ms);

#ifdef __cplusplus
}
#endif

#endif /* LMAP_H */
