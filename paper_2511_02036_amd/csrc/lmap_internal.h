// Internal definitions of the local-mapping searches (keyframe-store index,
// correspondence search, fusion candidate search, culling counters): kernel argument
// packs, the index and workspace layouts, and the launchers each kernel file exports.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lmap.h"

namespace lmap {

constexpr int kMaxLevels = 32;
constexpr int kCell = LMAP_CELL_PX;
constexpr int kDescBytes = 256;          // one descriptor as signed bytes
constexpr int kKpBits = 22;              // resolution keys: distance << 22 | index
constexpr uint32_t kKpMask = (1u << kKpBits) - 1u;
constexpr int kCorrRows = 256;           // free keypoints of the current keyframe per block

// validation verdict words in the workspace (each a count of offending entries)
enum {
    kErrKpOff = 0, kErrOct, kErrCoord, kErrQuery, kErrOutOff, kErrPoint, kErrObs, kErrCount = 8
};

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

inline int grid_cols(int width) { return (width + kCell - 1) / kCell; }
inline int grid_rows(int height) { return (height + kCell - 1) / kCell; }

// Byte offsets of the parts of a store's index.
struct IndexLayout {
    int ncx, ncy, ncells;
    size_t o_desc, o_celloff, o_cellkp, o_err, total;
};

inline IndexLayout index_layout(const lmap_store &s) {
    IndexLayout L;
    L.ncx = grid_cols(s.width);
    L.ncy = grid_rows(s.height);
    L.ncells = L.ncx * L.ncy;
    L.o_desc = 0;
    L.o_celloff = align256((size_t)s.n_kp * kDescBytes);
    L.o_cellkp = L.o_celloff + align256((size_t)s.n_kf * (L.ncells + 1) * sizeof(int32_t));
    L.o_err = L.o_cellkp + align256((size_t)s.n_kp * sizeof(int32_t));
    L.total = L.o_err + 256;
    return L;
}

// Device view of the store, passed by value to every search kernel.
struct StoreView {
    const int32_t *kp_off;
    const double *T;
    const float *u, *v, *ur;
    const uint8_t *oct;
    const uint32_t *desc;
    int8_t *desc_pm;           // n_kp x 256 signed bytes
    int32_t *cell_off;         // n_kf x (ncells + 1), offsets within the keyframe's keypoints
    int32_t *cell_kp;          // n_kp: keypoint (local index) in cell order, per keyframe
    int32_t n_kf, n_kp, max_kp, n_levels, width, height, ncx, ncy, ncells, pad;
    double fx, fy, cx, cy, bf;
    double sigma2[kMaxLevels];
    double scale[kMaxLevels];
};

struct CorrArgs {
    StoreView s;
    const uint8_t *kp_free;
    const int32_t *cur, *nbr;
    const int64_t *out_off;
    int64_t n_out;
    int32_t *match, *dist;
    double *geo;               // per query: F (9), epipole (2), 1 spare
    int32_t *qok;              // per query: 1 = indices valid
    int32_t *free_idx;         // per keyframe, at kp_off: local indices of the free keypoints
    int32_t *free_cnt;         // per keyframe
    uint32_t *owner;           // per query x max_kp: resolution key of each keypoint of nbr
    int32_t *err;
    int32_t n_q, th_low, resolve, blocks_per_q;
    double epi_chi2, epipole_min;
};

struct FuseArgs {
    StoreView s;
    const double *X, *normal, *dmin, *dmax;
    const uint32_t *pdesc;
    const int32_t *p0, *p1, *nbr;
    const int64_t *out_off;
    const uint8_t *skip;
    int32_t *match, *dist;
    int32_t *err;
    int64_t n_out;
    int32_t n_pt, n_q, th_low, blocks_per_q;
    double radius_th, chi2_mono, chi2_stereo;
};

struct CullArgs {
    const int32_t *kf, *pt;
    const uint8_t *oct, *active, *protect;
    int32_t *counters, *kf_obs, *kf_red;
    uint8_t *cull;
    int32_t *err;
    int32_t n_kf, n_pt, n_obs, n_levels, min_obs, slack, num, den;
};

// Per-kernel timing hooks (lmap_api.hip): no-ops unless profiling is enabled.
void prof_begin(int kernel_class, hipStream_t s);
void prof_end(hipStream_t s);

// launchers (k_lmap_index.hip, k_corr.hip, k_fuse.hip, k_cull.hip)
void launch_fill_i32(int32_t *p, int64_t n, int32_t value, hipStream_t s);
void launch_index_check(const StoreView &v, int32_t k0, int32_t k1, int32_t *err, hipStream_t s);
void launch_index_build(const StoreView &v, int32_t k0, int32_t k1, hipStream_t s);
void launch_corr_check(const CorrArgs &a, hipStream_t s);
void launch_corr(const CorrArgs &a, hipStream_t s);
void launch_fuse_check(const FuseArgs &a, hipStream_t s);
void launch_fuse(const FuseArgs &a, hipStream_t s);
void launch_cull_check(const CullArgs &a, hipStream_t s);
void launch_cull(const CullArgs &a, hipStream_t s);

}  // namespace lmap
