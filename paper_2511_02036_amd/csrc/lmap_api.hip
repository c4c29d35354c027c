// C ABI of the local-mapping searches (include/lmap.h): argument checks, workspace
// layout and launch sequencing.  The numerical work runs in k_lmap_index.hip,
// k_corr.hip, k_fuse.hip and k_cull.hip.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "lmap.h"
#include "lmap_internal.h"

using namespace lmap;

namespace {

thread_local std::string g_err;

lmap_status fail(lmap_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(call)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) return fail(LMAP_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

bool aligned256(const void *p) { return ((uintptr_t)p & 255) == 0; }

// Checks of the store's host-side fields; fills the device view.
lmap_status store_view(const lmap_store *s, bool need_index, StoreView *v) {
    if (!s) return fail(LMAP_ERR_INVALID_ARGUMENT, "store is NULL");
    if (s->n_kf < 1 || s->n_kp < 0) return fail(LMAP_ERR_INVALID_ARGUMENT, "n_kf must be >= 1 and n_kp >= 0");
    if (s->max_kp < 1 || s->max_kp > LMAP_MAX_KP)
        return fail(LMAP_ERR_UNSUPPORTED, "max_kp must be in 1..%d (got %d)", LMAP_MAX_KP, s->max_kp);
    if (s->n_levels < 1 || s->n_levels > kMaxLevels)
        return fail(LMAP_ERR_INVALID_ARGUMENT, "n_levels must be in 1..%d", kMaxLevels);
    if (s->width < 1 || s->height < 1) return fail(LMAP_ERR_INVALID_ARGUMENT, "image size must be positive");
    const IndexLayout L = index_layout(*s);
    if (L.ncells > LMAP_MAX_CELLS)
        return fail(LMAP_ERR_UNSUPPORTED, "%d cells of %d px exceed %d", L.ncells, kCell, LMAP_MAX_CELLS);
    if (!s->kp_off || !s->T_cw || (s->n_kp > 0 && (!s->kp_u || !s->kp_v || !s->kp_ur || !s->kp_oct || !s->kp_desc)))
        return fail(LMAP_ERR_INVALID_ARGUMENT, "a store array is NULL");
    if (!s->sigma2 || !s->scale) return fail(LMAP_ERR_INVALID_ARGUMENT, "sigma2 / scale are NULL");
    for (int l = 0; l < s->n_levels; ++l)
        if (!(s->sigma2[l] > 0.0) || !(s->scale[l] > 0.0) || !std::isfinite(s->sigma2[l]) || !std::isfinite(s->scale[l]))
            return fail(LMAP_ERR_INVALID_ARGUMENT, "sigma2[%d] and scale[%d] must be positive and finite", l, l);
    if (!(s->fx > 0.0) || !(s->fy > 0.0) || !std::isfinite(s->cx) || !std::isfinite(s->cy) || !std::isfinite(s->bf))
        return fail(LMAP_ERR_INVALID_ARGUMENT, "bad intrinsics");
    if (need_index && (!s->index || !aligned256(s->index)))
        return fail(LMAP_ERR_INVALID_ARGUMENT, "store index is NULL or not 256-byte aligned");
    memset(v, 0, sizeof(*v));
    v->kp_off = s->kp_off;
    v->T = s->T_cw;
    v->u = s->kp_u;
    v->v = s->kp_v;
    v->ur = s->kp_ur;
    v->oct = s->kp_oct;
    v->desc = s->kp_desc;
    char *ix = static_cast<char *>(s->index);
    v->desc_pm = ix ? reinterpret_cast<int8_t *>(ix + L.o_desc) : nullptr;
    v->cell_off = ix ? reinterpret_cast<int32_t *>(ix + L.o_celloff) : nullptr;
    v->cell_kp = ix ? reinterpret_cast<int32_t *>(ix + L.o_cellkp) : nullptr;
    v->n_kf = s->n_kf;
    v->n_kp = s->n_kp;
    v->max_kp = s->max_kp;
    v->n_levels = s->n_levels;
    v->width = s->width;
    v->height = s->height;
    v->ncx = L.ncx;
    v->ncy = L.ncy;
    v->ncells = L.ncells;
    v->fx = s->fx;
    v->fy = s->fy;
    v->cx = s->cx;
    v->cy = s->cy;
    v->bf = s->bf;
    for (int l = 0; l < s->n_levels; ++l) {
        v->sigma2[l] = s->sigma2[l];
        v->scale[l] = s->scale[l];
    }
    return LMAP_OK;
}

// Synchronise and read the validation words; a non-zero one becomes the error.
lmap_status read_verdict(const int32_t *err_dev, hipStream_t st) {
    int32_t e[kErrCount];
    HIPCHK(hipMemcpyAsync(e, err_dev, sizeof(e), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    static const char *what[kErrCount] = {"keypoint offsets (kp_off) are not a valid running sum within max_kp",
                                          "keypoint octaves out of range",
                                          "keypoint coordinates not finite",
                                          "query keyframe indices out of range",
                                          "output offsets do not match the query sizes",
                                          "map point data out of range or not finite",
                                          "observation indices or octaves out of range",
                                          ""};
    for (int k = 0; k < kErrCount; ++k)
        if (e[k]) return fail(LMAP_ERR_INVALID_ARGUMENT, "%s (%d entries)", what[k], e[k]);
    return LMAP_OK;
}

// Process-wide kernel timing (lmap_profile_enable).
struct Prof {
    std::mutex mu;
    bool on = false;
    std::vector<hipEvent_t> pool;
    std::vector<int> pending;   // class of pair i = events 2i, 2i + 1
    double ms[LMAP_KCLASS_COUNT] = {};
    int64_t n[LMAP_KCLASS_COUNT] = {};
};

Prof &prof() {
    static Prof p;
    return p;
}

// Synchronise and fold the recorded pairs into the counters (end of each call).
lmap_status prof_collect(hipStream_t s) {
    Prof &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    if (!P.on || P.pending.empty()) return LMAP_OK;
    HIPCHK(hipStreamSynchronize(s));
    for (size_t i = 0; i < P.pending.size(); ++i) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, P.pool[2 * i], P.pool[2 * i + 1]));
        P.ms[P.pending[i]] += ms;
        P.n[P.pending[i]] += 1;
    }
    P.pending.clear();
    return LMAP_OK;
}

struct CorrLayout {
    size_t o_geo, o_qok, o_free, o_fcnt, o_owner, o_err, total;
};

CorrLayout corr_layout(const lmap_store &s, int n_q) {
    CorrLayout L;
    size_t o = 0;
    L.o_err = o;
    o += align256(kErrCount * sizeof(int32_t));
    L.o_geo = o;
    o += align256((size_t)n_q * 12 * sizeof(double));
    L.o_qok = o;
    o += align256((size_t)n_q * sizeof(int32_t));
    L.o_free = o;
    o += align256((size_t)s.n_kp * sizeof(int32_t));
    L.o_fcnt = o;
    o += align256((size_t)s.n_kf * sizeof(int32_t));
    L.o_owner = o;
    o += align256((size_t)n_q * s.max_kp * sizeof(uint32_t));
    L.total = o;
    return L;
}

}  // namespace

namespace lmap {

void prof_begin(int cls, hipStream_t s) {
    Prof &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    if (!P.on) return;
    const size_t i = P.pending.size();
    while (P.pool.size() < 2 * (i + 1)) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return;
        P.pool.push_back(e);
    }
    if (hipEventRecord(P.pool[2 * i], s) != hipSuccess) return;
    P.pending.push_back(cls);
}

void prof_end(hipStream_t s) {
    Prof &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    if (!P.on || P.pending.empty()) return;
    (void)hipEventRecord(P.pool[2 * (P.pending.size() - 1) + 1], s);
}

}  // namespace lmap

extern "C" {

lmap_status lmap_profile_enable(int32_t enable) {
    g_err.clear();
    Prof &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    P.on = enable != 0;
    P.pending.clear();
    for (int i = 0; i < LMAP_KCLASS_COUNT; ++i) {
        P.ms[i] = 0.0;
        P.n[i] = 0;
    }
    return LMAP_OK;
}

lmap_status lmap_profile_read(int32_t kernel_class, int64_t *launches, double *total_ms) {
    g_err.clear();
    if (kernel_class < 0 || kernel_class >= LMAP_KCLASS_COUNT)
        return fail(LMAP_ERR_INVALID_ARGUMENT, "kernel class %d out of range", kernel_class);
    Prof &P = prof();
    std::lock_guard<std::mutex> g(P.mu);
    if (launches) *launches = P.n[kernel_class];
    if (total_ms) *total_ms = P.ms[kernel_class];
    return LMAP_OK;
}


int32_t lmap_abi_version(void) { return LMAP_ABI_VERSION; }

const char *lmap_status_string(lmap_status st) {
    switch (st) {
        case LMAP_OK: return "ok";
        case LMAP_ERR_INVALID_ARGUMENT: return "invalid argument";
        case LMAP_ERR_HIP: return "HIP runtime error";
        case LMAP_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case LMAP_ERR_UNSUPPORTED: return "unsupported problem size";
    }
    return "unknown status";
}

const char *lmap_last_error(void) { return g_err.c_str(); }

void lmap_default_corr_params(lmap_corr_params *p) {
    if (!p) return;
    p->th_low = 50;
    p->resolve = 1;
    p->epi_chi2 = 3.84;
    p->epipole_min = 100.0;
}

void lmap_default_fuse_params(lmap_fuse_params *p) {
    if (!p) return;
    p->th_low = 50;
    p->reserved = 0;
    p->radius_th = 3.0;
    p->chi2_mono = 5.991;
    p->chi2_stereo = 7.815;
}

void lmap_default_cull_params(lmap_cull_params *p) {
    if (!p) return;
    p->min_obs = 3;
    p->slack = 0;
    p->num = 9;
    p->den = 10;
}

lmap_status lmap_index_size(const lmap_store *store, size_t *bytes) {
    g_err.clear();
    StoreView v;
    lmap_status st = store_view(store, false, &v);
    if (st != LMAP_OK) return st;
    if (!bytes) return fail(LMAP_ERR_INVALID_ARGUMENT, "bytes is NULL");
    *bytes = index_layout(*store).total;
    return LMAP_OK;
}

lmap_status lmap_index_build(const lmap_store *store, int32_t k0, int32_t k1, size_t index_bytes, int32_t check,
                             void *stream) {
    g_err.clear();
    StoreView v;
    lmap_status st = store_view(store, true, &v);
    if (st != LMAP_OK) return st;
    if (k0 < 0 || k1 > store->n_kf || k0 > k1)
        return fail(LMAP_ERR_INVALID_ARGUMENT, "keyframe range [%d, %d) outside [0, %d)", k0, k1, store->n_kf);
    const IndexLayout L = index_layout(*store);
    if (index_bytes < L.total)
        return fail(LMAP_ERR_WORKSPACE_TOO_SMALL, "index needs %zu bytes, got %zu", L.total, index_bytes);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (check) {
        int32_t *err = reinterpret_cast<int32_t *>(static_cast<char *>(store->index) + L.o_err);
        launch_fill_i32(err, kErrCount, 0, s);
        launch_index_check(v, k0, k1, err, s);
        HIPCHK(hipGetLastError());
        st = read_verdict(err, s);
        if (st != LMAP_OK) return st;
    }
    launch_index_build(v, k0, k1, s);
    HIPCHK(hipGetLastError());
    return prof_collect(s);
}

lmap_status lmap_corr_workspace_size(const lmap_store *store, int32_t n_q, size_t *bytes) {
    g_err.clear();
    StoreView v;
    lmap_status st = store_view(store, false, &v);
    if (st != LMAP_OK) return st;
    if (n_q < 0 || !bytes) return fail(LMAP_ERR_INVALID_ARGUMENT, "n_q < 0 or bytes NULL");
    *bytes = corr_layout(*store, n_q).total;
    return LMAP_OK;
}

}  // extern "C"

// The no-allocation variant's scratch: one copy per GPU, in the code object's device
// memory, for the life of the process.  Host code must not pass `scratch` itself to a
// kernel (on the host it is only a stand-in symbol); its device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) unsigned char scratch[LMAP_NOALLOC_SCRATCH_BYTES];

namespace {

lmap_status corr_impl(const lmap_store *store, const lmap_corr_params *params, const uint8_t *kp_free, int32_t n_q,
                      const int32_t *cur, const int32_t *nbr, const int64_t *out_off, int64_t n_out, int32_t *match,
                      int32_t *dist, void *workspace, size_t workspace_bytes, int32_t check, void *stream) {
    CorrArgs a;
    memset(&a, 0, sizeof(a));
    lmap_status st = store_view(store, true, &a.s);
    if (st != LMAP_OK) return st;
    if (!params) return fail(LMAP_ERR_INVALID_ARGUMENT, "params is NULL");
    if (params->th_low < 0 || params->th_low > 256) return fail(LMAP_ERR_INVALID_ARGUMENT, "th_low must be in 0..256");
    if (!std::isfinite(params->epi_chi2) || !std::isfinite(params->epipole_min))
        return fail(LMAP_ERR_INVALID_ARGUMENT, "epi_chi2 / epipole_min must be finite");
    if (n_q < 0 || n_out < 0) return fail(LMAP_ERR_INVALID_ARGUMENT, "n_q and n_out must be >= 0");
    if (n_q > 0 && (!cur || !nbr || !out_off)) return fail(LMAP_ERR_INVALID_ARGUMENT, "query arrays are NULL");
    if (n_out > 0 && (!match || !dist)) return fail(LMAP_ERR_INVALID_ARGUMENT, "output arrays are NULL");
    if (store->n_kp > 0 && !kp_free) return fail(LMAP_ERR_INVALID_ARGUMENT, "kp_free is NULL");
    const CorrLayout L = corr_layout(*store, n_q);
    if (!workspace || !aligned256(workspace))
        return fail(LMAP_ERR_INVALID_ARGUMENT, "workspace is NULL or not 256-byte aligned");
    if (workspace_bytes < L.total)
        return fail(LMAP_ERR_WORKSPACE_TOO_SMALL, "workspace needs %zu bytes, got %zu", L.total, workspace_bytes);
    if ((int64_t)n_q * ((store->max_kp + kCorrRows - 1) / kCorrRows) > 0x7fffffff)
        return fail(LMAP_ERR_UNSUPPORTED, "too many queries for one launch");
    char *ws = static_cast<char *>(workspace);
    a.kp_free = kp_free;
    a.cur = cur;
    a.nbr = nbr;
    a.out_off = out_off;
    a.n_out = n_out;
    a.match = match;
    a.dist = dist;
    a.geo = reinterpret_cast<double *>(ws + L.o_geo);
    a.qok = reinterpret_cast<int32_t *>(ws + L.o_qok);
    a.free_idx = reinterpret_cast<int32_t *>(ws + L.o_free);
    a.free_cnt = reinterpret_cast<int32_t *>(ws + L.o_fcnt);
    a.owner = reinterpret_cast<uint32_t *>(ws + L.o_owner);
    a.err = reinterpret_cast<int32_t *>(ws + L.o_err);
    a.n_q = n_q;
    a.th_low = params->th_low;
    a.resolve = params->resolve ? 1 : 0;
    a.blocks_per_q = (store->max_kp + kCorrRows - 1) / kCorrRows;
    a.epi_chi2 = params->epi_chi2;
    a.epipole_min = params->epipole_min;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (check) {
        launch_fill_i32(a.err, kErrCount, 0, s);
        launch_index_check(a.s, 0, store->n_kf, a.err, s);
        if (n_q > 0) launch_corr_check(a, s);
        HIPCHK(hipGetLastError());
        st = read_verdict(a.err, s);
        if (st != LMAP_OK) return st;
    }
    launch_corr(a, s);
    HIPCHK(hipGetLastError());
    return prof_collect(s);
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

lmap_status scratch_address(void **out) {
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(LMAP_ERR_UNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p || !aligned256(p)) return fail(LMAP_ERR_HIP, "scratch symbol address not usable");
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return LMAP_OK;
}

}  // namespace

extern "C" {

lmap_status lmap_correspondence(const lmap_store *store, const lmap_corr_params *params, const uint8_t *kp_free,
                                int32_t n_q, const int32_t *cur, const int32_t *nbr, const int64_t *out_off,
                                int64_t n_out, int32_t *match, int32_t *dist, void *workspace,
                                size_t workspace_bytes, int32_t check, void *stream) {
    g_err.clear();
    return corr_impl(store, params, kp_free, n_q, cur, nbr, out_off, n_out, match, dist, workspace, workspace_bytes,
                     check, stream);
}

lmap_status lmap_correspondence_noalloc(const lmap_store *store, const lmap_corr_params *params,
                                        const uint8_t *kp_free, int32_t n_q, const int32_t *cur, const int32_t *nbr,
                                        const int64_t *out_off, int64_t n_out, int32_t *match, int32_t *dist,
                                        int32_t check, void *stream) {
    g_err.clear();
    StoreView v;
    lmap_status st = store_view(store, true, &v);
    if (st != LMAP_OK) return st;
    if (n_q < 0) return fail(LMAP_ERR_INVALID_ARGUMENT, "n_q must be >= 0");
    const size_t need = corr_layout(*store, n_q).total;
    if (need > LMAP_NOALLOC_SCRATCH_BYTES)
        return fail(LMAP_ERR_WORKSPACE_TOO_SMALL,
                    "this problem needs %zu bytes of scratch, above the %u the no-allocation entry point holds", need,
                    (unsigned)LMAP_NOALLOC_SCRATCH_BYTES);
    void *ws = nullptr;
    st = scratch_address(&ws);
    if (st != LMAP_OK) return st;
    return corr_impl(store, params, kp_free, n_q, cur, nbr, out_off, n_out, match, dist, ws,
                     LMAP_NOALLOC_SCRATCH_BYTES, check, stream);
}

lmap_status lmap_fuse_workspace_size(size_t *bytes) {
    g_err.clear();
    if (!bytes) return fail(LMAP_ERR_INVALID_ARGUMENT, "bytes is NULL");
    *bytes = 256;
    return LMAP_OK;
}

lmap_status lmap_fusion(const lmap_store *store, const lmap_fuse_params *params, const lmap_points *points,
                        int32_t n_q, const int32_t *p0, const int32_t *p1, const int32_t *nbr, const int64_t *out_off,
                        int64_t n_out, int32_t max_len, const uint8_t *skip, int32_t *match, int32_t *dist,
                        void *workspace, size_t workspace_bytes, int32_t check, void *stream) {
    g_err.clear();
    FuseArgs a;
    memset(&a, 0, sizeof(a));
    lmap_status st = store_view(store, true, &a.s);
    if (st != LMAP_OK) return st;
    if (!params || !points) return fail(LMAP_ERR_INVALID_ARGUMENT, "params / points are NULL");
    if (params->th_low < 0 || params->th_low > 256) return fail(LMAP_ERR_INVALID_ARGUMENT, "th_low must be in 0..256");
    if (!(params->radius_th >= 0.0) || !std::isfinite(params->radius_th) || !std::isfinite(params->chi2_mono) ||
        !std::isfinite(params->chi2_stereo))
        return fail(LMAP_ERR_INVALID_ARGUMENT, "radius_th must be finite and >= 0, chi2 finite");
    if (n_q < 0 || n_out < 0 || points->n_pt < 0) return fail(LMAP_ERR_INVALID_ARGUMENT, "negative size");
    if (n_q > 0 && (!p0 || !p1 || !nbr || !out_off)) return fail(LMAP_ERR_INVALID_ARGUMENT, "query arrays are NULL");
    if (n_out > 0 && (!match || !dist)) return fail(LMAP_ERR_INVALID_ARGUMENT, "output arrays are NULL");
    if (points->n_pt > 0 && (!points->X || !points->normal || !points->dmin || !points->dmax || !points->desc))
        return fail(LMAP_ERR_INVALID_ARGUMENT, "a point array is NULL");
    if (max_len < 1) return fail(LMAP_ERR_INVALID_ARGUMENT, "max_len must be >= 1");
    if (!workspace || !aligned256(workspace) || workspace_bytes < 256)
        return fail(workspace_bytes < 256 ? LMAP_ERR_WORKSPACE_TOO_SMALL : LMAP_ERR_INVALID_ARGUMENT,
                    "workspace must be 256 bytes, 256-byte aligned");
    a.X = points->X;
    a.normal = points->normal;
    a.dmin = points->dmin;
    a.dmax = points->dmax;
    a.pdesc = points->desc;
    a.p0 = p0;
    a.p1 = p1;
    a.nbr = nbr;
    a.out_off = out_off;
    a.skip = skip;
    a.match = match;
    a.dist = dist;
    a.err = static_cast<int32_t *>(workspace);
    a.n_out = n_out;
    a.n_pt = points->n_pt;
    a.n_q = n_q;
    a.th_low = params->th_low;
    a.blocks_per_q = std::min(65535, (max_len + 255) / 256);
    a.radius_th = params->radius_th;
    a.chi2_mono = params->chi2_mono;
    a.chi2_stereo = params->chi2_stereo;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (check) {
        launch_fill_i32(a.err, kErrCount, 0, s);
        launch_index_check(a.s, 0, store->n_kf, a.err, s);
        launch_fuse_check(a, s);
        HIPCHK(hipGetLastError());
        st = read_verdict(a.err, s);
        if (st != LMAP_OK) return st;
    }
    launch_fuse(a, s);
    HIPCHK(hipGetLastError());
    return prof_collect(s);
}

lmap_status lmap_cull_workspace_size(size_t *bytes) {
    g_err.clear();
    if (!bytes) return fail(LMAP_ERR_INVALID_ARGUMENT, "bytes is NULL");
    *bytes = 256;
    return LMAP_OK;
}

lmap_status lmap_culling(int32_t n_kf, int32_t n_pt, int32_t n_obs, int32_t n_levels, const int32_t *obs_kf,
                         const int32_t *obs_pt, const uint8_t *obs_oct, const uint8_t *active, const uint8_t *protect,
                         const lmap_cull_params *params, int32_t *counters, int32_t *kf_obs, int32_t *kf_red,
                         uint8_t *cull, void *workspace, size_t workspace_bytes, int32_t check, void *stream) {
    g_err.clear();
    if (n_kf < 0 || n_pt < 0 || n_obs < 0) return fail(LMAP_ERR_INVALID_ARGUMENT, "negative size");
    if (n_levels < 1 || n_levels > kMaxLevels) return fail(LMAP_ERR_INVALID_ARGUMENT, "n_levels must be in 1..32");
    if (!params) return fail(LMAP_ERR_INVALID_ARGUMENT, "params is NULL");
    if (params->min_obs < 0 || params->slack < 0 || params->num < 0 || params->den < 1)
        return fail(LMAP_ERR_INVALID_ARGUMENT, "min_obs, slack, num must be >= 0 and den >= 1");
    if (n_obs > 0 && (!obs_kf || !obs_pt || !obs_oct))
        return fail(LMAP_ERR_INVALID_ARGUMENT, "observation arrays are NULL");
    if ((n_pt > 0 && !counters) || (n_kf > 0 && (!kf_obs || !kf_red || !cull)))
        return fail(LMAP_ERR_INVALID_ARGUMENT, "output arrays are NULL");
    if ((int64_t)n_pt * n_levels > 0x7fffffffLL) return fail(LMAP_ERR_UNSUPPORTED, "n_pt x n_levels too large");
    if (!workspace || !aligned256(workspace) || workspace_bytes < 256)
        return fail(workspace_bytes < 256 ? LMAP_ERR_WORKSPACE_TOO_SMALL : LMAP_ERR_INVALID_ARGUMENT,
                    "workspace must be 256 bytes, 256-byte aligned");
    CullArgs a;
    memset(&a, 0, sizeof(a));
    a.kf = obs_kf;
    a.pt = obs_pt;
    a.oct = obs_oct;
    a.active = active;
    a.protect = protect;
    a.counters = counters;
    a.kf_obs = kf_obs;
    a.kf_red = kf_red;
    a.cull = cull;
    a.err = static_cast<int32_t *>(workspace);
    a.n_kf = n_kf;
    a.n_pt = n_pt;
    a.n_obs = n_obs;
    a.n_levels = n_levels;
    a.min_obs = params->min_obs;
    a.slack = params->slack;
    a.num = params->num;
    a.den = params->den;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (check) {
        launch_fill_i32(a.err, kErrCount, 0, s);
        launch_cull_check(a, s);
        HIPCHK(hipGetLastError());
        lmap_status st = read_verdict(a.err, s);
        if (st != LMAP_OK) return st;
    }
    if (n_kf > 0) launch_cull(a, s);
    HIPCHK(hipGetLastError());
    return prof_collect(s);
}

}  // extern "C"
