// Keypoint correspondence search of map-point creation (Sections III-A and IV-C): for
// every keypoint without a map point in the current keyframe, the best match among the
// free keypoints of a neighbour keyframe by descriptor distance, validated by the
// epipolar and epipole tests, with triangulation deferred to the caller.
//
// Descriptor distances on the matrix cores.  With descriptors stored as +-1 bytes, the
// dot product of two of them is 256 - 2 d, so all distances between 128 free keypoints
// of the current keyframe and 32 free keypoints of the neighbour are one 128x32 integer
// product over k = 256: per 32x32 tile, eight v_mfma_i32_32x32x32_i8.  Only pairs with
// d <= th_low (dot >= 256 - 2 th_low) are candidates; they are rare (a keypoint has about
// one true match among hundreds), so each wavefront appends them to an LDS list and
// validates 64 at a time, one per lane, in FP64.  Per row the best (distance, index)
// survives as one integer key d << 22 | j, kept with LDS atomicMin, which makes the
// result independent of the order in which candidates are found.
//
// The deferred resolution (a keypoint of the neighbour chosen by several keypoints keeps
// the closest) takes a second key per neighbour keypoint, d << 22 | i, by global
// atomicMin, and a second pass that drops the losers.
#include "lmap_internal.h"

namespace lmap {

typedef int v4i __attribute__((ext_vector_type(4)));
typedef int v16i __attribute__((ext_vector_type(16)));

// ---- geometry of a keyframe pair (FP64, products and sums in the written order) ---------

// C = A B, 3x3 row-major, each entry summed over k = 0, 1, 2 in order
__device__ void mat3_mul(const double *A, const double *B, double *C) {
#pragma clang fp contract(off)
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = A[i * 3] * B[j];
            acc = acc + A[i * 3 + 1] * B[3 + j];
            acc = acc + A[i * 3 + 2] * B[6 + j];
            C[i * 3 + j] = acc;
        }
}

// Fundamental matrix of the pair (a = current, b = neighbour), x_b^T F x_a = 0:
// relative pose R = R_b R_a^T, t = t_b - R t_a; E = [t]x R; F = K^-T E K^-1
// (Hartley & Zisserman, Multiple View Geometry, 2nd ed., Section 9.6).  Also the epipole
// of a in b: the pixel of a's camera centre -R_a^T t_a seen from b.
__device__ void pair_geometry(const StoreView &s, int a, int b, double *F, double *ep) {
#pragma clang fp contract(off)
    const double *Ta = s.T + 12 * (size_t)a, *Tb = s.T + 12 * (size_t)b;
    double Rb[9], RaT[9], R[9], t[3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            Rb[i * 3 + j] = Tb[i * 4 + j];
            RaT[i * 3 + j] = Ta[j * 4 + i];
        }
    mat3_mul(Rb, RaT, R);
    for (int i = 0; i < 3; ++i) {
        double acc = R[i * 3] * Ta[3];
        acc = acc + R[i * 3 + 1] * Ta[7];
        acc = acc + R[i * 3 + 2] * Ta[11];
        t[i] = Tb[i * 4 + 3] - acc;
    }
    const double tx[9] = {0.0, -t[2], t[1], t[2], 0.0, -t[0], -t[1], t[0], 0.0};
    const double ifx = 1.0 / s.fx, ify = 1.0 / s.fy;
    const double kx = -s.cx / s.fx, ky = -s.cy / s.fy;
    const double Kinv[9] = {ifx, 0.0, kx, 0.0, ify, ky, 0.0, 0.0, 1.0};
    const double KinvT[9] = {ifx, 0.0, 0.0, 0.0, ify, 0.0, kx, ky, 1.0};
    double E[9], M[9];
    mat3_mul(tx, R, E);
    mat3_mul(KinvT, E, M);
    mat3_mul(M, Kinv, F);
    double C[3], X[3];
    for (int i = 0; i < 3; ++i) {
        double acc = Ta[i] * Ta[3];
        acc = acc + Ta[4 + i] * Ta[7];
        acc = acc + Ta[8 + i] * Ta[11];
        C[i] = -acc;
    }
    for (int i = 0; i < 3; ++i) {
        double acc = Tb[i * 4] * C[0];
        acc = acc + Tb[i * 4 + 1] * C[1];
        acc = acc + Tb[i * 4 + 2] * C[2];
        X[i] = acc + Tb[i * 4 + 3];
    }
    ep[0] = s.fx * X[0] / X[2] + s.cx;
    ep[1] = s.fy * X[1] / X[2] + s.cy;
}

// The epipole test (both keypoints monocular) and the epipolar test of a candidate pair.
__device__ bool pair_consistent(const CorrArgs &a, const double *F, const double *ep, int i, int j) {
#pragma clang fp contract(off)
    const StoreView &s = a.s;
    const int o = s.oct[j];
    const double ua = s.u[i], va = s.v[i];
    const double ub = s.u[j], vb = s.v[j];
    if (s.ur[i] < 0.0f && s.ur[j] < 0.0f) {
        const double dx = ep[0] - ub, dy = ep[1] - vb;
        if (dx * dx + dy * dy < a.epipole_min * s.scale[o]) return false;
    }
    const double l0 = (F[0] * ua + F[1] * va) + F[2];
    const double l1 = (F[3] * ua + F[4] * va) + F[5];
    const double l2 = (F[6] * ua + F[7] * va) + F[8];
    const double num = (l0 * ub + l1 * vb) + l2;
    const double den = l0 * l0 + l1 * l1;
    if (den == 0.0) return false;
    const double e2 = num * num / den;
    return e2 < a.epi_chi2 * s.sigma2[o];
}

// ---- per-call set-up -----------------------------------------------------------------

__global__ __launch_bounds__(256) void k_corr_setup(CorrArgs a) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= a.n_q) return;
    const int c = a.cur[q], n = a.nbr[q];
    const bool ok = c >= 0 && c < a.s.n_kf && n >= 0 && n < a.s.n_kf;
    a.qok[q] = ok;
    if (!ok) return;
    double F[9], ep[2];
    pair_geometry(a.s, c, n, F, ep);
    double *g = a.geo + 12 * (size_t)q;
    for (int k = 0; k < 9; ++k) g[k] = F[k];
    g[9] = ep[0];
    g[10] = ep[1];
    g[11] = 0.0;
}

// One block per keyframe: the local indices of its free keypoints, in increasing order.
__global__ __launch_bounds__(256) void k_free_list(CorrArgs a) {
    __shared__ int wcount[4];
    const int k = blockIdx.x;
    const int b0 = a.s.kp_off[k], b1 = a.s.kp_off[k + 1];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int base = 0;
    for (int c0 = b0; c0 < b1; c0 += 256) {
        const int i = c0 + threadIdx.x;
        const bool f = i < b1 && a.kp_free[i] != 0;
        const uint64_t m = __ballot(f);
        if (lane == 0) wcount[wv] = __popcll(m);
        __syncthreads();
        int before = base;
        for (int w = 0; w < wv; ++w) before += wcount[w];
        if (f) a.free_idx[b0 + before + __popcll(m & ((1ull << lane) - 1ull))] = i - b0;
        base += wcount[0] + wcount[1] + wcount[2] + wcount[3];
        __syncthreads();
    }
    if (threadIdx.x == 0) a.free_cnt[k] = base;
}

// ---- the search --------------------------------------------------------------------------

constexpr int kCap = 256;   // candidate records per wavefront in LDS

// Validate the wavefront's candidate records [0, n), one per lane, and keep each row's
// best key.
__device__ void corr_flush(const CorrArgs &a, const double *geo, int ca, int na, const int32_t *rows,
                           const int32_t *cols, int row0, int nr, int nc, const uint32_t *rec_rd,
                           const int32_t *rec_col, int n, uint32_t *best) {
    for (int e0 = 0; e0 < n; e0 += 64) {
        const int e = e0 + (threadIdx.x & 63);
        if (e < n) {
            const uint32_t rd = rec_rd[e];
            const int rl = (int)(rd >> 16), d = (int)(rd & 0xffffu);
            const int col = rec_col[e];
            if (row0 + rl < nr && col < nc) {
                const int i = ca + rows[row0 + rl];
                const int jl = cols[col];
                if (pair_consistent(a, geo, geo + 9, i, na + jl))
                    atomicMin(&best[rl], ((uint32_t)d << kKpBits) | (uint32_t)jl);
            }
        }
    }
}

// One block = 4 wavefronts = 256 free keypoints (rows) of cur[q], two strips of 32 per
// wavefront, sweeping the free keypoints (columns) of nbr[q] in tiles of 32.  The tile's
// column descriptors are staged in LDS once for all four wavefronts (8 KB, columns 272
// bytes apart so that the 16-byte reads of 16 lanes fall in distinct banks), double
// buffered: tile i + 1 is written to LDS and tile i + 2 loaded from HBM while tile i is
// multiplied.  Per tile and wavefront: two independent chains of eight MFMAs.
constexpr int kColPad = 272;
constexpr int kStrips = 2;
static_assert(kCorrRows == 4 * 32 * kStrips, "rows per block");

__global__ __launch_bounds__(256) void k_corr_search(CorrArgs a) {
    __shared__ __align__(16) unsigned char tileB[2][32 * kColPad];
    __shared__ uint32_t best[kCorrRows];
    __shared__ uint32_t rec_rd[4][kCap];
    __shared__ int32_t rec_col[4][kCap];
    __shared__ double geo[12];
    const int q = blockIdx.x / a.blocks_per_q, rb = blockIdx.x % a.blocks_per_q;
    if (!a.qok[q]) return;
    const int c = a.cur[q], n = a.nbr[q];
    const int nr = a.free_cnt[c];
    const int row0 = rb * kCorrRows;
    if (row0 >= nr) return;
    const int nc = a.free_cnt[n];
    const int ca = a.s.kp_off[c], na = a.s.kp_off[n];
    const int32_t *rows = a.free_idx + ca, *cols = a.free_idx + na;
    const int tid = threadIdx.x, wv = tid >> 6, lane = tid & 63;
    const int li = lane & 31, half = lane >> 5;
    best[tid] = 0xffffffffu;
    if (tid < 12) geo[tid] = a.geo[12 * (size_t)q + tid];

    const v4i *pm = reinterpret_cast<const v4i *>(a.s.desc_pm);
    const v4i zero = {0, 0, 0, 0};
    // A: strip s of this wavefront, lane holds row li, bytes [32t + 16 half, +16) for t < 8
    v4i A[kStrips][8];
#pragma unroll
    for (int s = 0; s < kStrips; ++s) {
        const int r = row0 + 64 * wv + 32 * s + li;
        const v4i *src = pm + (size_t)(ca + (r < nr ? rows[r] : 0)) * 16 + half;
#pragma unroll
        for (int t = 0; t < 8; ++t) A[s][t] = r < nr ? src[2 * t] : zero;
    }
    // staging share of this thread: column tid / 8 of a tile, bytes [32 (tid % 8), +32)
    const int scol = tid >> 3, spart = tid & 7;
    v4i st0 = zero, st1 = zero;
    auto load = [&](int tile) {
        const int cc = tile * 32 + scol;
        if (cc < nc) {
            const v4i *src = pm + (size_t)(na + cols[cc]) * 16 + 2 * spart;
            st0 = src[0];
            st1 = src[1];
        } else {
            st0 = zero;
            st1 = zero;
        }
    };
    auto store = [&](int buf) {
        v4i *dst = reinterpret_cast<v4i *>(tileB[buf] + scol * kColPad + 32 * spart);
        dst[0] = st0;
        dst[1] = st1;
    };
    const int ntiles = (nc + 31) / 32;
    if (ntiles > 0) {
        load(0);
        store(0);
    }
    if (ntiles > 1) load(1);
    __syncthreads();

    const int thr = 256 - 2 * a.th_low;
    int ncand = 0;
    uint32_t *my_rd = rec_rd[wv];
    int32_t *my_col = rec_col[wv];
    const uint64_t below = (1ull << lane) - 1ull;
    for (int tile = 0; tile < ntiles; ++tile) {
        const int buf = tile & 1;
        // buf ^ 1 was last read in the previous iteration, which ended at a barrier
        if (tile + 1 < ntiles) store(buf ^ 1);
        if (tile + 2 < ntiles) load(tile + 2);
        v16i acc[kStrips];
#pragma unroll
        for (int s = 0; s < kStrips; ++s) acc[s] = v16i{};
        const unsigned char *bt = tileB[buf] + li * kColPad + 16 * half;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const v4i b = *reinterpret_cast<const v4i *>(bt + 32 * t);
#pragma unroll
            for (int s = 0; s < kStrips; ++s)
                acc[s] = __builtin_amdgcn_mfma_i32_32x32x32_i8(A[s][t], b, acc[s], 0, 0, 0);
        }
        const int col = tile * 32 + li;
        // any candidate in this lane's 32 products?
        int mx = acc[0][0];
#pragma unroll
        for (int s = 0; s < kStrips; ++s)
#pragma unroll
            for (int v = 0; v < 16; ++v) mx = max(mx, acc[s][v]);
        if (__ballot(mx >= thr)) {
            // output element v of lane l: row 8 (v / 4) + 4 (l / 32) + v % 4, column l % 32
#pragma unroll
            for (int s = 0; s < kStrips; ++s)
#pragma unroll
                for (int v = 0; v < 16; ++v) {
                    const bool pass = acc[s][v] >= thr;
                    const uint64_t m = __ballot(pass);
                    if (m) {
                        if (pass) {
                            const int pos = ncand + __popcll(m & below);
                            const int rl = 64 * wv + 32 * s + 8 * (v >> 2) + 4 * half + (v & 3);
                            my_rd[pos] = ((uint32_t)rl << 16) | (uint32_t)((256 - acc[s][v]) >> 1);
                            my_col[pos] = col;
                        }
                        ncand += __popcll(m);
                        if (ncand > kCap - 64) {
                            corr_flush(a, geo, ca, na, rows, cols, row0, nr, nc, my_rd, my_col, ncand, best);
                            ncand = 0;
                        }
                    }
                }
        }
        __syncthreads();
    }
    if (ncand > 0) corr_flush(a, geo, ca, na, rows, cols, row0, nr, nc, my_rd, my_col, ncand, best);
    __syncthreads();
    if (row0 + tid < nr) {
        const uint32_t key = best[tid];
        if (key != 0xffffffffu) {
            const int il = rows[row0 + tid];
            const int64_t o = a.out_off[q] + il;
            const uint32_t jl = key & kKpMask, d = key >> kKpBits;
            if (o >= 0 && o < a.n_out) {
                a.match[o] = (int32_t)jl;
                a.dist[o] = (int32_t)d;
            }
            if (a.resolve && (int)jl < a.s.max_kp)
                atomicMin(&a.owner[(size_t)q * a.s.max_kp + jl], (d << kKpBits) | (uint32_t)il);
        }
    }
}

// Deferred resolution: a row keeps its match only if it holds the neighbour keypoint's key.
__global__ __launch_bounds__(256) void k_corr_resolve(CorrArgs a) {
    const int q = blockIdx.x / a.blocks_per_q, rb = blockIdx.x % a.blocks_per_q;
    if (!a.qok[q]) return;
    const int c = a.cur[q];
    const int nr = a.free_cnt[c];
    const int r = rb * kCorrRows + threadIdx.x;
    if (threadIdx.x >= kCorrRows || r >= nr) return;
    const int il = a.free_idx[a.s.kp_off[c] + r];
    const int64_t o = a.out_off[q] + il;
    if (o < 0 || o >= a.n_out) return;
    const int jl = a.match[o];
    if (jl < 0 || jl >= a.s.max_kp) return;
    const uint32_t key = ((uint32_t)a.dist[o] << kKpBits) | (uint32_t)il;
    if (a.owner[(size_t)q * a.s.max_kp + jl] != key) {
        a.match[o] = -1;
        a.dist[o] = -1;
    }
}

// Validation of the queries and output offsets.
__global__ __launch_bounds__(256) void k_corr_check(CorrArgs a) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q > a.n_q) return;
    const int64_t o = a.out_off[q];
    if (q == 0 && o != 0) atomicAdd(&a.err[kErrOutOff], 1);
    if (q == a.n_q) {
        if (o > a.n_out || o < 0) atomicAdd(&a.err[kErrOutOff], 1);
        return;
    }
    const int c = a.cur[q], n = a.nbr[q];
    if (c < 0 || c >= a.s.n_kf || n < 0 || n >= a.s.n_kf) {
        atomicAdd(&a.err[kErrQuery], 1);
        return;
    }
    if (a.out_off[q + 1] - o != (int64_t)(a.s.kp_off[c + 1] - a.s.kp_off[c])) atomicAdd(&a.err[kErrOutOff], 1);
}

void launch_corr_check(const CorrArgs &a, hipStream_t s) {
    prof_begin(LMAP_KCLASS_CHECK, s);
    hipLaunchKernelGGL(k_corr_check, dim3((a.n_q + 1 + 255) / 256), dim3(256), 0, s, a);
    prof_end(s);
}

void launch_corr(const CorrArgs &a, hipStream_t s) {
    launch_fill_i32(a.match, a.n_out, -1, s);
    launch_fill_i32(a.dist, a.n_out, -1, s);
    if (a.n_q == 0) return;
    if (a.resolve) launch_fill_i32(reinterpret_cast<int32_t *>(a.owner), (int64_t)a.n_q * a.s.max_kp, -1, s);
    prof_begin(LMAP_KCLASS_PREP, s);
    hipLaunchKernelGGL(k_corr_setup, dim3((a.n_q + 255) / 256), dim3(256), 0, s, a);
    prof_end(s);
    prof_begin(LMAP_KCLASS_PREP, s);
    hipLaunchKernelGGL(k_free_list, dim3(a.s.n_kf), dim3(256), 0, s, a);
    prof_end(s);
    const unsigned blocks = (unsigned)((int64_t)a.n_q * a.blocks_per_q);
    prof_begin(LMAP_KCLASS_CORR_SEARCH, s);
    hipLaunchKernelGGL(k_corr_search, dim3(blocks), dim3(256), 0, s, a);
    prof_end(s);
    if (a.resolve) {
        prof_begin(LMAP_KCLASS_CORR_RESOLVE, s);
        hipLaunchKernelGGL(k_corr_resolve, dim3(blocks), dim3(256), 0, s, a);
        prof_end(s);
    }
}

}  // namespace lmap
