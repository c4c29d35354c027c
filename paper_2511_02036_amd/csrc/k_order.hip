// Point order for the linearisation.  Within each window the points are sorted by the
// lowest, then the highest, optimisable keyframe that observes them; points that no
// optimisable keyframe observes go last, and ties keep their index order.  The order
// only changes which points the linearisation kernel groups into one chunk: consecutive
// points of this order share most of their keyframes, so a chunk touches few camera
// blocks of the reduced system and each touched block gathers many pairs.  The sums it
// forms are the same (the Schur complement does not depend on the order of the points).
//
// Windows with few optimisable keyframes (kSortMinKopt or fewer), whose chunks touch few
// camera blocks in any order, keep the index order (k_order_identity writes it; the
// sort did not pay there in measurements).  The others use two kernels, run once per
// solve after the input checks:
//   k_order_keys  grid (x, window), one thread per point: key = lowest | highest << 6
//                 (Kopt for both when no optimisable keyframe observes the point);
//   k_order       one 1024-thread block per window: two stable counting-sort passes over
//                 Kopt + 1 buckets (by the highest, then by the lowest), each ranking a round
//                 of 1024 points with one ballot per bucket per wavefront.  The window's
//                 keys are staged in LDS when they fit.  The second pass writes, per
//                 position of the order, the point, its first observation and its
//                 observation count; a last scan adds the place of the point's first
//                 observation in the observation order that follows the points' order.
// The result is deterministic.  k_order_gather then copies the observations into that
// order (once per solve), and the outlier flags (once per round), so that the
// linearisation reads each chunk's observations as one contiguous range.
#include "lba_internal.h"

#include <algorithm>

namespace lba {

constexpr int kOrdThreads = 1024;
constexpr int kOrdWaves = kOrdThreads / kWave;
constexpr int kBuckets = 64;             // digit range: optimisable keyframe index, Kopt = none
constexpr int kOrdLdsPoints = 49152;     // windows up to this many points sort from LDS keys
constexpr int kSortMinKopt = 20;         // windows with more optimisable keyframes are sorted

__device__ __forceinline__ bool sorted_window(const OrderArgs &a, const WinInfo &W) {
    return a.by_keyframes && W.Kopt > kSortMinKopt;
}
static_assert(kMaxKoptFP64 < kBuckets && kMaxKoptMixed < kBuckets, "keyframe digit range");

__global__ __launch_bounds__(256) void k_order_identity(OrderArgs a) {
    const WinInfo W = a.win[blockIdx.y];
    if (sorted_window(a, W)) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < W.M; i += gridDim.x * blockDim.x) {
        const int P = W.pt0 + i;
        const int s = a.pt_start[P];
        a.pinfo[P] = make_int4(P, s, a.pt_start[P + 1] - s, s);
    }
}

__global__ __launch_bounds__(256) void k_order_keys(OrderArgs a) {
    const WinInfo W = a.win[blockIdx.y];
    if (!sorted_window(a, W)) return;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < W.M; i += gridDim.x * blockDim.x) {
        const int P = W.pt0 + i;
        const int o0 = a.pt_start[P], o1 = a.pt_start[P + 1];
        const int none = W.Kopt;
        int lo = none, hi = 0;
        for (int o = o0; o < o1; o += 4) {   // four observations per step: independent loads
            int kf[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) kf[u] = o + u < o1 ? a.obs_kf[o + u] : -1;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int k = kf[u] >= 0 ? a.opt_map[W.kf0 + kf[u]] : -1;
                if (k >= 0) {
                    lo = min(lo, k);
                    hi = max(hi, k);
                }
            }
        }
        if (lo == none) hi = none;
        a.keys[P] = (uint16_t)(lo | (hi << 6));
    }
}

// one stable counting-sort pass over the window's M points: element i of the input order
// is src[i] (window-local; the identity without src), its bucket the 6-bit digit of its
// key at bit sh (below nb = Kopt + 1).  The element goes to place pos of the output: dst[pos] (window-local),
// or, in the last pass, pinfo[pos].
template <bool kLast>
__device__ void order_pass(const OrderArgs &a, const WinInfo &W, const uint16_t *key, const int32_t *src,
                           int32_t *dst, int sh, int *base, int *wcnt) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, M = W.M;
    const int nb = W.Kopt + 1;
    if (tid < kBuckets) base[tid] = 0;
    __syncthreads();
    for (int i = tid; i < M; i += kOrdThreads) {
        const int e = src ? src[i] : i;
        atomicAdd(&base[(key[e] >> sh) & (kBuckets - 1)], 1);
    }
    __syncthreads();
    if (tid == 0) {
        int s = 0;
        for (int b = 0; b < nb; ++b) {
            const int c = base[b];
            base[b] = s;
            s += c;
        }
    }
    __syncthreads();
    for (int r = 0; r < M; r += kOrdThreads) {
        const int i = r + tid;
        const bool valid = i < M;
        const int e = valid ? (src ? src[i] : i) : -1;
        const int d = valid ? (key[e] >> sh) & (kBuckets - 1) : -1;
        int ps = 0, pe = 0;
        if (kLast && valid) {   // in flight during the ranking
            ps = a.pt_start[W.pt0 + e];
            pe = a.pt_start[W.pt0 + e + 1];
        }
        int rank = 0, mine = 0;
        for (int b = 0; b < nb; ++b) {
            const unsigned long long bal = __ballot(d == b);
            if (d == b) rank = __popcll(bal & ((1ull << lane) - 1ull));
            if (lane == b) mine = __popcll(bal);
        }
        if (lane < kBuckets) wcnt[wave * kBuckets + lane] = mine;
        __syncthreads();
        if (valid) {
            int pos = base[d] + rank;
            for (int w = 0; w < wave; ++w) pos += wcnt[w * kBuckets + d];
            if (kLast) a.pinfo[W.pt0 + pos] = make_int4(W.pt0 + e, ps, pe - ps, 0);
            else dst[pos] = e;
        }
        __syncthreads();
        if (tid < kBuckets) {
            int s = 0;
            for (int w = 0; w < kOrdWaves; ++w) s += wcnt[w * kBuckets + tid];
            base[tid] += s;
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(kOrdThreads) void k_order(OrderArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int base[kBuckets];
    __shared__ int wcnt[kOrdWaves * kBuckets];
    const WinInfo W = a.win[blockIdx.x];
    if (!sorted_window(a, W)) return;
    const uint16_t *key = a.keys + W.pt0;
    if (W.M <= kOrdLdsPoints) {
        uint16_t *lk = reinterpret_cast<uint16_t *>(smem);
        for (int i = threadIdx.x; i < W.M; i += kOrdThreads) lk[i] = key[i];
        key = lk;
    }
    __syncthreads();
    int32_t *tmp = a.tmp + W.pt0;
    order_pass<false>(a, W, key, nullptr, tmp, 6, base, wcnt);   // by the highest keyframe
    __syncthreads();
    order_pass<true>(a, W, key, tmp, nullptr, 0, base, wcnt);    // then, stably, by the lowest
    __syncthreads();
    // places of the observations: the window's first observation plus the exclusive
    // prefix of the counts in the new order
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    int carry = W.ob0;
    for (int r = 0; r < W.M; r += kOrdThreads) {
        const int i = r + tid;
        const int m = i < W.M ? a.pinfo[W.pt0 + i].z : 0;
        int x = m;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(x, o, 64);
            if (lane >= o) x += y;
        }
        if (lane == 63) wcnt[wave] = x;
        __syncthreads();
        int add = carry, tot = 0;
        for (int w = 0; w < kOrdWaves; ++w) {
            const int v = wcnt[w];
            add += w < wave ? v : 0;
            tot += v;
        }
        if (i < W.M) a.pinfo[W.pt0 + i].w = add + x - m;
        carry += tot;
        __syncthreads();
    }
}

// Each wavefront takes 64 consecutive positions of the order; their places form one
// contiguous range (a point's observations follow the previous position's, across
// windows too).  The lanes walk that range 64 places at a time (coalesced writes); each
// finds the point of its place by binary lifting over the lanes' inclusive counts.
template <bool kMask>
__global__ __launch_bounds__(256) void k_order_gather(OrderArgs a) {
    const int lane = threadIdx.x & 63;
    const int64_t nwv = (int64_t)gridDim.x * (blockDim.x / 64);
    for (int64_t b = ((int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6)) * 64; b < a.n_pt; b += nwv * 64) {
        const int64_t pos = b + lane;
        int4 pi = make_int4(0, 0, 0, 0);
        if (pos < a.n_pt) pi = a.pinfo[pos];
        int incl = pi.z;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            const int y = __shfl_up(incl, o, 64);
            if (lane >= o) incl += y;
        }
        const int total = __shfl(incl, 63, 64);
        const int first = __shfl(pi.w, 0, 64);   // place of the range's first observation
        for (int d0 = 0; d0 < total; d0 += 64) {   // uniform trip count: every lane shuffles
            const int d = d0 + lane;
            int j = 0;   // the first lane whose inclusive count exceeds d (fixed six steps)
#pragma unroll
            for (int step = 32; step > 0; step >>= 1)
                if (__shfl(incl, j + step - 1, 64) <= d) j += step;
            const int excl = __shfl(incl, j, 64) - __shfl(pi.z, j, 64);
            const int o = __shfl(pi.y, j, 64) + (d - excl), dst = first + d;
            if (d >= total) continue;
            if (kMask) {
                a.smask[dst] = a.mask[o];
            } else {
                a.sobs_kf[dst] = a.obs.kf[o];
                a.sobs_type[dst] = a.obs.type[o];
                a.sobs_oct[dst] = a.obs.oct[o];
                if (a.obs.z_f32) {
                    const float *z = static_cast<const float *>(a.obs.z);
                    float *sz = static_cast<float *>(a.sobs_z);
#pragma unroll
                    for (int c = 0; c < 3; ++c) sz[(int64_t)c * a.obs.n_obs + dst] = z[(int64_t)c * a.obs.n_obs + o];
                } else {
                    const double *z = static_cast<const double *>(a.obs.z);
                    double *sz = static_cast<double *>(a.sobs_z);
#pragma unroll
                    for (int c = 0; c < 3; ++c) sz[(int64_t)c * a.obs.n_obs + dst] = z[(int64_t)c * a.obs.n_obs + o];
                }
            }
        }
    }
}

hipError_t launch_order_gather(const OrderArgs &a, bool mask, hipStream_t s) {
    if (a.n_pt <= 0) return hipSuccess;
    const int blocks = (int)std::min<int64_t>(4096, (a.n_pt + 255) / 256);   // 64 positions per wavefront
    if (mask) hipLaunchKernelGGL(k_order_gather<true>, dim3(blocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_order_gather<false>, dim3(blocks), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_order(const OrderArgs &a, int n_windows, int max_points, int max_kopt, hipStream_t s) {
    if (n_windows <= 0) return hipSuccess;
    const int bx = std::max(1, std::min(64, (max_points + 255) / 256));
    hipLaunchKernelGGL(k_order_identity, dim3(bx, n_windows), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !a.by_keyframes || max_kopt <= kSortMinKopt) return e;
    hipLaunchKernelGGL(k_order_keys, dim3(bx, n_windows), dim3(256), 0, s, a);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t lds = sizeof(uint16_t) * (size_t)std::min(max_points, kOrdLdsPoints);
    hipLaunchKernelGGL(k_order, dim3(n_windows), dim3(kOrdThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace lba
