// Keyframe-store index (Section IV-B, the persistent GPU keyframe storage): built once
// per keyframe when it enters the store.  Two parts:
//   - every 256-bit descriptor as 256 signed bytes, +1 for a set bit and -1 for a clear
//     one, so that the correspondence search can take descriptor distances on the
//     matrix cores (for +-1 vectors a, b of length 256, a.b = 256 - 2 hamming(a, b));
//   - the keypoints of each keyframe sorted into 16x16-pixel cells, so that the fusion
//     search visits only the cells around a projection.
#include "lmap_internal.h"

namespace lmap {

__global__ __launch_bounds__(256) void k_fill_i32(int32_t *p, int64_t n, int32_t value) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = value;
}

void launch_fill_i32(int32_t *p, int64_t n, int32_t value, hipStream_t s) {
    if (n <= 0) return;
    const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
    prof_begin(LMAP_KCLASS_PREP, s);
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)blocks), dim3(256), 0, s, p, n, value);
    prof_end(s);
}

// Four bits to four signed bytes: bit b of n becomes byte b, +1 (0x01) if set and -1
// (0xff) if clear.  Multiplying by 0x204081 copies bit b to bit 8b (shifts 0, 7, 14, 21:
// the partial products never overlap, so nothing carries).
__device__ inline uint32_t spread4(uint32_t n) {
    const uint32_t s = (n * 0x00204081u) & 0x01010101u;
    return (s * 0xfeu) ^ 0xffffffffu;   // 1 -> 0xfe -> 0x01, 0 -> 0x00 -> 0xff
}

__device__ inline int cell_of(const StoreView &v, float u, float vv) {
    int cx = (int)floorf(u * (1.0f / kCell));
    int cy = (int)floorf(vv * (1.0f / kCell));
    cx = min(max(cx, 0), v.ncx - 1);
    cy = min(max(cy, 0), v.ncy - 1);
    return cy * v.ncx + cx;
}

// Exclusive scan of cnt[0 .. n) in LDS by one block of 256 threads; returns the total.
__device__ int block_exclusive_scan(int *cnt, int n, int *wsum) {
    const int tid = threadIdx.x;
    const int per = (n + 255) / 256;
    const int b0 = min(n, tid * per), b1 = min(n, b0 + per);
    int local = 0;
    for (int i = b0; i < b1; ++i) local += cnt[i];
    // inclusive scan of the 256 partial sums: within each wave by shuffles, then waves
    int x = local;
    const int lane = tid & 63, wv = tid >> 6;
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    int before = 0;
    for (int w = 0; w < wv; ++w) before += wsum[w];
    const int total = wsum[0] + wsum[1] + wsum[2] + wsum[3];
    int run = before + x - local;
    for (int i = b0; i < b1; ++i) {
        const int c = cnt[i];
        cnt[i] = run;
        run += c;
    }
    __syncthreads();
    return total;
}

// One block per keyframe: counting sort of its keypoints by cell.
__global__ __launch_bounds__(256) void k_grid(StoreView v, int32_t k0) {
    extern __shared__ int cnt[];   // ncells + 1
    __shared__ int wsum[4];
    const int k = k0 + blockIdx.x;
    const int a = v.kp_off[k], b = v.kp_off[k + 1];
    for (int c = threadIdx.x; c <= v.ncells; c += 256) cnt[c] = 0;
    __syncthreads();
    for (int i = a + threadIdx.x; i < b; i += 256) atomicAdd(&cnt[cell_of(v, v.u[i], v.v[i])], 1);
    __syncthreads();
    const int total = block_exclusive_scan(cnt, v.ncells, wsum);
    int32_t *off = v.cell_off + (size_t)k * (v.ncells + 1);
    for (int c = threadIdx.x; c < v.ncells; c += 256) off[c] = cnt[c];
    if (threadIdx.x == 0) off[v.ncells] = total;
    __syncthreads();
    for (int i = a + threadIdx.x; i < b; i += 256) {
        const int pos = atomicAdd(&cnt[cell_of(v, v.u[i], v.v[i])], 1);
        v.cell_kp[a + pos] = i - a;
    }
    __syncthreads();
    // the order within a cell depends on the atomics: sort each cell (a few entries)
    for (int c = threadIdx.x; c < v.ncells; c += 256) {
        int32_t *e = v.cell_kp + a + off[c];
        const int m = off[c + 1] - off[c];
        for (int i = 1; i < m; ++i) {
            const int x = e[i];
            int j = i - 1;
            while (j >= 0 && e[j] > x) {
                e[j + 1] = e[j];
                --j;
            }
            e[j + 1] = x;
        }
    }
}

// Validation of the keyframes [k0, k1): offsets, octaves, finite coordinates.
__global__ __launch_bounds__(256) void k_index_check(StoreView v, int32_t k0, int32_t k1, int32_t *err) {
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t <= v.n_kf) {
        const int o = v.kp_off[t];
        bool bad = (t == 0 && o != 0) || (t == v.n_kf && o != v.n_kp) || o < 0 || o > v.n_kp;
        if (t < v.n_kf) {
            const int o1 = v.kp_off[t + 1];
            bad = bad || o1 < o || o1 - o > v.max_kp;
        }
        if (bad) atomicAdd(&err[kErrKpOff], 1);
    }
}

__global__ __launch_bounds__(256) void k_kp_check(StoreView v, int64_t i0, int64_t i1, int32_t *err) {
    for (int64_t i = i0 + blockIdx.x * 256 + threadIdx.x; i < i1; i += (int64_t)gridDim.x * 256) {
        if (v.oct[i] >= v.n_levels) atomicAdd(&err[kErrOct], 1);
        if (!isfinite(v.u[i]) || !isfinite(v.v[i]) || isnan(v.ur[i])) atomicAdd(&err[kErrCoord], 1);
    }
}

void launch_index_check(const StoreView &v, int32_t k0, int32_t k1, int32_t *err, hipStream_t s) {
    prof_begin(LMAP_KCLASS_CHECK, s);
    hipLaunchKernelGGL(k_index_check, dim3((v.n_kf + 1 + 255) / 256), dim3(256), 0, s, v, k0, k1, err);
    prof_end(s);
    // keypoint ranges of [k0, k1) are only known on the device: check all keypoints
    if (v.n_kp > 0) {
        prof_begin(LMAP_KCLASS_CHECK, s);
        hipLaunchKernelGGL(k_kp_check, dim3((unsigned)std::min<int64_t>((v.n_kp + 255) / 256, 2048)), dim3(256), 0, s,
                           v, (int64_t)0, (int64_t)v.n_kp, err);
        prof_end(s);
    }
}

// Expansion of every keypoint of [k0, k1): the keypoint range is read on the device, so
// the launch covers up to (k1 - k0) * max_kp keypoints from kp_off[k0] on.
__global__ __launch_bounds__(256) void k_expand_range(const StoreView v, int32_t k0, int32_t k1) {
    const int64_t a = v.kp_off[k0], b = v.kp_off[k1];
    const int64_t n16 = (b - a) * 16;
    for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < n16; t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t kp = a + (t >> 4);
        const int c = (int)(t & 15);
        const uint32_t w = v.desc[kp * 8 + (c >> 1)];
        const uint32_t h = (c & 1) ? (w >> 16) : (w & 0xffffu);
        int4 r;
        r.x = (int)spread4(h & 0xfu);
        r.y = (int)spread4((h >> 4) & 0xfu);
        r.z = (int)spread4((h >> 8) & 0xfu);
        r.w = (int)spread4(h >> 12);
        reinterpret_cast<int4 *>(v.desc_pm)[kp * 16 + c] = r;
    }
}

void launch_index_build(const StoreView &v, int32_t k0, int32_t k1, hipStream_t s) {
    if (k1 <= k0) return;
    const int64_t work = (int64_t)(k1 - k0) * v.max_kp * 16;
    const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 8192));
    prof_begin(LMAP_KCLASS_INDEX, s);
    hipLaunchKernelGGL(k_expand_range, dim3((unsigned)blocks), dim3(256), 0, s, v, k0, k1);
    prof_end(s);
    prof_begin(LMAP_KCLASS_INDEX, s);
    hipLaunchKernelGGL(k_grid, dim3(k1 - k0), dim3(256), (size_t)(v.ncells + 1) * sizeof(int), s, v, k0);
    prof_end(s);
}

}  // namespace lmap
