// Per-scale observation counters of keyframe culling (Sections III-D and IV-F).  The
// paper keeps, per map point, a small array of its observation counts per octave, so
// that the redundancy test of an observation -- are there at least min_obs other
// observations of the point at the same or a finer scale? -- is a sum over a few
// counters instead of a walk over the point's observation list.  Here the counters are
// built on the GPU from the window's observations (where the bundle adjustment leaves
// them, outlier flags included), in three passes:
//   1. counters[j][o] += 1 for every active observation (integer atomics: exact, and
//      independent of the order);
//   2. per active observation (k, j, o): others = counters[j][0 .. o + slack] summed,
//      minus itself; redundant if others >= min_obs; per-keyframe totals of observations
//      and redundant observations, summed first in LDS when the block's keyframes span
//      a short range, else with global atomics;
//   3. per keyframe: culled if not protected, it has observations and
//      den * redundant >= num * observations.
#include "lmap_internal.h"

namespace lmap {

__global__ __launch_bounds__(256) void k_cull_count(CullArgs a) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < a.n_obs; i += gridDim.x * 256) {
        if (a.active && !a.active[i]) continue;
        const int j = a.pt[i], o = a.oct[i];
        if (j < 0 || j >= a.n_pt || o >= a.n_levels) continue;
        atomicAdd(&a.counters[(size_t)j * a.n_levels + o], 1);
    }
}

constexpr int kCullSpan = 1024;   // keyframes per block summed in LDS

__global__ __launch_bounds__(256) void k_cull_redundant(CullArgs a, int per_block) {
    __shared__ int h_obs[kCullSpan], h_red[kCullSpan];
    __shared__ int wmin[4], wmax[4];
    const int i0 = blockIdx.x * per_block, i1 = min(a.n_obs, i0 + per_block);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // keyframe span of the block
    int kmin = 0x7fffffff, kmax = -1;
    for (int i = i0 + threadIdx.x; i < i1; i += 256) {
        const int k = a.kf[i];
        kmin = min(kmin, k);
        kmax = max(kmax, k);
    }
    for (int o = 32; o > 0; o >>= 1) {
        kmin = min(kmin, __shfl_xor(kmin, o, 64));
        kmax = max(kmax, __shfl_xor(kmax, o, 64));
    }
    if (lane == 0) {
        wmin[wv] = kmin;
        wmax[wv] = kmax;
    }
    for (int k = threadIdx.x; k < kCullSpan; k += 256) h_obs[k] = h_red[k] = 0;
    __syncthreads();
    kmin = min(min(wmin[0], wmin[1]), min(wmin[2], wmin[3]));
    kmax = max(max(wmax[0], wmax[1]), max(wmax[2], wmax[3]));
    const bool local = kmax >= kmin && kmax - kmin < kCullSpan;
    const int L = a.n_levels;
    for (int i = i0 + threadIdx.x; i < i1; i += 256) {
        if (a.active && !a.active[i]) continue;
        const int k = a.kf[i], j = a.pt[i], o = a.oct[i];
        if (k < 0 || k >= a.n_kf || j < 0 || j >= a.n_pt || o >= L) continue;
        const int top = min(L - 1, o + a.slack);
        const int32_t *c = a.counters + (size_t)j * L;
        int others = -1;   // the observation itself is one of the counted
        for (int l = 0; l <= top; ++l) others += c[l];
        const int red = others >= a.min_obs ? 1 : 0;
        if (local) {
            atomicAdd(&h_obs[k - kmin], 1);
            if (red) atomicAdd(&h_red[k - kmin], 1);
        } else {
            atomicAdd(&a.kf_obs[k], 1);
            if (red) atomicAdd(&a.kf_red[k], 1);
        }
    }
    if (!local) return;
    __syncthreads();
    for (int k = threadIdx.x; k <= kmax - kmin; k += 256) {
        if (h_obs[k]) atomicAdd(&a.kf_obs[kmin + k], h_obs[k]);
        if (h_red[k]) atomicAdd(&a.kf_red[kmin + k], h_red[k]);
    }
}

__global__ __launch_bounds__(256) void k_cull_decide(CullArgs a) {
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= a.n_kf) return;
    const int no = a.kf_obs[k], nr = a.kf_red[k];
    const bool prot = a.protect && a.protect[k];
    a.cull[k] = (!prot && no > 0 && (int64_t)a.den * nr >= (int64_t)a.num * no) ? 1 : 0;
}

__global__ __launch_bounds__(256) void k_cull_check(CullArgs a) {
    for (int i = blockIdx.x * 256 + threadIdx.x; i < a.n_obs; i += gridDim.x * 256) {
        const int k = a.kf[i], j = a.pt[i], o = a.oct[i];
        if (k < 0 || k >= a.n_kf || j < 0 || j >= a.n_pt || o >= a.n_levels) atomicAdd(&a.err[kErrObs], 1);
    }
}

void launch_cull_check(const CullArgs &a, hipStream_t s) {
    if (a.n_obs <= 0) return;
    prof_begin(LMAP_KCLASS_CHECK, s);
    hipLaunchKernelGGL(k_cull_check, dim3((unsigned)std::min(4096, (a.n_obs + 255) / 256)), dim3(256), 0, s, a);
    prof_end(s);
}

void launch_cull(const CullArgs &a, hipStream_t s) {
    launch_fill_i32(a.counters, (int64_t)a.n_pt * a.n_levels, 0, s);
    launch_fill_i32(a.kf_obs, a.n_kf, 0, s);
    launch_fill_i32(a.kf_red, a.n_kf, 0, s);
    if (a.n_obs > 0) {
        const unsigned blocks = (unsigned)std::min(8192, (a.n_obs + 255) / 256);
        prof_begin(LMAP_KCLASS_CULL_COUNT, s);
        hipLaunchKernelGGL(k_cull_count, dim3(blocks), dim3(256), 0, s, a);
        prof_end(s);
        const int per_block = 2048;
        prof_begin(LMAP_KCLASS_CULL_REDUNDANT, s);
        hipLaunchKernelGGL(k_cull_redundant, dim3((a.n_obs + per_block - 1) / per_block), dim3(256), 0, s, a,
                           per_block);
        prof_end(s);
    }
    prof_begin(LMAP_KCLASS_CULL_DECIDE, s);
    hipLaunchKernelGGL(k_cull_decide, dim3((a.n_kf + 255) / 256), dim3(256), 0, s, a);
    prof_end(s);
}

}  // namespace lmap
