// Per-solve bookkeeping kernels: state set-up, point-to-observation offsets, input
// validation, the chi-square outlier pass and the final copy-out with statistics.
#include "lba_internal.h"

namespace lba {

// window of a global index given the window offsets (n_windows + 1, non-decreasing)
__device__ __forceinline__ int find_window(const int32_t *off, int nw, int idx) {
    int lo = 0, hi = nw - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (off[mid] <= idx) lo = mid; else hi = mid - 1;
    }
    return lo;
}

enum : int32_t {
    ERR_KF_INDEX = 1, ERR_PT_INDEX = 2, ERR_OCTAVE = 4, ERR_TYPE = 8, ERR_UNSORTED = 16,
    ERR_NONFINITE_OBS = 32, ERR_NONFINITE_POSE = 64, ERR_NONFINITE_POINT = 128,
    ERR_TOO_MANY_OBS = 256, ERR_STEREO_NO_BASELINE = 512
};

// copy the inputs into the working state, reset the control blocks and form the cost
// layer's perturbed poses (each of these steps is skipped when its destination is null),
// then the point -> observation offsets
__global__ void k_setup(MiscArgs a) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * blockDim.x;
    if (a.T)
        for (int64_t i = tid; i < (int64_t)a.n_kf * 12; i += nth) a.T[i] = a.T_in[i];
    if (a.X0)
        for (int64_t i = tid; i < (int64_t)a.n_pt * 3; i += nth) a.X0[i] = a.X_in[i];
    // cost layer: the perturbed poses Exp(xi_k) T_k, composed in FP64 once per call and
    // used in FP32 by every tile of the keyframe's window
    for (int64_t k = tid; a.Pf && k < a.n_kf; k += nth) {
        const double *T0 = a.T_in + k * 12;
        double Tk[12];
        if (a.xi) {
            double x[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) x[q] = (double)a.xi[k * 6 + q];
            se3_left_update(x, T0, Tk);
        } else {
#pragma unroll
            for (int i = 0; i < 12; ++i) Tk[i] = T0[i];
        }
#pragma unroll
        for (int i = 0; i < 12; ++i) a.Pf[k * 12 + i] = (float)Tk[i];
    }
    for (int64_t w = tid; a.ctl && w < a.c.n_windows; w += nth) {
        Ctl c;
        c.lambda = 0.0; c.nu = 2.0; c.F = 0.0; c.F_trial = 0.0; c.denom_p = 0.0;
        c.F_initial = 0.0; c.F_end_r1 = 0.0; c.F_start_r2 = 0.0;
        c.running = 0; c.iter = 0; c.trial = 0; c.trials_total = 0;
        c.cur = 0; c.solve_ok = 0; c.iters_r1 = 0; c.iters_r2 = 0;
        c.term_r1 = 0; c.term_r2 = 0; c.n_outliers = 0; c.round = 0;
        a.ctl[w] = c;
    }
    // point -> first observation: lower bound of the point's local index among the
    // window's (sorted) observation point indices
    for (int64_t p = tid; p <= a.n_pt; p += nth) {
        if (p == a.n_pt) {
            a.pt_start[p] = a.obs.n_obs;
            continue;
        }
        const int w = find_window(a.pt_off_dev, a.c.n_windows, (int)p);
        const int j = (int)p - a.pt_off_dev[w];
        int lo = a.obs_off_dev[w], hi = a.obs_off_dev[w + 1];
        while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (a.obs.pt[mid] < j) lo = mid + 1; else hi = mid;
        }
        a.pt_start[p] = lo;
    }
    if (tid == 0) a.err[0] = 0;
}

hipError_t launch_setup(const MiscArgs &a, int n_windows, hipStream_t s) {
    (void)n_windows;
    hipLaunchKernelGGL(k_setup, dim3(1024), dim3(256), 0, s, a);
    return hipGetLastError();
}

// grid (x, window): the blocks of row y check window y's observations; all blocks
// together check the poses, points and per-point observation counts
__global__ void k_validate(MiscArgs a) {
    const int w = blockIdx.y;
    const int64_t o0 = a.obs_off_dev[w], o1 = a.obs_off_dev[w + 1];
    const int K = a.kf_off_dev[w + 1] - a.kf_off_dev[w];
    const int M = a.pt_off_dev[w + 1] - a.pt_off_dev[w];
    int32_t err = 0;
    for (int64_t o = o0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < o1;
         o += (int64_t)gridDim.x * blockDim.x) {
        const int kf = a.obs.kf[o], pt = a.obs.pt[o];
        if (kf < 0 || kf >= K) err |= ERR_KF_INDEX;
        if (pt < 0 || pt >= M) err |= ERR_PT_INDEX;
        if (o > o0 && pt < a.obs.pt[o - 1]) err |= ERR_UNSORTED;
        if (a.obs.oct[o] >= a.n_levels) err |= ERR_OCTAVE;
        const int ty = a.obs.type[o];
        if (ty > 1) err |= ERR_TYPE;
        if (ty == 1 && !(a.c.cam.bf > 0.0)) err |= ERR_STEREO_NO_BASELINE;
        double u, v, ur;
        if (a.obs.z_f32) load_z<float>(a.obs, (int)o, u, v, ur);
        else load_z<double>(a.obs, (int)o, u, v, ur);
        if (!isfinite(u) || !isfinite(v) || (ty == 1 && !isfinite(ur))) err |= ERR_NONFINITE_OBS;
    }
    const int64_t tid = ((int64_t)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t nth = (int64_t)gridDim.x * gridDim.y * blockDim.x;
    if (a.T_in)
        for (int64_t i = tid; i < (int64_t)a.n_kf * 12; i += nth)
            if (!isfinite(a.T_in[i])) err |= ERR_NONFINITE_POSE;
    if (a.X_in)
        for (int64_t i = tid; i < (int64_t)a.n_pt * 3; i += nth)
            if (!isfinite(a.X_in[i])) err |= ERR_NONFINITE_POINT;
    for (int64_t p = tid; p < a.n_pt; p += nth)
        if (a.pt_start[p + 1] - a.pt_start[p] > kMaxObsPerPoint) err |= ERR_TOO_MANY_OBS;
    if (err) atomicOr(a.err, err);
}

// blocks per window row of the (x, window) grids: enough for the largest window
static int row_blocks(int64_t max_obs) {
    int64_t bx = (max_obs + 2047) / 2048;
    return (int)(bx < 1 ? 1 : (bx > 128 ? 128 : bx));
}

hipError_t launch_validate(const MiscArgs &a, int n_windows, int64_t max_obs, hipStream_t s) {
    if (n_windows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_validate, dim3(row_blocks(max_obs), n_windows), dim3(256), 0, s, a);
    return hipGetLastError();
}

// chi-square outlier test of every observation at the current state; grid (x, window).
// With a.count set, each wavefront also adds its number of flagged observations to the
// window's control block (integer atomics: the total does not depend on their order).
__global__ void k_flags(MiscArgs a) {
    // the weights by octave and the thresholds by type, read per observation: from LDS
    // rather than from the kernel arguments (one dependent memory round trip less)
    __shared__ double wt[kMaxLevels + 2];
    if (threadIdx.x < kMaxLevels + 2)
        wt[threadIdx.x] = threadIdx.x < kMaxLevels ? a.c.inv_sigma2[threadIdx.x] : a.c.chi2[threadIdx.x - kMaxLevels];
    __syncthreads();
    const int w = blockIdx.y;
    const int64_t o0 = a.obs_off_dev[w], o1 = a.obs_off_dev[w + 1];
    Ctl &c = a.ctl[w];
    const double *X = c.cur ? a.X1 : a.X0;
    const int kf0 = a.kf_off_dev[w];
    const int64_t pt0 = a.pt_off_dev[w];
    int nflag = 0;
    for (int64_t o = o0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; o < o1;
         o += (int64_t)gridDim.x * blockDim.x) {
        const int kf = kf0 + a.obs.kf[o];
        const int64_t pt = pt0 + a.obs.pt[o];
        const int stereo = a.obs.type[o];
        double u, v, ur;
        if (a.obs.z_f32) load_z<float>(a.obs, (int)o, u, v, ur);
        else load_z<double>(a.obs, (int)o, u, v, ur);
        double xc, yc, zc, eu, ev, er;
        const double e2 = residual(a.c.cam, a.T + 12 * (int64_t)kf, X[3 * pt], X[3 * pt + 1], X[3 * pt + 2],
                                   u, v, ur, stereo, xc, yc, zc, eu, ev, er);
        const double s = e2 * wt[a.obs.oct[o]];
        const int f = (s > wt[kMaxLevels + stereo] || zc <= 0.0) ? 1 : 0;
        a.flags[o] = (uint8_t)f;
        nflag += f;
    }
    if (a.count) {
#pragma unroll
        for (int d = 32; d > 0; d >>= 1) nflag += __shfl_xor(nflag, d, 64);
        if ((threadIdx.x & 63) == 0 && nflag) atomicAdd(&c.n_outliers, nflag);
    }
}

hipError_t launch_flags(const MiscArgs &a, int n_windows, int64_t max_obs, hipStream_t s) {
    if (a.obs.n_obs <= 0 || n_windows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flags, dim3(row_blocks(max_obs), n_windows), dim3(256), 0, s, a);
    return hipGetLastError();
}

// copy-out of the final state and per-window statistics: grid (x, window); every block
// copies a slice of its window's points, block x == 0 also the poses and the statistics
__global__ __launch_bounds__(256) void k_finalize(MiscArgs a) {
    const int w = blockIdx.y;
    const WinInfo W = a.win[w];
    const Ctl c = a.ctl[w];
    const double *X = c.cur ? a.X1 : a.X0;
    const int64_t x0 = 3 * (int64_t)W.pt0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < 3 * (int64_t)W.M;
         i += (int64_t)gridDim.x * blockDim.x)
        a.X_out[x0 + i] = X[x0 + i];
    if (blockIdx.x != 0) return;
    for (int i = threadIdx.x; i < 12 * W.K; i += blockDim.x)
        a.T_out[12 * (int64_t)W.kf0 + i] = a.T[12 * (int64_t)W.kf0 + i];
    if (threadIdx.x == 0) {
        const int tot = c.n_outliers;
        double *st = a.stats + 12 * (int64_t)w;
        st[0] = c.F_initial;
        st[1] = c.F;
        st[2] = c.iters_r1;
        st[3] = c.iters_r2;
        st[4] = c.trials_total;
        st[5] = c.lambda;
        st[6] = c.term_r1;
        st[7] = c.term_r2;
        st[8] = tot;
        st[9] = c.F_end_r1;
        st[10] = c.F_start_r2;
        st[11] = W.Kopt;
    }
}

hipError_t launch_finalize(const MiscArgs &a, int n_windows, hipStream_t s) {
    if (n_windows <= 0) return hipSuccess;
    int bx = (int)((3 * (int64_t)a.n_pt / n_windows + 1023) / 1024);
    bx = bx < 1 ? 1 : (bx > 256 ? 256 : bx);
    hipLaunchKernelGGL(k_finalize, dim3(bx, n_windows), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace lba
