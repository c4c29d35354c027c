// Reduced camera system: fixed-order reduction of the per-tile partial sums, FP64 dense
// Cholesky and triangular solves for the pose step, and the per-window Levenberg-
// Marquardt decision (gain ratio, accept / reject, damping update, pose retraction).
#include "lba_internal.h"

namespace lba {

// ------------------------------------------------------------------------------------
// partial sums -> reduced system.  grid = (ceil(max(E + 2n) / 256), n_windows); each
// thread sums one entry over the window's tiles in tile order (deterministic).
// ------------------------------------------------------------------------------------
template <typename Real>
__global__ __launch_bounds__(256) void k_reduce(ReduceArgs a) {
    const int w = blockIdx.y;
    const WinInfo W = a.win[w];
    if (!a.ctl[w].running) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    const int tot = W.E + 2 * W.n;
    const Real *part = static_cast<const Real *>(a.part) + W.part_off;
    if (i < tot) {
        double acc = 0.0;
        for (int t = 0; t < W.ntiles; ++t) acc += (double)part[(int64_t)t * W.part_stride + i];
        a.red[W.red_off + i] = acc;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        double fl = 0.0;
        for (int t = 0; t < W.ntiles; ++t) fl = fmax(fl, a.partd[4 * (W.tile0 + t) + 2]);
        a.redflag[w] = fl;
    }
}

hipError_t launch_reduce(const ReduceArgs &a, int n_windows, hipStream_t s) {
    if (n_windows <= 0) return hipSuccess;
    dim3 grid((a.max_E2n + 255) / 256 > 0 ? (a.max_E2n + 255) / 256 : 1, n_windows), block(256);
    if (a.mixed) hipLaunchKernelGGL(k_reduce<float>, grid, block, 0, s, a);
    else hipLaunchKernelGGL(k_reduce<double>, grid, block, 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// dense FP64 Cholesky of S + lambda I (packed lower triangle in LDS) and the two
// triangular solves, one wavefront per window (wave-synchronous, no block barriers)
// ------------------------------------------------------------------------------------
size_t chol_lds_bytes(int n) {
    const size_t E = (size_t)n * (n + 1) / 2;
    return sizeof(double) * (E + 2 * (size_t)n + 2);
}

__device__ __forceinline__ void tri_decode(int e, int &ii, int &jj) {
    int r = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    while (r * (r + 1) / 2 > e) --r;
    while ((r + 1) * (r + 2) / 2 <= e) ++r;
    ii = r;
    jj = e - r * (r + 1) / 2;
}

__global__ __launch_bounds__(64) void k_cholesky(CholArgs a) {
    extern __shared__ __align__(16) double cs[];
    const int w = blockIdx.x;
    const WinInfo W = a.win[w];
    Ctl *ctl = a.ctl + w;
    if (!ctl->running) return;
    const int n = W.n, E = W.E;
    const int lane = threadIdx.x;
    const double lambda = ctl->lambda;
    double *A = cs;          // E
    double *y = cs + E;      // n
    double *bp = y + n;      // n
    const double *red = a.red + W.red_off;
    for (int i = lane; i < E; i += 64) A[i] = red[i];
    for (int i = lane; i < n; i += 64) {
        y[i] = red[E + i];
        bp[i] = red[E + n + i];
    }
    wave_sync();
    for (int i = lane; i < n; i += 64) A[packed_lower(i, i)] += lambda;
    wave_sync();
    int ok = a.redflag[w] == 0.0;
    for (int k = 0; k < n && ok; ++k) {
        const double d = A[packed_lower(k, k)];
        if (!(d > 0.0) || !isfinite(d)) {
            ok = 0;
            break;
        }
        const double ld = sqrt(d), il = 1.0 / ld;
        wave_sync();
        for (int i = k + 1 + lane; i < n; i += 64) A[packed_lower(i, k)] *= il;
        if (lane == 0) A[packed_lower(k, k)] = ld;
        wave_sync();
        const int m = n - k - 1;
        const int tot = m * (m + 1) / 2;
        for (int e = lane; e < tot; e += 64) {
            int ii, jj;
            tri_decode(e, ii, jj);
            const int i = k + 1 + ii, j = k + 1 + jj;
            A[packed_lower(i, j)] -= A[packed_lower(i, k)] * A[packed_lower(j, k)];
        }
        wave_sync();
    }
    double *dp = a.dp + W.dp_off;
    if (ok) {
        // L y = r
        for (int k = 0; k < n; ++k) {
            const double yk = y[k] / A[packed_lower(k, k)];
            wave_sync();
            for (int i = k + 1 + lane; i < n; i += 64) y[i] -= A[packed_lower(i, k)] * yk;
            if (lane == 0) y[k] = yk;
            wave_sync();
        }
        // L^T x = y
        for (int k = n - 1; k >= 0; --k) {
            const double xk = y[k] / A[packed_lower(k, k)];
            wave_sync();
            for (int i = lane; i < k; i += 64) y[i] -= A[packed_lower(k, i)] * xk;
            if (lane == 0) y[k] = xk;
            wave_sync();
        }
    }
    double den = 0.0;
    for (int i = lane; i < n; i += 64) {
        const double x = ok ? y[i] : 0.0;
        dp[i] = x;
        den += x * (lambda * x + bp[i]);
    }
    den = wave_sum(den);
    if (lane == 0) {
        ctl->solve_ok = ok;
        ctl->denom_p = den;
    }
}

hipError_t launch_cholesky(const CholArgs &a, int n_windows, size_t lds, hipStream_t s) {
    if (n_windows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_cholesky, dim3(n_windows), dim3(64), lds, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// LM decision per window (one wavefront): gain ratio, accept / reject, damping update
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_decide(DecideArgs a) {
    __shared__ int s_acc;
    const int w = blockIdx.x;
    const WinInfo W = a.win[w];
    Ctl *ctl = a.ctl + w;
    if (!ctl->running) return;
    const int lane = threadIdx.x;
    if (lane == 0) {
        double Ft = 0.0, den = ctl->denom_p, fl = 0.0;
        for (int t = 0; t < W.ntiles; ++t) {
            Ft += a.partu[4 * (W.tile0 + t)];
            den += a.partu[4 * (W.tile0 + t) + 1];
            fl = fmax(fl, a.partu[4 * (W.tile0 + t) + 2]);
        }
        const int ok = ctl->solve_ok && fl == 0.0;
        const double gain = (ctl->F - Ft) / den;
        const int acc = ok && isfinite(Ft) && isfinite(gain) && gain > 0.0;
        ctl->F_trial = Ft;
        ctl->trials_total += 1;
        const int iters = a.c.iters[a.round - 1];
        if (acc) {
            ctl->F = Ft;
            const double f = 2.0 * gain - 1.0;
            ctl->lambda *= fmax(1.0 / 3.0, 1.0 - f * f * f);
            ctl->nu = 2.0;
            ctl->cur ^= 1;
            ctl->iter += 1;
            ctl->trial = 0;
            if (a.round == 1) ctl->iters_r1 = ctl->iter;
            else ctl->iters_r2 = ctl->iter;
            if (ctl->iter >= iters) ctl->running = 0;
        } else {
            ctl->lambda *= ctl->nu;
            ctl->nu *= 2.0;
            ctl->trial += 1;
            if (ctl->trial >= a.c.max_trials) {
                ctl->running = 0;
                if (a.round == 1) ctl->term_r1 = 1;
                else ctl->term_r2 = 1;
            }
        }
        s_acc = acc;
    }
    __syncthreads();
    if (s_acc) {
        // accepted: T_k <- Exp(dp_k) T_k for the window's optimisable keyframes
        const double *dp = a.dp + W.dp_off;
        for (int k = lane; k < W.K; k += 64) {
            const int ok = a.opt_map[W.kf0 + k];
            if (ok < 0) continue;
            double *T = a.T + 12 * (int64_t)(W.kf0 + k);
            double Tin[12];
#pragma unroll
            for (int i = 0; i < 12; ++i) Tin[i] = T[i];
            se3_left_update(dp + 6 * ok, Tin, T);
        }
    }
}

hipError_t launch_decide(const DecideArgs &a, int n_windows, hipStream_t s) {
    if (n_windows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_decide, dim3(n_windows), dim3(64), 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// damping initialisation of a round: F and lambda0 = tau * max diag(H)
// ------------------------------------------------------------------------------------
template <typename Real>
__global__ __launch_bounds__(64) void k_init_reduce(InitReduceArgs a) {
    const int w = blockIdx.x;
    const WinInfo W = a.win[w];
    Ctl *ctl = a.ctl + w;
    const int lane = threadIdx.x;
    const Real *part = static_cast<const Real *>(a.part) + W.part_off;
    double md = 0.0;
    for (int i = lane; i < W.n; i += 64) {
        double acc = 0.0;
        for (int t = 0; t < W.ntiles; ++t) acc += (double)part[(int64_t)t * W.part_stride + W.E + W.n + i];
        md = fmax(md, acc);
    }
    md = wave_max(md);
    if (lane == 0) {
        double F = 0.0;
        for (int t = 0; t < W.ntiles; ++t) {
            F += a.partd[4 * (W.tile0 + t)];
            md = fmax(md, a.partd[4 * (W.tile0 + t) + 1]);
        }
        if (a.round == 1) {
            ctl->F_initial = F;
        } else {
            ctl->F_end_r1 = ctl->F;
            ctl->F_start_r2 = F;
        }
        ctl->F = F;
        ctl->lambda = a.c.tau * md;
        ctl->nu = 2.0;
        ctl->iter = 0;
        ctl->trial = 0;
        ctl->round = a.round;
        ctl->running = a.c.iters[a.round - 1] > 0 ? 1 : 0;
    }
}

hipError_t launch_init_reduce(const InitReduceArgs &a, int n_windows, hipStream_t s) {
    if (n_windows <= 0) return hipSuccess;
    if (a.mixed) hipLaunchKernelGGL(k_init_reduce<float>, dim3(n_windows), dim3(64), 0, s, a);
    else hipLaunchKernelGGL(k_init_reduce<double>, dim3(n_windows), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace lba
