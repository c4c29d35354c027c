// Differentiation form: the robust reprojection cost of each window as a function of
// left pose perturbations xi, points X and measurements z, and its hand-written
// backward pass.
//
//   cost_w = sum over active observations i of window w of rho(s_i),
//   s_i = |z_i - pi(Exp(xi_k) T_k X_j)|^2 / sigma2[octave_i]      (Huber rho on s)
//
// Backward, for an upstream gradient g_w per window, with e = z - pi and the IRLS weight
// rho'(s):
//   dL/dz_i   = g_w 2 rho' e / sigma2                       (one row per observation)
//   dL/dX_j   = sum_i R_k^T P_i^T (-dL/dz_i)                 (P = d pi / d Xc)
//   dL/dxi_k  = J_l(xi_k)^T sum_i (Xc x gc ; gc),  gc = P_i^T (-dL/dz_i)
// The Jacobians are recomputed from the inputs in the backward pass (nothing is stored
// between the two passes).  Arithmetic per observation is FP32; the cost and the pose
// sums accumulate in FP64 and are reduced in a fixed order, so results are bitwise
// reproducible.
//
// One 256-thread block per tile of whole points of one window.  A tile is walked in
// chunks of whole points with at most 256 observations (one per thread):
//   - the point gradient is the sum over the point's (contiguous) observations, formed by
//     one thread per point from per-observation terms staged in LDS;
//   - the pose terms are added per keyframe into per-wavefront LDS rows (LDS atomics
//     within one wavefront only), which the block adds in a fixed order at the end of
//     the tile.
#include "lba_internal.h"

namespace lba {

constexpr int kCostThreads = 256;
constexpr int kCostWaves = kCostThreads / kWave;
constexpr int kCostChunk = kCostThreads;   // observations per chunk (a point has at most 64)

static __host__ __device__ inline size_t cost_align(size_t x) { return (x + 15) / 16 * 16; }

size_t cost_lds_bytes(int K, bool backward) {
    size_t o = cost_align(sizeof(float) * 12 * K);               // perturbed poses
    if (backward) {
        o += cost_align(sizeof(double) * kCostWaves * K * 6);    // per-wave pose sums
        o += cost_align(sizeof(float) * kCostChunk * 3);         // per-observation point terms
    }
    o += sizeof(double) * kCostWaves;
    return o;
}

template <bool BWD>
__global__ __launch_bounds__(kCostThreads) void k_cost(CostArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile tile = a.tiles[blockIdx.x];
    const CostWin W = a.win[tile.win];
    const int K = W.K;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    unsigned char *cur = smem;
    float *P = reinterpret_cast<float *>(cur);
    cur += cost_align(sizeof(float) * 12 * K);
    double *gc = reinterpret_cast<double *>(cur);
    if (BWD) cur += cost_align(sizeof(double) * kCostWaves * K * 6);
    float *gx = reinterpret_cast<float *>(cur);
    if (BWD) cur += cost_align(sizeof(float) * kCostChunk * 3);
    double *red = reinterpret_cast<double *>(cur);

    // poses Exp(xi_k) T_k (formed in FP64 by the set-up kernel), used in FP32
    for (int i = tid; i < 12 * K; i += kCostThreads) P[i] = a.Pf[(int64_t)W.kf0 * 12 + i];
    if (BWD)
        for (int i = tid; i < kCostWaves * K * 6; i += kCostThreads) gc[i] = 0.0;
    __syncthreads();

    const float fx = (float)a.cam.fx, fy = (float)a.cam.fy, cx = (float)a.cam.cx, cy = (float)a.cam.cy;
    const float bf = (float)a.cam.bf;
    const float gw = BWD ? (float)a.grad_cost[tile.win] : 0.0f;
    double Facc = 0.0;
    int bad = 0;

    for (int p = tile.p0; p < tile.p1;) {
        // chunk of whole points holding at most kCostChunk observations
        const int base = a.pt_start[p];
        const int cand = p + tid;
        const int ok = cand < tile.p1 && a.pt_start[cand + 1] - base <= kCostChunk;
        const int q = p + __syncthreads_count(ok);
        if (q == p) {   // cannot happen for points with at most 64 observations
            bad = 1;
            break;
        }
        const int nob = a.pt_start[q] - base;
        const int o = base + tid;
        bool valid = false;
        int kl = -1;
        float gd[6] = {0, 0, 0, 0, 0, 0};
        if (tid < nob) {
            kl = a.obs_kf[o];
            const int jl = a.obs_pt[o];
            const bool inr = kl >= 0 && kl < K && jl >= 0 && jl < W.M;
            if (!inr) bad = 1;
            valid = inr && !(a.mask && a.mask[o]);
            float gzu = 0.0f, gzv = 0.0f, gzr = 0.0f;
            float gX0 = 0.0f, gX1 = 0.0f, gX2 = 0.0f;
            if (valid) {
                const int64_t j = W.pt0 + jl;
                const int stereo = a.obs_type[o] != 0;
                const float isg = (float)a.inv_sigma2[a.obs_oct[o]];
                const float zu = a.z[o], zv = a.z[(int64_t)a.n_obs + o], zr = a.z[2 * (int64_t)a.n_obs + o];
                const float X0 = a.X[3 * j], X1 = a.X[3 * j + 1], X2 = a.X[3 * j + 2];
                const float *T = P + kl * 12;
                const float xc = T[0] * X0 + T[1] * X1 + T[2] * X2 + T[3];
                const float yc = T[4] * X0 + T[5] * X1 + T[6] * X2 + T[7];
                const float zc = T[8] * X0 + T[9] * X1 + T[10] * X2 + T[11];
                const float iz = 1.0f / zc;
                const float u = fx * xc * iz + cx, v = fy * yc * iz + cy;
                const float eu = zu - u, ev = zv - v, er = stereo ? zr - (u - bf * iz) : 0.0f;
                const float s = (eu * eu + ev * ev + er * er) * isg;
                const float d2 = (float)a.huber2[stereo];
                float rho, w;
                if (s <= d2) {
                    rho = s;
                    w = 1.0f;
                } else {
                    const float rs = sqrtf(s), d = sqrtf(d2);
                    rho = 2.0f * d * rs - d2;
                    w = d / rs;
                }
                Facc += (double)rho;
                if (BWD) {
                    const float c = 2.0f * w * isg * gw;
                    gzu = c * eu;
                    gzv = c * ev;
                    gzr = c * er;
                    // gradient at the camera point: P^T (-dL/dz)
                    const float iz2 = iz * iz;
                    const float g0 = -fx * iz * (gzu + gzr);
                    const float g1 = -fy * iz * gzv;
                    const float g2 = iz2 * (fx * xc * gzu + fy * yc * gzv + (fx * xc - bf) * gzr);
                    gX0 = T[0] * g0 + T[4] * g1 + T[8] * g2;
                    gX1 = T[1] * g0 + T[5] * g1 + T[9] * g2;
                    gX2 = T[2] * g0 + T[6] * g1 + T[10] * g2;
                    gd[0] = yc * g2 - zc * g1;
                    gd[1] = zc * g0 - xc * g2;
                    gd[2] = xc * g1 - yc * g0;
                    gd[3] = g0;
                    gd[4] = g1;
                    gd[5] = g2;
                }
            }
            if (BWD) {
                a.g_z[o] = gzu;
                a.g_z[(int64_t)a.n_obs + o] = gzv;
                a.g_z[2 * (int64_t)a.n_obs + o] = gzr;
                gx[tid * 3] = gX0;
                gx[tid * 3 + 1] = gX1;
                gx[tid * 3 + 2] = gX2;
            }
        }
        if (BWD) {
            // pose terms into this wavefront's own rows: lanes of one wavefront that hit the
            // same keyframe are serialised by the LDS unit in a fixed order, and no other
            // wavefront touches these rows, so the sums are the same on every run
            if (valid) {
                double *row = gc + (wave * K + kl) * 6;
#pragma unroll
                for (int qd = 0; qd < 6; ++qd) lds_add(row + qd, (double)gd[qd]);
            }
            __syncthreads();
            // point gradients: one thread per point of the chunk (points without
            // observations get zero)
            for (int t = tid; t < q - p; t += kCostThreads) {
                const int s0 = a.pt_start[p + t] - base, s1 = a.pt_start[p + t + 1] - base;
                float h0 = 0.0f, h1 = 0.0f, h2 = 0.0f;
                for (int m = s0; m < s1; ++m) {
                    h0 += gx[m * 3];
                    h1 += gx[m * 3 + 1];
                    h2 += gx[m * 3 + 2];
                }
                const int64_t j = p + t;
                a.g_X[3 * j] = h0;
                a.g_X[3 * j + 1] = h1;
                a.g_X[3 * j + 2] = h2;
            }
            __syncthreads();
        }
        p = q;
    }

    Facc = wave_sum(Facc);
    const int anybad = __syncthreads_or(bad);
    if (lane == 0) red[wave] = Facc;
    __syncthreads();
    if (tid == 0) {
        double F = 0.0;
        for (int w = 0; w < kCostWaves; ++w) F += red[w];
        a.partF[blockIdx.x] = F;
        if (anybad) a.err[0] = 1;
    }
    if (BWD) {
        double *dst = a.partG + W.g_off + (int64_t)(blockIdx.x - W.tile0) * K * 6;
        for (int i = tid; i < K * 6; i += kCostThreads) {
            double v = 0.0;
            for (int w = 0; w < kCostWaves; ++w) v += gc[w * K * 6 + i];
            dst[i] = v;
        }
    }
}

// y = J_l(xi)^T g for the SE(3) left Jacobian J_l = sum_n ad_xi^n / (n + 1)!, with
// ad_xi = [[w^, 0], [v^, w^]] in (rotation, translation) order.  The series is summed by
// Horner's rule to the first N with a^N / (N + 1)! < 1e-17, a = |w|_1 + |v|_1 >= the
// infinity norm of ad_xi (N = 0 for xi = 0), at most 60 terms.
__device__ inline void se3_left_jacobian_t(const double *xi, const double *g, double *y) {
    double ad[36];
#pragma unroll
    for (int i = 0; i < 36; ++i) ad[i] = 0.0;
    const double w0 = xi[0], w1 = xi[1], w2 = xi[2], v0 = xi[3], v1 = xi[4], v2 = xi[5];
    const double Wh[9] = {0.0, -w2, w1, w2, 0.0, -w0, -w1, w0, 0.0};
    const double Vh[9] = {0.0, -v2, v1, v2, 0.0, -v0, -v1, v0, 0.0};
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            ad[r * 6 + c] = Wh[r * 3 + c];
            ad[(r + 3) * 6 + c + 3] = Wh[r * 3 + c];
            ad[(r + 3) * 6 + c] = Vh[r * 3 + c];
        }
    // J^T g = sum_n (ad^T)^n g / (n + 1)!: Horner on the vector, y = g + ad^T (g + ad^T (...)) / k
    const double an = fabs(w0) + fabs(w1) + fabs(w2) + fabs(v0) + fabs(v1) + fabs(v2);
    int N = 0;
    for (double term = 1.0; N < 60 && term >= 1e-17; ++N) term *= an / (double)(N + 2);
    if (an == 0.0) N = 0;
    double acc[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) acc[i] = g[i];
    for (int n = N; n >= 1; --n) {
        double t[6];
        for (int i = 0; i < 6; ++i) {
            double s = 0.0;
            for (int k = 0; k < 6; ++k) s += ad[k * 6 + i] * acc[k];
            t[i] = s / (double)(n + 1);
        }
        for (int i = 0; i < 6; ++i) acc[i] = g[i] + t[i];
    }
    for (int i = 0; i < 6; ++i) y[i] = acc[i];
}

// per window: cost = sum of the tile costs; backward: pose gradients (all keyframes,
// fixed or not) = J_l(xi)^T times the sum of the tile partials.  Both sums run in a
// fixed order: thread i adds the tiles i, i + G, ... (G threads per entry), then the
// block adds the G partial sums in order.
constexpr int kCostRedThreads = 256;

template <bool BWD>
__global__ __launch_bounds__(kCostRedThreads) void k_cost_reduce(CostArgs a, int n_windows) {
    __shared__ double part[kCostRedThreads];
    __shared__ double gsum[kMaxKf * 6];
    const int w = blockIdx.x;
    if (w >= n_windows) return;
    const CostWin W = a.win[w];
    const int tid = threadIdx.x;
    if (!BWD) {
        double F = 0.0;
        for (int t = tid; t < W.ntiles; t += kCostRedThreads) F += a.partF[W.tile0 + t];
        part[tid] = F;
        __syncthreads();
        if (tid == 0) {
            double s = 0.0;
            for (int i = 0; i < kCostRedThreads; ++i) s += part[i];
            a.cost[w] = s;
        }
        return;
    }
    const int KE = W.K * 6;   // entries of the window's pose gradient (K <= kMaxKf)
    const double *src = a.partG + W.g_off;
    if (KE > 0 && KE <= kCostRedThreads) {   // G threads per entry, then G partials in order
        const int G = kCostRedThreads / KE;
        const int e = tid % KE, gi = tid / KE;
        double g = 0.0;
        if (gi < G)
            for (int t = gi; t < W.ntiles; t += G) g += src[(int64_t)t * KE + e];
        part[tid] = g;
        __syncthreads();
        if (tid < KE) {
            double s = 0.0;
            for (int q = 0; q < G; ++q) s += part[q * KE + tid];
            gsum[tid] = s;
        }
    } else {
        for (int e = tid; e < KE; e += kCostRedThreads) {
            double s = 0.0;
            for (int t = 0; t < W.ntiles; ++t) s += src[(int64_t)t * KE + e];
            gsum[e] = s;
        }
    }
    __syncthreads();
    for (int k = tid; k < W.K; k += kCostRedThreads) {
        double y[6];
        if (a.xi) {
            double x[6];
#pragma unroll
            for (int q = 0; q < 6; ++q) x[q] = (double)a.xi[(int64_t)(W.kf0 + k) * 6 + q];
            se3_left_jacobian_t(x, gsum + 6 * k, y);
        } else {
#pragma unroll
            for (int q = 0; q < 6; ++q) y[q] = gsum[6 * k + q];
        }
#pragma unroll
        for (int q = 0; q < 6; ++q) a.g_xi[(int64_t)(W.kf0 + k) * 6 + q] = (float)y[q];
    }
}

size_t cost_static_lds() {
    return std::max(kernel_static_lds((const void *)k_cost<true>), kernel_static_lds((const void *)k_cost<false>));
}

hipError_t launch_cost(const CostArgs &a, int ntiles, int max_k, bool backward, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    const size_t lds = cost_lds_bytes(max_k, backward);
    if (backward)
        hipLaunchKernelGGL(k_cost<true>, dim3(ntiles), dim3(kCostThreads), lds, s, a);
    else
        hipLaunchKernelGGL(k_cost<false>, dim3(ntiles), dim3(kCostThreads), lds, s, a);
    return hipGetLastError();
}

hipError_t launch_cost_reduce(const CostArgs &a, int n_windows, bool backward, hipStream_t s) {
    if (n_windows <= 0) return hipSuccess;
    if (backward)
        hipLaunchKernelGGL(k_cost_reduce<true>, dim3(n_windows), dim3(kCostRedThreads), 0, s, a, n_windows);
    else
        hipLaunchKernelGGL(k_cost_reduce<false>, dim3(n_windows), dim3(kCostRedThreads), 0, s, a, n_windows);
    return hipGetLastError();
}

}  // namespace lba
