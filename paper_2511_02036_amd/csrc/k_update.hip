// Back-substitution, retraction and trial cost.
//
// One block per tile of points (same tiles as the linearisation).  The block forms the
// trial poses Exp(dp_k) T_k of its window in LDS, then walks its points in chunks of
// whole points (one observation per lane).  The Jacobians are recomputed at the current
// state instead of being stored: each lane forms Hll_a, bl_a and W_a^T dp_k(a) in FP64
// (the same arithmetic in both precisions, since the point blocks are FP64 there too); lanes of a point sum them, factor V = Hll + lambda I = L L^T and solve
//   dl_j = V^-1 (bl_j - q_j),   q_j = sum_a W_a^T dp_k(a),   X'_j = X_j + dl_j,
// then every lane evaluates its observation's robust cost at (T', X') in FP64.  The block
// writes its trial cost and its part of the gain-ratio denominator,
//   sum_j [ dl_j^T (lambda dl_j + bl_j) + q_j^T V_j^-1 bl_j ],
// the second term completing dp^T bp from the dp^T r the Cholesky kernel forms.
#include "lba_internal.h"

namespace lba {

static __host__ __device__ inline size_t align_up_u(size_t x, size_t a) { return (x + a - 1) / a * a; }

template <typename Real>
struct UpdSmem {
    double *T;      // K x 12 current poses
    double *Tn;     // K x 12 trial poses
    int *opt;       // K
    double *dp;     // n
    double *stg;    // waves x 64 x 6: Hll_a
    double *stgd;   // waves x 64 x 6: bl_a, q_a
    double *pslot;  // waves x 64 x 4: per chunk point (dl, denominator part)
    double *red;    // waves x 3
};

static size_t upd_lds_t(int K, int n, int waves, size_t real) {
    size_t o = 0;
    o = align_up_u(o + sizeof(double) * 12 * K, 16);
    o = align_up_u(o + sizeof(double) * 12 * K, 16);
    o = align_up_u(o + sizeof(int) * K, 16);
    o = align_up_u(o + sizeof(double) * (n > 0 ? n : 1), 16);
    o = align_up_u(o + sizeof(double) * waves * 64 * 6, 16);
    o = align_up_u(o + sizeof(double) * waves * 64 * 6, 16);
    o = align_up_u(o + sizeof(double) * waves * 64 * 4, 16);
    o += sizeof(double) * waves * 3;
    (void)real;
    return o;
}

size_t upd_lds_bytes(int K, int n, int waves, bool mixed) {
    return upd_lds_t(K, n, waves, mixed ? sizeof(float) : sizeof(double));
}

template <typename Real>
__device__ inline UpdSmem<Real> carve_upd(unsigned char *base, int K, int n, int waves) {
    UpdSmem<Real> s;
    size_t o = 0;
    s.T = reinterpret_cast<double *>(base + o);
    o = align_up_u(o + sizeof(double) * 12 * K, 16);
    s.Tn = reinterpret_cast<double *>(base + o);
    o = align_up_u(o + sizeof(double) * 12 * K, 16);
    s.opt = reinterpret_cast<int *>(base + o);
    o = align_up_u(o + sizeof(int) * K, 16);
    s.dp = reinterpret_cast<double *>(base + o);
    o = align_up_u(o + sizeof(double) * (n > 0 ? n : 1), 16);
    s.stg = reinterpret_cast<double *>(base + o);
    o = align_up_u(o + sizeof(double) * waves * 64 * 6, 16);
    s.stgd = reinterpret_cast<double *>(base + o);
    o = align_up_u(o + sizeof(double) * waves * 64 * 6, 16);
    s.pslot = reinterpret_cast<double *>(base + o);
    o = align_up_u(o + sizeof(double) * waves * 64 * 4, 16);
    s.red = reinterpret_cast<double *>(base + o);
    return s;
}

template <typename Real, typename ZT>
__global__ __launch_bounds__(kUpdThreads) void k_update(UpdArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile tile = a.tiles[blockIdx.x];
    const WinInfo W = a.win[tile.win];
    const Ctl ctl = a.ctl[tile.win];
    if (!ctl.running) return;
    const int K = W.K, n = W.n;
    const int waves = a.waves;
    UpdSmem<Real> sm = carve_upd<Real>(smem, K, n, waves);
    const double lambda = ctl.lambda;
    const double *Xs = ctl.cur ? a.X1 : a.X0;
    double *Xn = ctl.cur ? a.X0 : a.X1;
    const double *dpw = a.dp + W.dp_off;

    for (int i = threadIdx.x; i < 12 * K; i += blockDim.x) sm.T[i] = a.T[(int64_t)W.kf0 * 12 + i];
    for (int i = threadIdx.x; i < K; i += blockDim.x) sm.opt[i] = a.opt_map[W.kf0 + i];
    for (int i = threadIdx.x; i < n; i += blockDim.x) sm.dp[i] = dpw[i];
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const int ok = sm.opt[k];
        if (ok >= 0) {
            se3_left_update(sm.dp + 6 * ok, sm.T + 12 * k, sm.Tn + 12 * k);
        } else {
#pragma unroll
            for (int i = 0; i < 12; ++i) sm.Tn[12 * k + i] = sm.T[12 * k + i];
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double *stg = sm.stg + wave * 64 * 6;
    double *stgd = sm.stgd + wave * 64 * 6;
    double *ps = sm.pslot + wave * 64 * 4;
    const int np = tile.p1 - tile.p0;
    const int wp0 = tile.p0 + (int)(((int64_t)np * wave) / waves);
    const int wp1 = tile.p0 + (int)(((int64_t)np * (wave + 1)) / waves);
    const CamParams cam = a.c.cam;
    double Ftr = 0.0, den = 0.0;
    int fail = 0;

    for (int p = wp0; p < wp1;) {
        const int base = a.pt_start[p];
        const int cand = p + lane;
        int ok = 0;
        if (cand < wp1) ok = (a.pt_start[cand + 1] - base) <= kMaxObsPerPoint;
        const int q = p + __popcll(__ballot(ok));
        if (q == p) {   // a point with more observations than one wavefront: not solvable here
            fail = 1;
            break;
        }
        const int nob = a.pt_start[q] - base;
        const bool has = lane < nob;
        const int o = base + lane;

        int s0 = 0, s1 = 0, kl = 0, j = 0, stereo = 0, oct = 0;
        bool act = false;
        double zu = 0, zv = 0, zr = 0;
        double Hll[6] = {0, 0, 0, 0, 0, 0};
        double bl[3] = {0, 0, 0}, qv[3] = {0, 0, 0};
        double X0 = 0, X1 = 0, X2 = 0;
        if (has) {
            const int jl = a.obs.pt[o];
            j = W.pt0 + jl;
            s0 = a.pt_start[j] - base;
            s1 = a.pt_start[j + 1] - base;
            kl = a.obs.kf[o];
            const int ka = sm.opt[kl];
            act = !a.mask || !a.mask[o];
            stereo = a.obs.type[o];
            oct = a.obs.oct[o];
            load_z<ZT>(a.obs, o, zu, zv, zr);
            X0 = Xs[3 * (int64_t)j];
            X1 = Xs[3 * (int64_t)j + 1];
            X2 = Xs[3 * (int64_t)j + 2];
            if (act) {
                const double *T = sm.T + kl * 12;
                double xc, yc, zc, eu, ev, er;
                const double e2 = residual(cam, T, X0, X1, X2, zu, zv, zr, stereo, xc, yc, zc, eu, ev, er);
                const double isg = a.c.inv_sigma2[oct];
                double rho, w;
                huber(e2 * isg, a.c.huber2[stereo], a.robust, rho, w);
                const double omd = w * isg;
                // W_a^T dp = R^T G c with the camera-frame motion c = dw x x + dv
                double c0 = 0.0, c1 = 0.0, c2 = 0.0;
                if (ka >= 0) {
                    const double *d = sm.dp + 6 * ka;
                    c0 = d[1] * zc - d[2] * yc + d[3];
                    c1 = d[2] * xc - d[0] * zc + d[4];
                    c2 = d[0] * yc - d[1] * xc + d[5];
                }
                point_block_step_fp64(cam, T, xc, yc, zc, eu, ev, er, stereo, omd, c0, c1, c2, Hll, bl, qv);
            }
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) stg[lane * 6 + i] = Hll[i];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            stgd[lane * 6 + i] = bl[i];
            stgd[lane * 6 + 3 + i] = qv[i];
        }
        wave_sync();
        // the first lane of each point solves for its dl and publishes it
        if (has && lane == s0) {
            double V[6] = {0, 0, 0, 0, 0, 0};
            double bs[3] = {0, 0, 0}, qs[3] = {0, 0, 0};
            for (int m = s0; m < s1; ++m) {
#pragma unroll
                for (int i = 0; i < 6; ++i) V[i] += stg[m * 6 + i];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    bs[i] += stgd[m * 6 + i];
                    qs[i] += stgd[m * 6 + 3 + i];
                }
            }
            V[0] += lambda;
            V[3] += lambda;
            V[5] += lambda;
            double Li[6];
            double d0 = 0, d1 = 0, d2 = 0, dq = 0;
            if (chol3_inv<double>(V, Li)) {
                const double L0 = Li[0], L1 = Li[1], L2 = Li[2], L3 = Li[3], L4 = Li[4], L5 = Li[5];
                // y = L^-1 (bl - q), dl = L^-T y
                const double r0 = bs[0] - qs[0], r1 = bs[1] - qs[1], r2 = bs[2] - qs[2];
                const double y0 = L0 * r0, y1 = L1 * r0 + L2 * r1, y2 = L3 * r0 + L4 * r1 + L5 * r2;
                d0 = L0 * y0 + L1 * y1 + L3 * y2;
                d1 = L2 * y1 + L4 * y2;
                d2 = L5 * y2;
                // q^T V^-1 bl = (L^-1 q) . (L^-1 bl)
                const double u0 = L0 * qs[0], u1 = L1 * qs[0] + L2 * qs[1], u2 = L3 * qs[0] + L4 * qs[1] + L5 * qs[2];
                const double v0 = L0 * bs[0], v1 = L1 * bs[0] + L2 * bs[1], v2 = L3 * bs[0] + L4 * bs[1] + L5 * bs[2];
                dq = u0 * v0 + u1 * v1 + u2 * v2;
            } else {
                fail = 1;
            }
            const int slot = j - p;
            ps[slot * 4 + 0] = d0;
            ps[slot * 4 + 1] = d1;
            ps[slot * 4 + 2] = d2;
            ps[slot * 4 + 3] = d0 * (lambda * d0 + bs[0]) + d1 * (lambda * d1 + bs[1]) + d2 * (lambda * d2 + bs[2]) + dq;
        }
        // points of the chunk without observations keep their position
        const int npts = q - p;
        if (lane < npts && a.pt_start[p + lane + 1] == a.pt_start[p + lane]) {
#pragma unroll
            for (int i = 0; i < 4; ++i) ps[lane * 4 + i] = 0.0;
        }
        wave_sync();
        // one lane per point writes X' and its part of the denominator
        if (lane < npts) {
            const int64_t jp = p + lane;
            Xn[3 * jp] = Xs[3 * jp] + ps[lane * 4];
            Xn[3 * jp + 1] = Xs[3 * jp + 1] + ps[lane * 4 + 1];
            Xn[3 * jp + 2] = Xs[3 * jp + 2] + ps[lane * 4 + 2];
            den += ps[lane * 4 + 3];
        }
        // trial cost of every active observation at (T', X')
        if (has && act) {
            const int slot = j - p;
            const double Y0 = X0 + ps[slot * 4], Y1 = X1 + ps[slot * 4 + 1], Y2 = X2 + ps[slot * 4 + 2];
            double xc, yc, zc, eu, ev, er;
            const double e2 = residual(cam, sm.Tn + kl * 12, Y0, Y1, Y2, zu, zv, zr, stereo, xc, yc, zc, eu, ev, er);
            double rho, w;
            huber(e2 * a.c.inv_sigma2[oct], a.c.huber2[stereo], a.robust, rho, w);
            Ftr += rho;
        }
        wave_sync();
        p = q;
    }

    Ftr = wave_sum(Ftr);
    den = wave_sum(den);
    const int anyfail = __any(fail);
    if (lane == 0) {
        sm.red[wave * 3] = Ftr;
        sm.red[wave * 3 + 1] = den;
        sm.red[wave * 3 + 2] = anyfail ? 1.0 : 0.0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double F = 0.0, D = 0.0, fl = 0.0;
        for (int w = 0; w < waves; ++w) {
            F += sm.red[w * 3];
            D += sm.red[w * 3 + 1];
            fl = fmax(fl, sm.red[w * 3 + 2]);
        }
        const int t = blockIdx.x;
        a.partu[4 * t] = F;
        a.partu[4 * t + 1] = D;
        a.partu[4 * t + 2] = fl;
        a.partu[4 * t + 3] = 0.0;
    }
}

hipError_t launch_update(const UpdArgs &a, int ntiles, size_t lds, bool mixed, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    dim3 grid(ntiles), block(64 * a.waves);
    const bool zf = a.obs.z_f32 != 0;
    if (mixed) {
        if (zf) hipLaunchKernelGGL((k_update<float, float>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_update<float, double>), grid, block, lds, s, a);
    } else {
        if (zf) hipLaunchKernelGGL((k_update<double, float>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_update<double, double>), grid, block, lds, s, a);
    }
    return hipGetLastError();
}

}  // namespace lba
