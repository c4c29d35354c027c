// Back-substitution, retraction and trial cost.
//
// One block per tile of points (same tiles as the linearisation).  The block forms the
// trial poses Exp(dp_k) T_k of its window in LDS, then walks its points in chunks of
// whole points (one observation per lane).  The Jacobians are recomputed at the current
// state instead of being stored: each lane forms Hll_a, bl_a and W_a^T dp_k(a); lanes of
// a point sum them, factor V = Hll + lambda I and solve
//   dl_j = V^-1 (bl_j - sum_a W_a^T dp_k(a)),   X'_j = X_j + dl_j,
// then every lane evaluates its observation's robust cost at (T', X') in FP64.  The block
// writes its trial cost and its part dl^T (lambda dl + bl) of the gain-ratio denominator.
#include "lba_internal.h"

namespace lba {

static __host__ __device__ inline size_t align_up_u(size_t x, size_t a) { return (x + a - 1) / a * a; }

template <typename Real>
struct UpdSmem {
    double *T;      // K x 12 current poses
    double *Tn;     // K x 12 trial poses
    int *opt;       // K
    Real *dp;       // n (Real copy of the pose step)
    Real *stage;    // waves x 64 x 12
    Real *pslot;    // waves x 64 x 6: per chunk point (dl, bl)
    double *red;    // waves x 3
};

static size_t upd_lds_t(int K, int n, int waves, size_t real) {
    size_t o = 0;
    o = align_up_u(o + sizeof(double) * 12 * K, 16);
    o = align_up_u(o + sizeof(double) * 12 * K, 16);
    o = align_up_u(o + sizeof(int) * K, 16);
    o = align_up_u(o + real * (n > 0 ? n : 1), 16);
    o = align_up_u(o + real * waves * 64 * 12, 16);
    o = align_up_u(o + real * waves * 64 * 6, 16);
    o += sizeof(double) * waves * 3;
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
    s.dp = reinterpret_cast<Real *>(base + o);
    o = align_up_u(o + sizeof(Real) * (n > 0 ? n : 1), 16);
    s.stage = reinterpret_cast<Real *>(base + o);
    o = align_up_u(o + sizeof(Real) * waves * 64 * 12, 16);
    s.pslot = reinterpret_cast<Real *>(base + o);
    o = align_up_u(o + sizeof(Real) * waves * 64 * 6, 16);
    s.red = reinterpret_cast<double *>(base + o);
    return s;
}

template <typename Real, typename ZT>
__global__ __launch_bounds__(kLinThreads) void k_update(UpdArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile tile = a.tiles[blockIdx.x];
    const WinInfo W = a.win[tile.win];
    const Ctl ctl = a.ctl[tile.win];
    if (!ctl.running) return;
    const int K = W.K, n = W.n;
    const int waves = a.waves;
    UpdSmem<Real> sm = carve_upd<Real>(smem, K, n, waves);
    const double lambda = ctl.lambda;
    const Real lam = (Real)lambda;
    const double *Xs = ctl.cur ? a.X1 : a.X0;
    double *Xn = ctl.cur ? a.X0 : a.X1;
    const double *dpw = a.dp + W.dp_off;

    for (int i = threadIdx.x; i < 12 * K; i += blockDim.x) sm.T[i] = a.T[(int64_t)W.kf0 * 12 + i];
    for (int i = threadIdx.x; i < K; i += blockDim.x) sm.opt[i] = a.opt_map[W.kf0 + i];
    for (int i = threadIdx.x; i < n; i += blockDim.x) sm.dp[i] = (Real)dpw[i];
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) {
        const int ok = sm.opt[k];
        if (ok >= 0) {
            se3_left_update(dpw + 6 * ok, sm.T + 12 * k, sm.Tn + 12 * k);
        } else {
#pragma unroll
            for (int i = 0; i < 12; ++i) sm.Tn[12 * k + i] = sm.T[12 * k + i];
        }
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    Real *stg = sm.stage + wave * 64 * 12;
    Real *ps = sm.pslot + wave * 64 * 6;
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
        Real Hll[6] = {0, 0, 0, 0, 0, 0}, bl[3] = {0, 0, 0}, qv[3] = {0, 0, 0};
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
                ObsBlocks<Real> B;
                obs_blocks<Real>(cam, T, xc, yc, zc, eu, ev, er, stereo, (Real)(w * isg), B);
                point_terms<Real>(B, Hll, bl);
                if (ka >= 0) {
                    // W_a^T dp = M^T (A dp),  A dp = dw x x + dv
                    const Real *d = sm.dp + 6 * ka;
                    Real c0, c1, c2;
                    const Real dw[3] = {d[0], d[1], d[2]};
                    cross3(dw, B.x[0], B.x[1], B.x[2], c0, c1, c2);
                    c0 += d[3]; c1 += d[4]; c2 += d[5];
#pragma unroll
                    for (int m = 0; m < 3; ++m) qv[m] = B.M[m] * c0 + B.M[3 + m] * c1 + B.M[6 + m] * c2;
                }
            }
        }
#pragma unroll
        for (int i = 0; i < 6; ++i) stg[lane * 12 + i] = Hll[i];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            stg[lane * 12 + 6 + i] = bl[i];
            stg[lane * 12 + 9 + i] = qv[i];
        }
        wave_sync();
        // the first lane of each point solves for its dl and publishes it with bl
        if (has && lane == s0) {
            Real V[6] = {0, 0, 0, 0, 0, 0}, bs[3] = {0, 0, 0}, qs[3] = {0, 0, 0};
            for (int m = s0; m < s1; ++m) {
#pragma unroll
                for (int i = 0; i < 6; ++i) V[i] += stg[m * 12 + i];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    bs[i] += stg[m * 12 + 6 + i];
                    qs[i] += stg[m * 12 + 9 + i];
                }
            }
            V[0] += lam;
            V[3] += lam;
            V[5] += lam;
            Real Li[6];
            Real d0 = 0, d1 = 0, d2 = 0;
            if (chol3_inv<Real>(V, Li)) {
                Real y0, y1, y2;
                lmul<Real>(Li, bs[0] - qs[0], bs[1] - qs[1], bs[2] - qs[2], y0, y1, y2);
                ltmul<Real>(Li, y0, y1, y2, d0, d1, d2);
            } else {
                fail = 1;
            }
            const int slot = j - p;
            ps[slot * 6 + 0] = d0; ps[slot * 6 + 1] = d1; ps[slot * 6 + 2] = d2;
            ps[slot * 6 + 3] = bs[0]; ps[slot * 6 + 4] = bs[1]; ps[slot * 6 + 5] = bs[2];
        }
        // points of the chunk without observations keep their position
        const int npts = q - p;
        if (lane < npts && a.pt_start[p + lane + 1] == a.pt_start[p + lane]) {
#pragma unroll
            for (int i = 0; i < 6; ++i) ps[lane * 6 + i] = Real(0);
        }
        wave_sync();
        // one lane per point writes X' and its part of the denominator
        if (lane < npts) {
            const int jp = p + lane;
            const double dl0 = (double)ps[lane * 6], dl1 = (double)ps[lane * 6 + 1], dl2 = (double)ps[lane * 6 + 2];
            Xn[3 * (int64_t)jp] = Xs[3 * (int64_t)jp] + dl0;
            Xn[3 * (int64_t)jp + 1] = Xs[3 * (int64_t)jp + 1] + dl1;
            Xn[3 * (int64_t)jp + 2] = Xs[3 * (int64_t)jp + 2] + dl2;
            den += dl0 * (lambda * dl0 + (double)ps[lane * 6 + 3]) + dl1 * (lambda * dl1 + (double)ps[lane * 6 + 4]) +
                   dl2 * (lambda * dl2 + (double)ps[lane * 6 + 5]);
        }
        // trial cost of every active observation at (T', X')
        if (has && act) {
            const int slot = j - p;
            const double Y0 = X0 + (double)ps[slot * 6], Y1 = X1 + (double)ps[slot * 6 + 1],
                         Y2 = X2 + (double)ps[slot * 6 + 2];
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
