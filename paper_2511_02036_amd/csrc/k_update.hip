// Back-substitution, retraction and trial cost.
//
// One block per part of a tile of points (the linearisation's tiles, each split into
// `split` parts of about 512 points, in index order).  The block forms the trial poses
// Exp(dp_k) T_k of its window in LDS, then each wavefront walks its share of the points
// in chunks of whole points (one observation per lane; the point ends of the next chunk
// are loaded while the current one is processed).  Each lane forms W_a^T dp_k(a) =
// R^T G c in FP64 at the current state (G = om P^T P, c the camera-frame motion of dp);
// lane l then sums them for the chunk's point l and back-substitutes with the point
// factor the linearisation of the same step stored, V = L L^T, t = L^-1 bl:
//   dl_j = L^-T (t - L^-1 q_j),   q_j = sum_a W_a^T dp_k(a),   X'_j = X_j + dl_j,
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
    double *wt;     // 34: 1 / sigma2 per octave (32), Huber thresholds mono, stereo
    int *opt;       // K
    double *dp;     // n
    double *pslot;  // waves x 64 x 4: per chunk observation q_a (3), then per chunk point
                    // (dl, denominator part): the q_a are read before dl is written
    double *xs;     // waves x 64 x 3: positions of the chunk's points
    int *pst;       // waves x 65: chunk-local first observation of each point
    double *red;    // waves x 3
};

static size_t upd_lds_t(int K, int n, int waves, size_t real) {
    size_t o = 0;
    o = align_up_u(o + sizeof(double) * 12 * K, 16);
    o = align_up_u(o + sizeof(double) * 12 * K, 16);
    o = align_up_u(o + sizeof(double) * (kMaxLevels + 2), 16);
    o = align_up_u(o + sizeof(int) * K, 16);
    o = align_up_u(o + sizeof(double) * (n > 0 ? n : 1), 16);
    o = align_up_u(o + sizeof(double) * waves * 64 * 4, 16);
    o = align_up_u(o + sizeof(double) * waves * 64 * 3, 16);
    o = align_up_u(o + sizeof(int) * waves * 65, 16);
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
    s.wt = reinterpret_cast<double *>(base + o);
    o = align_up_u(o + sizeof(double) * (kMaxLevels + 2), 16);
    s.opt = reinterpret_cast<int *>(base + o);
    o = align_up_u(o + sizeof(int) * K, 16);
    s.dp = reinterpret_cast<double *>(base + o);
    o = align_up_u(o + sizeof(double) * (n > 0 ? n : 1), 16);
    s.pslot = reinterpret_cast<double *>(base + o);
    o = align_up_u(o + sizeof(double) * waves * 64 * 4, 16);
    s.xs = reinterpret_cast<double *>(base + o);
    o = align_up_u(o + sizeof(double) * waves * 64 * 3, 16);
    s.pst = reinterpret_cast<int *>(base + o);
    o = align_up_u(o + sizeof(int) * waves * 65, 16);
    s.red = reinterpret_cast<double *>(base + o);
    return s;
}

template <typename Real, typename ZT>
// six wavefronts per SIMD: 80 VGPRs (no scratch) and about 25 KB of LDS per block
__global__ __launch_bounds__(kUpdThreads) __attribute__((amdgpu_waves_per_eu(6))) void k_update(UpdArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    // block b: part b % split of tile order[b / split] (the tile's points split evenly)
    const int tt = a.order[blockIdx.x / a.split], sub = blockIdx.x % a.split;
    const Tile tile = a.tiles[tt];
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
    // the weights by octave and type, read per observation: from LDS rather than from the
    // kernel arguments (one dependent memory round trip less per chunk)
    if (threadIdx.x < kMaxLevels + 2)
        sm.wt[threadIdx.x] = threadIdx.x < kMaxLevels ? a.c.inv_sigma2[threadIdx.x] : a.c.huber2[threadIdx.x - kMaxLevels];
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

    // (the wavefront index is uniform: its LDS rows are addressed from scalar registers)
    const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    double *ps = sm.pslot + wave * 64 * 4;
    double *stgd = ps;   // the chunk's q_a (3 per lane), read before ps is written
    double *xs = sm.xs + wave * 64 * 3;
    int *pst = sm.pst + wave * 65;
    const int sp0 = tile.p0 + (int)(((int64_t)(tile.p1 - tile.p0) * sub) / a.split);
    const int sp1 = tile.p0 + (int)(((int64_t)(tile.p1 - tile.p0) * (sub + 1)) / a.split);
    const int np = sp1 - sp0;
    const int wp0 = sp0 + (int)(((int64_t)np * wave) / waves);
    const int wp1 = sp0 + (int)(((int64_t)np * (wave + 1)) / waves);
    const CamParams cam = a.c.cam;
    double Ftr = 0.0, den = 0.0;
    int fail = 0;

    // the point ends of the next chunk are loaded one chunk ahead: lane l holds the end
    // of point p + l, and the chunk's base is the end of the point before it
    int pend = wp0 + lane < wp1 ? a.pt_start[wp0 + lane + 1] : 0;
    int base = wp0 < wp1 ? a.pt_start[wp0] : 0;
    for (int p = wp0; p < wp1;) {
        const int cand = p + lane;
        int ok = 0, e = 0;
        if (cand < wp1) {
            e = pend - base;
            ok = e <= kMaxObsPerPoint;
        }
        const int q = p + __popcll(__ballot(ok));
        if (q == p) {   // a point with more observations than one wavefront: not solvable here
            fail = 1;
            break;
        }
        const int npts = q - p;
        const int nbase = __shfl(pend, npts - 1, 64);   // end of point q - 1 = start of point q
        pend = q + lane < wp1 ? a.pt_start[q + lane + 1] : 0;
        // the chunk's point ranges and positions (lane l: point p + l) into this
        // wavefront's LDS rows, loaded together with the observations
        if (lane < npts) {
            pst[lane + 1] = e;
            xs[3 * lane] = Xs[3 * (int64_t)cand];
            xs[3 * lane + 1] = Xs[3 * (int64_t)cand + 1];
            xs[3 * lane + 2] = Xs[3 * (int64_t)cand + 2];
        }
        if (lane == 0) pst[0] = 0;
        const int o = base + lane;
        int jl = 0, kl = 0, stereo = 0, oct = 0;
        bool act = false;
        ZT zu = 0, zv = 0, zr = 0;   // converted where used
        if (o < a.obs.n_obs) {
            jl = a.obs.pt[o];
            kl = a.obs.kf[o];
            // the flag is loaded without a branch (from a readable byte array when there
            // is none), so that it issues with the other loads
            const uint8_t flag = (a.mask ? a.mask : a.obs.type)[o];
            act = (a.mask == nullptr) | (flag == 0);
            stereo = a.obs.type[o];
            oct = a.obs.oct[o];
            const ZT *zp = static_cast<const ZT *>(a.obs.z);
            zu = zp[o];
            zv = zp[(int64_t)a.obs.n_obs + o];
            zr = zp[2 * (int64_t)a.obs.n_obs + o];
        }
        wave_sync();
        const int nob = pst[npts];
        const bool has = lane < nob;

        int j = 0, pl = 0;
        double qv[3] = {0, 0, 0};
        double X0 = 0, X1 = 0, X2 = 0;
        if (has) {
            j = W.pt0 + jl;
            pl = j - p;
            const int ka = sm.opt[kl];
            X0 = xs[3 * pl];
            X1 = xs[3 * pl + 1];
            X2 = xs[3 * pl + 2];
            if (act && ka >= 0) {
                // W_a^T dp = R^T G c with the camera-frame motion c = dw x x + dv
                const double *T = sm.T + kl * 12;
                double xc, yc, zc, eu, ev, er;
                const double e2 = residual(cam, T, X0, X1, X2, zu, zv, zr, stereo, xc, yc, zc, eu, ev, er);
                const double isg = sm.wt[oct];
                double rho, w;
                huber(e2 * isg, sm.wt[kMaxLevels + stereo], a.robust, rho, w);
                const double *d = sm.dp + 6 * ka;
                obs_step_q(cam, T, xc, yc, zc, stereo, w * isg, d[1] * zc - d[2] * yc + d[3],
                           d[2] * xc - d[0] * zc + d[4], d[0] * yc - d[1] * xc + d[5], qv);
            }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) stgd[lane * 3 + i] = qv[i];
        wave_sync();
        // lane l back-substitutes point p + l with the point factor the linearisation of
        // this step left behind, and publishes dl (points without observations keep their
        // position)
        double res[4] = {0, 0, 0, 0};
        if (lane < npts && pst[lane + 1] > pst[lane]) {
            const int m0 = pst[lane], m1 = pst[lane + 1];
            double qs[3] = {0, 0, 0};
            for (int m = m0; m < m1; ++m) {
#pragma unroll
                for (int i = 0; i < 3; ++i) qs[i] += stgd[m * 3 + i];
            }
            const double *f = a.pf + 12 * (int64_t)(p + lane);
            const double L0 = f[0], L1 = f[1], L2 = f[2], L3 = f[3], L4 = f[4], L5 = f[5];
            const double t0 = f[6], t1 = f[7], t2 = f[8];
            const double b0 = f[9], b1 = f[10], b2 = f[11];
            // u = L^-1 q, y = L^-1 (bl - q) = t - u, dl = L^-T y
            const double u0 = L0 * qs[0], u1 = L1 * qs[0] + L2 * qs[1], u2 = L3 * qs[0] + L4 * qs[1] + L5 * qs[2];
            const double y0 = t0 - u0, y1 = t1 - u1, y2 = t2 - u2;
            const double d0 = L0 * y0 + L1 * y1 + L3 * y2;
            const double d1 = L2 * y1 + L4 * y2;
            const double d2 = L5 * y2;
            // q^T V^-1 bl = (L^-1 q) . (L^-1 bl)
            const double dq = u0 * t0 + u1 * t1 + u2 * t2;
            res[0] = d0;
            res[1] = d1;
            res[2] = d2;
            res[3] = d0 * (lambda * d0 + b0) + d1 * (lambda * d1 + b1) + d2 * (lambda * d2 + b2) + dq;
        }
        wave_sync();   // every lane has read the q_a that the results overwrite
        if (lane < npts) {
#pragma unroll
            for (int i = 0; i < 4; ++i) ps[lane * 4 + i] = res[i];
        }
        wave_sync();
        // one lane per point writes X' and its part of the denominator
        if (lane < npts) {
            const int64_t jp = p + lane;
            Xn[3 * jp] = xs[3 * lane] + ps[lane * 4];
            Xn[3 * jp + 1] = xs[3 * lane + 1] + ps[lane * 4 + 1];
            Xn[3 * jp + 2] = xs[3 * lane + 2] + ps[lane * 4 + 2];
            den += ps[lane * 4 + 3];
        }
        // trial cost of every active observation at (T', X')
        if (has && act) {
            const int slot = j - p;
            // (the position is read again from LDS rather than kept in registers)
            const double Y0 = xs[3 * slot] + ps[slot * 4], Y1 = xs[3 * slot + 1] + ps[slot * 4 + 1],
                         Y2 = xs[3 * slot + 2] + ps[slot * 4 + 2];
            double xc, yc, zc, eu, ev, er;
            const double e2 = residual(cam, sm.Tn + kl * 12, Y0, Y1, Y2, zu, zv, zr, stereo, xc, yc, zc, eu, ev, er);
            double rho, w;
            huber(e2 * sm.wt[oct], sm.wt[kMaxLevels + stereo], a.robust, rho, w);
            Ftr += rho;
        }
        wave_sync();
        p = q;
        base = nbase;
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
        const int64_t t = (int64_t)tt * a.split + sub;
        a.partu[4 * t] = F;
        a.partu[4 * t + 1] = D;
        a.partu[4 * t + 2] = fl;
        a.partu[4 * t + 3] = 0.0;
    }
}

hipError_t launch_update(const UpdArgs &a, int ntiles, size_t lds, bool mixed, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    dim3 grid(ntiles * a.split), block(64 * a.waves);
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
