// Linearisation + Schur complement kernel.
//
// One block per tile of consecutive points of one window.  Each wavefront walks its share
// of the tile in chunks of whole points holding at most 64 observations (one observation
// per lane, read from the structure-of-arrays inputs).  Per chunk:
//   1. every lane forms its observation's residual (FP64), robust weight, and the
//      Gauss-Newton blocks Hpp_a, W_a, Hll_a, bp_a, bl_a (Real) in factored form;
//   2. lanes of the same point sum Hll and bl through wave-private LDS staging, factor
//      V = Hll + lambda I = L L^T and form Z_a = W_a L^-T and t = L^-1 bl, so that
//      W_a V^-1 W_b^T = Z_a Z_b^T and W_a V^-1 bl = Z_a t;
//   3. the reduced camera system S = Hpp + lambda I - sum Z_a Z_b^T and its right side
//      r = bp - sum Z_a t accumulate in a block-private LDS copy of S (packed lower
//      triangle) with LDS atomics: the camera diagonal block from the lane that owns
//      the observation, the off-diagonal blocks from pair lanes (a < b of one point).
// The block then writes its partial S / r / bp to global memory once; a separate kernel
// sums the partials of a window in a fixed order (no global atomics).
//
// INIT mode computes only what the damping initialisation needs: the cost, the diagonal
// of Hpp per camera and the largest point-block diagonal.
#include "lba_internal.h"

namespace lba {

template <typename Real>
struct LinSmem {
    double *T;      // K x 12 poses (FP64)
    int *opt;       // K optimisable index or -1
    Real *S;        // E packed lower
    Real *r;        // n
    Real *bp;       // n
    Real *stage;    // waves x 64 x 18
    int *kz;        // waves x 64 camera index of the lane's observation (-1: none)
    int *off;       // waves x 64 pair offsets
    double *red;    // waves x 2
};

static __host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

template <typename Real>
__device__ inline LinSmem<Real> carve_lin(unsigned char *base, int K, int n, int waves) {
    LinSmem<Real> s;
    size_t o = 0;
    s.T = reinterpret_cast<double *>(base + o);
    o = align_up(o + sizeof(double) * 12 * K, 16);
    s.opt = reinterpret_cast<int *>(base + o);
    o = align_up(o + sizeof(int) * K, 16);
    const int E = n * (n + 1) / 2;
    s.S = reinterpret_cast<Real *>(base + o);
    o = align_up(o + sizeof(Real) * E, 16);
    s.r = reinterpret_cast<Real *>(base + o);
    o = align_up(o + sizeof(Real) * n, 16);
    s.bp = reinterpret_cast<Real *>(base + o);
    o = align_up(o + sizeof(Real) * n, 16);
    s.stage = reinterpret_cast<Real *>(base + o);
    o = align_up(o + sizeof(Real) * waves * 64 * 18, 16);
    s.kz = reinterpret_cast<int *>(base + o);
    o = align_up(o + sizeof(int) * waves * 64, 16);
    s.off = reinterpret_cast<int *>(base + o);
    o = align_up(o + sizeof(int) * waves * 64, 16);
    s.red = reinterpret_cast<double *>(base + o);
    return s;
}

static size_t lin_lds_bytes_t(int K, int n, int waves, size_t real) {
    size_t o = 0;
    o = align_up(o + sizeof(double) * 12 * K, 16);
    o = align_up(o + sizeof(int) * K, 16);
    o = align_up(o + real * (size_t)(n * (n + 1) / 2), 16);
    o = align_up(o + real * n, 16);
    o = align_up(o + real * n, 16);
    o = align_up(o + real * waves * 64 * 18, 16);
    o = align_up(o + sizeof(int) * waves * 64, 16);
    o = align_up(o + sizeof(int) * waves * 64, 16);
    o += sizeof(double) * waves * 2;
    return o;
}

size_t lin_lds_bytes(int K, int n, int waves, bool mixed) {
    return lin_lds_bytes_t(K, n, waves, mixed ? sizeof(float) : sizeof(double));
}

// add v to S[row][col] of the symmetric matrix stored as packed lower triangle
template <typename Real>
__device__ __forceinline__ void add_sym(Real *S, int row, int col, Real v) {
    if (row < col) { int t = row; row = col; col = t; }
    lds_add(&S[packed_lower(row, col)], v);
}

template <typename Real, typename ZT, bool INIT>
__global__ __launch_bounds__(kLinThreads) void k_linearize(LinArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile tile = a.tiles[blockIdx.x];
    const WinInfo W = a.win[tile.win];
    const Ctl ctl = a.ctl[tile.win];
    if (!INIT && !ctl.running) return;
    const int K = W.K, n = W.n, E = W.E;
    const int waves = a.waves;
    LinSmem<Real> sm = carve_lin<Real>(smem, K, n, waves);
    const double lambda = ctl.lambda;
    const Real lam = (Real)lambda;
    const double *Xs = ctl.cur ? a.X1 : a.X0;

    for (int i = threadIdx.x; i < 12 * K; i += blockDim.x) sm.T[i] = a.T[(int64_t)W.kf0 * 12 + i];
    for (int i = threadIdx.x; i < K; i += blockDim.x) sm.opt[i] = a.opt_map[W.kf0 + i];
    if (!INIT)
        for (int i = threadIdx.x; i < E; i += blockDim.x) sm.S[i] = Real(0);
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        sm.r[i] = Real(0);
        sm.bp[i] = Real(0);
    }
    __syncthreads();

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    Real *stg = sm.stage + wave * 64 * 18;
    int *kz = sm.kz + wave * 64;
    int *offs = sm.off + wave * 64;
    const int np = tile.p1 - tile.p0;
    const int wp0 = tile.p0 + (int)(((int64_t)np * wave) / waves);
    const int wp1 = tile.p0 + (int)(((int64_t)np * (wave + 1)) / waves);
    const CamParams cam = a.c.cam;
    double Facc = 0.0;
    double mdiag = 0.0;
    int fail = 0;

    for (int p = wp0; p < wp1;) {
        // ---- chunk of whole points with <= 64 observations --------------------------
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

        int s0 = 0, s1 = 0, kl = 0, ka = -1;
        bool act = false;
        ObsBlocks<Real> B;
        Real Hll[6], bl[3];
        double rho = 0.0;
        if (has) {
            const int jl = a.obs.pt[o];
            const int j = W.pt0 + jl;
            s0 = a.pt_start[j] - base;
            s1 = a.pt_start[j + 1] - base;
            kl = a.obs.kf[o];
            ka = sm.opt[kl];
            act = !a.mask || !a.mask[o];
            const int stereo = a.obs.type[o];
            double zu, zv, zr;
            load_z<ZT>(a.obs, o, zu, zv, zr);
            const double *T = sm.T + kl * 12;
            double xc, yc, zc, eu, ev, er;
            const double e2 = residual(cam, T, Xs[3 * (int64_t)j], Xs[3 * (int64_t)j + 1],
                                       Xs[3 * (int64_t)j + 2], zu, zv, zr, stereo, xc, yc, zc, eu, ev, er);
            const double isg = a.c.inv_sigma2[a.obs.oct[o]];
            const double s = e2 * isg;
            double w;
            huber(s, a.c.huber2[stereo], a.robust, rho, w);
            if (!act) rho = 0.0;
            const Real om = act ? (Real)(w * isg) : Real(0);
            obs_blocks<Real>(cam, T, xc, yc, zc, eu, ev, er, stereo, om, B);
            point_terms<Real>(B, Hll, bl);
        } else {
#pragma unroll
            for (int i = 0; i < 6; ++i) Hll[i] = Real(0);
            bl[0] = bl[1] = bl[2] = Real(0);
        }
        Facc += rho;
        if (!act) ka = -1;

        // ---- per-point sums of Hll, bl -----------------------------------------------
#pragma unroll
        for (int i = 0; i < 6; ++i) stg[lane * 18 + i] = Hll[i];
#pragma unroll
        for (int i = 0; i < 3; ++i) stg[lane * 18 + 6 + i] = bl[i];
        wave_sync();
        Real V[6] = {0, 0, 0, 0, 0, 0}, bs[3] = {0, 0, 0};
        if (has) {
            for (int m = s0; m < s1; ++m) {
#pragma unroll
                for (int i = 0; i < 6; ++i) V[i] += stg[m * 18 + i];
#pragma unroll
                for (int i = 0; i < 3; ++i) bs[i] += stg[m * 18 + 6 + i];
            }
        }
        wave_sync();

        if (INIT) {
            if (has && lane == s0) mdiag = fmax(mdiag, (double)fmax(V[0], fmax(V[3], V[5])));
            if (ka >= 0) {
                Real H[36], bpa[6];
                pose_terms<Real>(B, H, bpa);
#pragma unroll
                for (int i = 0; i < 6; ++i) lds_add(&sm.bp[ka * 6 + i], H[i * 7]);
            }
            p = q;
            continue;
        }

        // ---- point block factor, Z_a, t ----------------------------------------------
        Real Li[6] = {0, 0, 0, 0, 0, 0}, t0 = 0, t1 = 0, t2 = 0;
        if (has) {
            V[0] += lam;
            V[3] += lam;
            V[5] += lam;
            if (!chol3_inv<Real>(V, Li)) fail = 1;
            lmul<Real>(Li, bs[0], bs[1], bs[2], t0, t1, t2);
        }
        Real Z[18];
        if (ka >= 0) {
            Real Wm[18], H[36], bpa[6];
            pose_point_block<Real>(B, Wm);
            pose_terms<Real>(B, H, bpa);
#pragma unroll
            for (int i = 0; i < 6; ++i)
                lmul<Real>(Li, Wm[i * 3], Wm[i * 3 + 1], Wm[i * 3 + 2], Z[i * 3], Z[i * 3 + 1], Z[i * 3 + 2]);
            const int r0 = ka * 6;
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                lds_add(&sm.bp[r0 + i], bpa[i]);
                lds_add(&sm.r[r0 + i], bpa[i] - (Z[i * 3] * t0 + Z[i * 3 + 1] * t1 + Z[i * 3 + 2] * t2));
            }
            // diagonal camera block: Hpp_a - Z_a Z_a^T (lower triangle of the block)
#pragma unroll
            for (int i = 0; i < 6; ++i)
#pragma unroll
                for (int j = 0; j <= i; ++j) {
                    const Real v = H[i * 6 + j] - (Z[i * 3] * Z[j * 3] + Z[i * 3 + 1] * Z[j * 3 + 1] +
                                                   Z[i * 3 + 2] * Z[j * 3 + 2]);
                    lds_add(&sm.S[packed_lower(r0 + i, r0 + j)], v);
                }
#pragma unroll
            for (int i = 0; i < 18; ++i) stg[lane * 18 + i] = Z[i];
        }
        kz[lane] = ka;
        // pairs (a, b) with a < b inside one point: lane a owns s1 - a - 1 of them
        const int cnt = has ? (s1 - lane - 1) : 0;
        const int off = wave_exclusive_scan(cnt, lane);
        offs[lane] = off;
        const int Q = __shfl(off + cnt, 63, 64);
        wave_sync();
        for (int qi = lane; qi < Q; qi += 64) {
            // owner lane: largest l with offs[l] <= qi (offs is non-decreasing)
            int lo = 0, hi = 63;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (offs[mid] <= qi) lo = mid; else hi = mid - 1;
            }
            // lanes owning no pair share their offset with the next lane, so the largest
            // such index is the owner of pair qi
            const int la = lo;
            const int lb = la + 1 + (qi - offs[la]);
            const int kA = kz[la], kB = kz[lb];
            if (kA < 0 || kB < 0) continue;
            const Real *za = stg + la * 18;
            const Real *zb = stg + lb * 18;
            Real A[18], Bv[18];
#pragma unroll
            for (int i = 0; i < 18; ++i) { A[i] = za[i]; Bv[i] = zb[i]; }
            const int ra = kA * 6, rb = kB * 6;
            if (kA != kB) {
#pragma unroll
                for (int i = 0; i < 6; ++i)
#pragma unroll
                    for (int j = 0; j < 6; ++j) {
                        const Real v = -(A[i * 3] * Bv[j * 3] + A[i * 3 + 1] * Bv[j * 3 + 1] +
                                         A[i * 3 + 2] * Bv[j * 3 + 2]);
                        add_sym<Real>(sm.S, ra + i, rb + j, v);
                    }
            } else {
                // same camera twice on one point: the block gets Z_a Z_b^T + Z_b Z_a^T
#pragma unroll
                for (int i = 0; i < 6; ++i)
#pragma unroll
                    for (int j = 0; j <= i; ++j) {
                        const Real v = -(A[i * 3] * Bv[j * 3] + A[i * 3 + 1] * Bv[j * 3 + 1] +
                                         A[i * 3 + 2] * Bv[j * 3 + 2] + Bv[i * 3] * A[j * 3] +
                                         Bv[i * 3 + 1] * A[j * 3 + 1] + Bv[i * 3 + 2] * A[j * 3 + 2]);
                        lds_add(&sm.S[packed_lower(ra + i, ra + j)], v);
                    }
            }
        }
        wave_sync();
        p = q;
    }

    // ---- block reductions and write-out ---------------------------------------------
    Facc = wave_sum(Facc);
    mdiag = wave_max(mdiag);
    const int anyfail = __any(fail);
    if (lane == 0) {
        sm.red[wave * 2] = Facc;
        sm.red[wave * 2 + 1] = mdiag;
        if (anyfail) sm.kz[wave * 64] = -2;  // reuse: failure marker
        else sm.kz[wave * 64] = 0;
    }
    __syncthreads();
    const int t = blockIdx.x;
    Real *part = static_cast<Real *>(a.part) + W.part_off + (int64_t)(t - W.tile0) * W.part_stride;
    if (!INIT)
        for (int i = threadIdx.x; i < E; i += blockDim.x) part[i] = sm.S[i];
    for (int i = threadIdx.x; i < n; i += blockDim.x) {
        part[E + i] = sm.r[i];
        part[E + n + i] = sm.bp[i];
    }
    if (threadIdx.x == 0) {
        double F = 0.0, md = 0.0;
        int fl = 0;
        for (int w = 0; w < waves; ++w) {
            F += sm.red[w * 2];
            md = fmax(md, sm.red[w * 2 + 1]);
            fl |= (sm.kz[w * 64] == -2);
        }
        a.partd[4 * t] = F;
        a.partd[4 * t + 1] = md;
        a.partd[4 * t + 2] = fl ? 1.0 : 0.0;
        a.partd[4 * t + 3] = 0.0;
    }
}

hipError_t launch_linearize(const LinArgs &a, int ntiles, size_t lds, bool init, bool mixed,
                            hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    dim3 grid(ntiles), block(64 * a.waves);
    const bool zf = a.obs.z_f32 != 0;
#define LBA_LAUNCH(R, Z, I) hipLaunchKernelGGL((k_linearize<R, Z, I>), grid, block, lds, s, a)
    if (mixed) {
        if (zf) { if (init) LBA_LAUNCH(float, float, true); else LBA_LAUNCH(float, float, false); }
        else { if (init) LBA_LAUNCH(float, double, true); else LBA_LAUNCH(float, double, false); }
    } else {
        if (zf) { if (init) LBA_LAUNCH(double, float, true); else LBA_LAUNCH(double, float, false); }
        else { if (init) LBA_LAUNCH(double, double, true); else LBA_LAUNCH(double, double, false); }
    }
#undef LBA_LAUNCH
    return hipGetLastError();
}

}  // namespace lba
