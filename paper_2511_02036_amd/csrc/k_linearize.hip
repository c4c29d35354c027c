// Linearisation + Schur complement kernel (owner-computes).
//
// One 512-thread block per tile of consecutive points of one window.  The block's share
// of the reduced camera system
//     S = Hpp + lambda I - sum_j sum_{a,b in obs(j)} W_a V_j^-1 W_b^T,
//     r = bp - sum_j sum_{a in obs(j)} W_a V_j^-1 bl_j,
// lives in registers for the whole tile: the 6 x 6 block of every pair of optimisable
// keyframes is split into six rows, and each thread owns up to six such rows (their
// partial sums stay in FP64 registers, so no two threads ever add into the same entry
// and no atomics touch S).  The tile is walked in chunks of whole points holding at most
// CO observations (CO = 512 for FP32 arithmetic, 256 for FP64); per chunk:
//   1. one thread per observation forms the residual (FP64), the robust weight, the
//      Gauss-Newton blocks Hll_a, W_a, Hpp_a in factored form (Real) and the gradient
//      pieces bl_a, bp_a (FP64);
//   2. the threads of each point sum Hll (Real) and bl (FP64) through LDS, factor
//      V = Hll + lambda I = L L^T, and stage Z_a = W_a L^-T, D_a = Hpp_a - Z_a Z_a^T and
//      r_a = bp_a - Z_a L^-1 bl (so W_a V^-1 W_b^T = Z_a Z_b^T) in LDS;
//   3. every pair (a, b), a <= b, of optimisable observations of one point is counted
//      and then placed, by camera block, into a block-sorted pair list (LDS integer
//      atomics give each pair its slot in its block's list);
//   4. every owner walks the pair lists of its block rows and accumulates -Z_a Z_b^T
//      (or D_a for a pair of an observation with itself); the owners of r walk the
//      diagonal-block lists.
// At the end of the tile each owner writes its rows to the tile's partial system; a
// separate kernel sums the partials of a window in a fixed order (no global atomics).
// The gradient bp itself is not needed: the gain-ratio denominator uses
// dp^T bp = dp^T r + sum_j q_j^T V_j^-1 bl_j (q_j = sum_a W_a^T dp), whose point part
// the update kernel forms.
//
// INIT mode computes only what the damping initialisation needs: the cost, the diagonal
// of Hpp per camera (in the r slots) and the largest point-block diagonal.
#include "lba_internal.h"

namespace lba {

constexpr int kNT = kLinThreads;           // 512
constexpr int kSlots = 6;                  // block rows per thread (6 * 512 >= 6 * 465)
constexpr int kMaxBlocks = 465;            // Kopt <= 30
constexpr int kMaxN = 180;

template <typename Real>
struct LinCfg {
    static constexpr int CO = sizeof(Real) == 4 ? 512 : 256;          // observations per chunk
    static constexpr int PCAP = sizeof(Real) == 4 ? 4096 : 2080;      // pairs per chunk (>= 64*65/2)
};

template <typename Real>
struct LinSmem {
    double *T;       // K x 12 poses
    int *opt;        // K
    Real *Z;         // CO x 18
    Real *D;         // CO x 21   lower triangle of Hpp_a - Z_a Z_a^T (phase 1: FP64 Hll_a, 6 each)
    double *rd;      // CO x 6    (phase 1: bl_a in the first 3) r_a
    double *hd;      // kMaxN: INIT only, diagonal of Hpp
    unsigned *pairs; // PCAP
    int *cnt;        // kMaxBlocks + 1 (then list offsets)
    int *cur;        // kMaxBlocks
    int *oka;        // CO: optimisable camera of the chunk observation (-1: none)
    int *oseg;       // CO: s0 | s1 << 16 (chunk-local observation range of its point)
    int *scan;       // 16: per-wavefront totals
    double *red;     // 16 x 2
};

static __host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

template <typename Real>
__host__ __device__ inline size_t lin_carve(unsigned char *base, int K, LinSmem<Real> *s) {
    using C = LinCfg<Real>;
    size_t o = 0;
    auto take = [&](size_t bytes) { void *p = base ? (void *)(base + o) : nullptr; o = align_up(o + bytes, 16); return p; };
    void *T = take(sizeof(double) * 12 * K);
    void *opt = take(sizeof(int) * K);
    void *Z = take(sizeof(Real) * C::CO * 18);
    void *D = take(sizeof(Real) * C::CO * 21);
    void *rd = take(sizeof(double) * C::CO * 6);
    void *pairs = take(sizeof(unsigned) * C::PCAP);
    void *cnt = take(sizeof(int) * (kMaxBlocks + 1));
    void *cur = take(sizeof(int) * kMaxBlocks);
    void *oka = take(sizeof(int) * C::CO);
    void *oseg = take(sizeof(int) * C::CO);
    void *scan = take(sizeof(int) * 16);
    void *red = take(sizeof(double) * 32);
    void *hd = take(sizeof(double) * kMaxN);
    if (s) {
        s->T = (double *)T; s->opt = (int *)opt; s->Z = (Real *)Z; s->D = (Real *)D; s->rd = (double *)rd;
        s->pairs = (unsigned *)pairs; s->cnt = (int *)cnt; s->cur = (int *)cur; s->oka = (int *)oka;
        s->oseg = (int *)oseg; s->scan = (int *)scan; s->red = (double *)red; s->hd = (double *)hd;
    }
    return o;
}

size_t lin_lds_bytes(int K, int n, int waves, bool mixed) {
    (void)n;
    (void)waves;
    return mixed ? lin_carve<float>(nullptr, K, nullptr) : lin_carve<double>(nullptr, K, nullptr);
}

// index of block (ka <= kb) of the upper block triangle, row-major
__device__ __forceinline__ int block_id(int ka, int kb, int Kopt) { return ka * Kopt - ka * (ka - 1) / 2 + (kb - ka); }

// inclusive scan of one int per thread over the block (512 threads)
__device__ __forceinline__ int block_inclusive_scan(int v, int *scan, int tid) {
    const int lane = tid & 63, wave = tid >> 6;
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) scan[wave] = x;
    __syncthreads();
    int add = 0;
    for (int w = 0; w < wave; ++w) add += scan[w];
    __syncthreads();
    return x + add;
}

template <typename Real, typename ZT, bool INIT>
__global__ __launch_bounds__(kNT) void k_linearize(LinArgs a) {
    using C = LinCfg<Real>;
    extern __shared__ __align__(16) unsigned char smem[];
    const Tile tile = a.tiles[blockIdx.x];
    const WinInfo W = a.win[tile.win];
    const Ctl ctl = a.ctl[tile.win];
    if (!INIT && !ctl.running) return;
    const int K = W.K, n = W.n, E = W.E, Kopt = W.Kopt;
    const int nblk = Kopt * (Kopt + 1) / 2;
    LinSmem<Real> sm;
    lin_carve<Real>(smem, K, &sm);
    const double lambda = ctl.lambda;
    const double *Xs = ctl.cur ? a.X1 : a.X0;
    const int tid = threadIdx.x;

    for (int i = tid; i < 12 * K; i += kNT) sm.T[i] = a.T[(int64_t)W.kf0 * 12 + i];
    for (int i = tid; i < K; i += kNT) sm.opt[i] = a.opt_map[W.kf0 + i];

    // ---- owned block rows: slot s = tid + k * kNT -> block s / 6 (kA <= kB), row s % 6 ----
    const int nslot = INIT ? 0 : 6 * nblk;
    double acc[kSlots][6];
#pragma unroll
    for (int k = 0; k < kSlots; ++k)
#pragma unroll
        for (int j = 0; j < 6; ++j) acc[k][j] = 0.0;
    double racc = 0.0;   // r[tid] (INIT: Hpp diagonal entry tid)
    __syncthreads();

    const CamParams cam = a.c.cam;
    double Facc = 0.0, mdiag = 0.0;
    int fail = 0;

    for (int p = tile.p0; p < tile.p1;) {
        // ---- chunk of whole points: <= CO observations and <= PCAP pairs ------------
        const int base = a.pt_start[p];
        const int cand = p + tid;
        int mpairs = 0, inrange = 0, obs_incl = 0;
        if (cand < tile.p1) {
            const int e = a.pt_start[cand + 1];
            const int m = e - a.pt_start[cand];
            mpairs = m * (m + 1) / 2;
            obs_incl = e - base;
            inrange = 1;
        }
        const int pincl = block_inclusive_scan(mpairs, sm.scan, tid);
        const int ok = inrange && obs_incl <= C::CO && pincl <= C::PCAP;
        const int q = p + __syncthreads_count(ok);
        if (q == p) {   // one point exceeds a chunk: not solvable here
            fail = 1;
            break;
        }
        const int nob = a.pt_start[q] - base;
        const bool has = tid < nob;
        const int o = base + tid;

        // ---- 1. per-observation terms -------------------------------------------------
        // (only the raw observation stays in registers across the point-sum barrier; the
        //  factored blocks are recomputed from it in phase 2)
        int s0 = 0, s1 = 0, ka = -1, kl = 0, stereo = 0;
        bool act = false;
        double zu = 0, zv = 0, zr = 0, X0 = 0, X1 = 0, X2 = 0, omd = 0.0;
        double rho = 0.0;
        if (has) {
            const int jl = a.obs.pt[o];
            const int j = W.pt0 + jl;
            s0 = a.pt_start[j] - base;
            s1 = a.pt_start[j + 1] - base;
            kl = a.obs.kf[o];
            ka = sm.opt[kl];
            act = !a.mask || !a.mask[o];
            stereo = a.obs.type[o];
            load_z<ZT>(a.obs, o, zu, zv, zr);
            X0 = Xs[3 * (int64_t)j];
            X1 = Xs[3 * (int64_t)j + 1];
            X2 = Xs[3 * (int64_t)j + 2];
            const double *T = sm.T + kl * 12;
            double xc, yc, zc, eu, ev, er;
            const double e2 = residual(cam, T, X0, X1, X2, zu, zv, zr, stereo, xc, yc, zc, eu, ev, er);
            const double isg = a.c.inv_sigma2[a.obs.oct[o]];
            double w;
            huber(e2 * isg, a.c.huber2[stereo], a.robust, rho, w);
            if (!act) rho = 0.0;
            omd = act ? w * isg : 0.0;
            double Hll[6], bl[3];
            point_block_fp64(cam, T, xc, yc, zc, eu, ev, er, stereo, omd, Hll, bl);
            double *hs = reinterpret_cast<double *>(sm.D);
#pragma unroll
            for (int i = 0; i < 6; ++i) hs[tid * 6 + i] = Hll[i];
#pragma unroll
            for (int i = 0; i < 3; ++i) sm.rd[tid * 6 + i] = bl[i];
            if (!act) ka = -1;
            sm.oka[tid] = ka;
            sm.oseg[tid] = s0 | (s1 << 16);
        }
        Facc += rho;
        __syncthreads();

        // ---- 2. per-point sums, point factor, staged Z_a, D_a, r_a ---------------------
        double V[6] = {0, 0, 0, 0, 0, 0};
        double bs[3] = {0, 0, 0};
        if (has) {
            const double *hs = reinterpret_cast<const double *>(sm.D);
            for (int m = s0; m < s1; ++m) {
#pragma unroll
                for (int i = 0; i < 6; ++i) V[i] += hs[m * 6 + i];
#pragma unroll
                for (int i = 0; i < 3; ++i) bs[i] += sm.rd[m * 6 + i];
            }
        }
        if (INIT && tid < n) sm.hd[tid] = 0.0;
        __syncthreads();
        if (INIT) {
            if (has && tid == s0) mdiag = fmax(mdiag, fmax(V[0], fmax(V[3], V[5])));
            if (ka >= 0) {
                const double *T = sm.T + kl * 12;
                double xc, yc, zc, eu, ev, er;
                residual(cam, T, X0, X1, X2, zu, zv, zr, stereo, xc, yc, zc, eu, ev, er);
                ObsBlocks<Real> Bk;
                obs_blocks<Real>(cam, T, xc, yc, zc, eu, ev, er, stereo, (Real)omd, Bk);
                Real H[36], bpa[6];
                pose_terms<Real>(Bk, H, bpa);
                // diagonal of Hpp_a into the block's LDS sums (entry order rotated by thread)
                const int rot = tid % 6;
                for (int e = 0; e < 6; ++e) {
                    int i = e + rot;
                    i -= i >= 6 ? 6 : 0;
                    double v = 0.0;
#pragma unroll
                    for (int c = 0; c < 6; ++c)
                        if (c == i) v = (double)H[c * 7];
                    lds_add(&sm.hd[ka * 6 + i], v);
                }
            }
            __syncthreads();
            if (tid < n) racc += sm.hd[tid];
            __syncthreads();
            p = q;
            continue;
        }
        double Li[6] = {0, 0, 0, 0, 0, 0};
        double t0 = 0, t1 = 0, t2 = 0;
        if (has) {
            V[0] += lambda;
            V[3] += lambda;
            V[5] += lambda;
            if (!chol3_inv<double>(V, Li)) fail = 1;
            lmul<double>(Li, bs[0], bs[1], bs[2], t0, t1, t2);
        }
        if (ka >= 0) {
            const double *T = sm.T + kl * 12;
            double xc, yc, zc, eu, ev, er;
            residual(cam, T, X0, X1, X2, zu, zv, zr, stereo, xc, yc, zc, eu, ev, er);
            ObsBlocks<Real> Bk;
            obs_blocks<Real>(cam, T, xc, yc, zc, eu, ev, er, stereo, (Real)omd, Bk);
            double gd[3];
            obs_gradient(cam, xc, yc, zc, eu, ev, er, stereo, omd, gd);
            Real Wm[18], H[36], bpa[6], Zr[18];
            pose_point_block<Real>(Bk, Wm);
            pose_terms<Real>(Bk, H, bpa);
#pragma unroll
            for (int i = 0; i < 6; ++i) {
                double z0, z1, z2;
                lmul<double>(Li, (double)Wm[i * 3], (double)Wm[i * 3 + 1], (double)Wm[i * 3 + 2], z0, z1, z2);
                Zr[i * 3] = (Real)z0;
                Zr[i * 3 + 1] = (Real)z1;
                Zr[i * 3 + 2] = (Real)z2;
            }
            // bp_a = (x cross g ; g) in FP64, r_a = bp_a - Z_a t
            double bpd[6];
            bpd[0] = yc * gd[2] - zc * gd[1];
            bpd[1] = zc * gd[0] - xc * gd[2];
            bpd[2] = xc * gd[1] - yc * gd[0];
            bpd[3] = gd[0]; bpd[4] = gd[1]; bpd[5] = gd[2];
#pragma unroll
            for (int i = 0; i < 6; ++i)
                sm.rd[tid * 6 + i] =
                    bpd[i] - ((double)Zr[i * 3] * t0 + (double)Zr[i * 3 + 1] * t1 + (double)Zr[i * 3 + 2] * t2);
#pragma unroll
            for (int i = 0; i < 18; ++i) sm.Z[tid * 18 + i] = Zr[i];
            int e = 0;
#pragma unroll
            for (int i = 0; i < 6; ++i)
#pragma unroll
                for (int j = 0; j <= i; ++j, ++e)
                    sm.D[tid * 21 + e] =
                        H[i * 6 + j] - (Zr[i * 3] * Zr[j * 3] + Zr[i * 3 + 1] * Zr[j * 3 + 1] + Zr[i * 3 + 2] * Zr[j * 3 + 2]);
        }
        for (int B = tid; B < nblk; B += kNT) {
            sm.cnt[B] = 0;
            sm.cur[B] = 0;
        }
        __syncthreads();

        // ---- 3. pair lists sorted by camera block --------------------------------------
        if (ka >= 0) {
            for (int b = tid; b < s1; ++b) {
                const int kb = sm.oka[b];
                if (kb < 0) continue;
                atomicAdd(&sm.cnt[ka <= kb ? block_id(ka, kb, Kopt) : block_id(kb, ka, Kopt)], 1);
            }
        }
        __syncthreads();
        {
            const int v = tid < nblk ? sm.cnt[tid] : 0;
            const int incl = block_inclusive_scan(v, sm.scan, tid);
            if (tid < nblk) sm.cnt[tid] = incl - v;   // exclusive offsets
            if (tid == nblk - 1) sm.cnt[nblk] = incl;
        }
        __syncthreads();
        if (ka >= 0) {
            for (int b = tid; b < s1; ++b) {
                const int kb = sm.oka[b];
                if (kb < 0) continue;
                const int B = ka <= kb ? block_id(ka, kb, Kopt) : block_id(kb, ka, Kopt);
                const int pos = sm.cnt[B] + atomicAdd(&sm.cur[B], 1);
                // first = the observation on the lower camera; flag 1 = a with itself,
                // flag 2 = two observations of one point on the same camera
                const int first = ka <= kb ? tid : b, second = ka <= kb ? b : tid;
                const unsigned fl = b == tid ? 1u : (ka == kb ? 2u : 0u);
                sm.pairs[pos] = (unsigned)first | ((unsigned)second << 10) | (fl << 20);
            }
        }
        __syncthreads();

        // ---- 4. owners accumulate their block rows and r -------------------------------
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            const int s_ = tid + k * kNT;
            if (s_ >= nslot) continue;
            const int B = s_ / 6, i = s_ - 6 * B;
            const int p0 = sm.cnt[B], p1 = sm.cnt[B + 1];
            for (int pi = p0; pi < p1; ++pi) {
                const unsigned e = sm.pairs[pi];
                const int la = e & 1023, lb = (e >> 10) & 1023, fl = e >> 20;
                if (fl == 1) {
                    const Real *d = sm.D + la * 21 + i * (i + 1) / 2;
#pragma unroll
                    for (int j = 0; j < 6; ++j)
                        if (j <= i) acc[k][j] += (double)d[j];
                } else {
                    const Real *za = sm.Z + la * 18, *zb = sm.Z + lb * 18;
                    const Real a0 = za[i * 3], a1 = za[i * 3 + 1], a2 = za[i * 3 + 2];
                    if (fl == 0) {
#pragma unroll
                        for (int j = 0; j < 6; ++j)
                            acc[k][j] -= (double)(a0 * zb[j * 3] + a1 * zb[j * 3 + 1] + a2 * zb[j * 3 + 2]);
                    } else {
                        const Real c0 = zb[i * 3], c1 = zb[i * 3 + 1], c2 = zb[i * 3 + 2];
#pragma unroll
                        for (int j = 0; j < 6; ++j)
                            if (j <= i)
                                acc[k][j] -= (double)(a0 * zb[j * 3] + a1 * zb[j * 3 + 1] + a2 * zb[j * 3 + 2] +
                                                      c0 * za[j * 3] + c1 * za[j * 3 + 1] + c2 * za[j * 3 + 2]);
                    }
                }
            }
        }
        if (tid < n) {
            const int kc = tid / 6, ic = tid % 6;
            const int B = block_id(kc, kc, Kopt);
            for (int pi = sm.cnt[B]; pi < sm.cnt[B + 1]; ++pi) {
                const unsigned e = sm.pairs[pi];
                if ((e >> 20) == 1) racc += sm.rd[(e & 1023) * 6 + ic];
            }
        }
        __syncthreads();
        p = q;
    }

    // ---- write-out: owned rows of S, r, and the tile's scalars ----------------------
    const int t = blockIdx.x;
    if (!INIT) {
        double *part = a.part + W.part_off + (int64_t)(t - W.tile0) * W.part_stride;
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            const int s_ = tid + k * kNT;
            if (s_ >= nslot) continue;
            const int B = s_ / 6, i = s_ - 6 * B;
            int kA = 0;
            while (kA + 1 < Kopt && block_id(kA + 1, kA + 1, Kopt) <= B) ++kA;
            const int kB = kA + (B - block_id(kA, kA, Kopt));
            const int ra = 6 * kA + i, cb = 6 * kB;
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                if (kA == kB && j > i) continue;
                const int col = cb + j;
                part[ra >= col ? packed_lower(ra, col) : packed_lower(col, ra)] = acc[k][j];
            }
        }
    }
    if (tid < n) a.partr[W.partr_off + (int64_t)(t - W.tile0) * n + tid] = racc;
    Facc = wave_sum(Facc);
    mdiag = wave_max(mdiag);
    const int anyfail = __syncthreads_or(fail);
    if ((tid & 63) == 0) {
        sm.red[(tid >> 6) * 2] = Facc;
        sm.red[(tid >> 6) * 2 + 1] = mdiag;
    }
    __syncthreads();
    if (tid == 0) {
        double F = 0.0, md = 0.0;
        for (int w = 0; w < kNT / 64; ++w) {
            F += sm.red[w * 2];
            md = fmax(md, sm.red[w * 2 + 1]);
        }
        a.partd[4 * t] = F;
        a.partd[4 * t + 1] = md;
        a.partd[4 * t + 2] = anyfail ? 1.0 : 0.0;
        a.partd[4 * t + 3] = 0.0;
    }
    (void)E;
}

hipError_t launch_linearize(const LinArgs &a, int ntiles, size_t lds, bool init, bool mixed,
                            hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    dim3 grid(ntiles), block(kNT);
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
