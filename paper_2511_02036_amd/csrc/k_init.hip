// Damping initialisation pass: per tile, the robust cost, the diagonal of the pose blocks
// of the Gauss-Newton matrix per optimisable camera, and the largest diagonal entry of the
// point blocks, at the start of an LM round (lambda_0 = tau * max diag H).
//
// One 256-thread block per tile of points; each of the four wavefronts walks its share of
// the tile's points in chunks of whole points with at most 64 observations (one per
// lane).  Per observation, in FP64: the residual, the robust weight w = rho'(s) and
// G = (w / sigma^2) P^T P (P = d pi / d Xc); the pose-block diagonal is
//   ([x]x G [x]x^T)_ii  (rotation)  and  G_ii  (translation),  x = Xc,
// and the point-block diagonal is diag(R^T G R).  The point sums are formed by the first
// lane of each point; the camera sums go into per-wavefront LDS rows (LDS atomics within
// one wavefront), added in a fixed order at the end of the tile.
#include "lba_internal.h"

namespace lba {

constexpr int kInitThreads = 256;
constexpr int kInitWaves = kInitThreads / kWave;

static __host__ __device__ inline size_t init_align(size_t x) { return (x + 15) / 16 * 16; }

size_t init_lds_bytes(int K, int n) {
    size_t o = init_align(sizeof(double) * (12 * K + kMaxLevels + 2));   // poses, weights
    o += init_align(sizeof(int) * K);                          // optimisable index
    o += init_align(sizeof(double) * kInitWaves * (n > 0 ? n : 1));   // per-wave camera rows
    o += init_align(sizeof(double) * kInitWaves * 64 * 3);     // point-block diagonals
    o += init_align(sizeof(double) * kInitWaves * 64 * 3);     // point positions
    o += init_align(sizeof(int) * kInitWaves * 65);            // observation ranges
    o += sizeof(double) * kInitWaves * 3;
    return o;
}

__global__ __launch_bounds__(kInitThreads) void k_init(LinArgs a) {
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = a.order[blockIdx.x];
    const Tile tile = a.tiles[t];
    const WinInfo W = a.win[tile.win];
    const Ctl ctl = a.ctl[tile.win];
    const int K = W.K, n = W.n;
    unsigned char *cur = smem;
    double *T = reinterpret_cast<double *>(cur);
    double *wt = T + 12 * K;   // 1 / sigma2 per octave (32), Huber thresholds mono, stereo
    cur += init_align(sizeof(double) * (12 * K + kMaxLevels + 2));
    int *opt = reinterpret_cast<int *>(cur);
    cur += init_align(sizeof(int) * K);
    double *hdw = reinterpret_cast<double *>(cur);
    cur += init_align(sizeof(double) * kInitWaves * (n > 0 ? n : 1));
    double *stg = reinterpret_cast<double *>(cur);
    cur += init_align(sizeof(double) * kInitWaves * 64 * 3);
    double *xsa = reinterpret_cast<double *>(cur);
    cur += init_align(sizeof(double) * kInitWaves * 64 * 3);
    int *psa = reinterpret_cast<int *>(cur);
    cur += init_align(sizeof(int) * kInitWaves * 65);
    double *red = reinterpret_cast<double *>(cur);

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    for (int i = tid; i < 12 * K; i += kInitThreads) T[i] = a.T[(int64_t)W.kf0 * 12 + i];
    for (int i = tid; i < K; i += kInitThreads) opt[i] = a.opt_map[W.kf0 + i];
    // the weights by octave and type, read per observation: from LDS rather than from the
    // kernel arguments (one dependent memory round trip less per chunk)
    if (tid < kMaxLevels + 2) wt[tid] = tid < kMaxLevels ? a.c.inv_sigma2[tid] : a.c.huber2[tid - kMaxLevels];
    for (int i = tid; i < kInitWaves * n; i += kInitThreads) hdw[i] = 0.0;
    __syncthreads();

    const double *Xs = ctl.cur ? a.X1 : a.X0;
    const CamParams cam = a.c.cam;
    double *hw = hdw + wave * n, *st = stg + wave * 64 * 3, *xs = xsa + wave * 64 * 3;
    int *pst = psa + wave * 65;
    const int np = tile.p1 - tile.p0;
    const int wp0 = tile.p0 + (int)(((int64_t)np * wave) / kInitWaves);
    const int wp1 = tile.p0 + (int)(((int64_t)np * (wave + 1)) / kInitWaves);
    double F = 0.0, md = 0.0;
    int fail = 0;

    for (int p = wp0; p < wp1;) {
        const int base = a.pt_start[p];
        const int cand = p + lane;
        int ok = 0, e = 0;
        if (cand < wp1) {
            e = a.pt_start[cand + 1] - base;
            ok = e <= kMaxObsPerPoint;
        }
        const int q = p + __popcll(__ballot(ok));
        if (q == p) {   // a point with more observations than one wavefront
            fail = 1;
            break;
        }
        const int npts = q - p;
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
        double zu = 0, zv = 0, zr = 0;
        if (o < a.obs.n_obs) {
            jl = a.obs.pt[o];
            kl = a.obs.kf[o];
            // the flag is loaded without a branch (from a readable byte array when there
            // is none), so that it issues with the other loads
            const uint8_t flag = (a.mask ? a.mask : a.obs.type)[o];
            act = (a.mask == nullptr) | (flag == 0);
            stereo = a.obs.type[o];
            oct = a.obs.oct[o];
            if (a.obs.z_f32) load_z<float>(a.obs, o, zu, zv, zr);
            else load_z<double>(a.obs, o, zu, zv, zr);
        }
        wave_sync();
        const int nob = pst[npts];
        const bool has = lane < nob;
        int s0 = 0, s1 = 0;
        double h0 = 0.0, h1 = 0.0, h2 = 0.0;
        if (has) {
            const int pl = W.pt0 + jl - p;
            s0 = pst[pl];
            s1 = pst[pl + 1];
            if (act) {
                const double *Tk = T + kl * 12;
                double xc, yc, zc, eu, ev, er;
                const double e2 = residual(cam, Tk, xs[3 * pl], xs[3 * pl + 1], xs[3 * pl + 2], zu, zv, zr, stereo,
                                           xc, yc, zc, eu, ev, er);
                const double isg = wt[oct];
                double rho, w;
                huber(e2 * isg, wt[kMaxLevels + stereo], a.robust, rho, w);
                F += rho;
                const double om = w * isg;
                const double iz = 1.0 / zc, sf = stereo ? 1.0 : 0.0;
                const double p00 = cam.fx * iz, p02 = -cam.fx * xc * iz * iz;
                const double p11 = cam.fy * iz, p12 = -cam.fy * yc * iz * iz;
                const double p22 = -(cam.fx * xc - cam.bf) * iz * iz;
                const double G00 = om * (p00 * p00 * (1.0 + sf)), G02 = om * (p00 * p02 + sf * p00 * p22);
                const double G11 = om * (p11 * p11), G12 = om * (p11 * p12);
                const double G22 = om * (p02 * p02 + p12 * p12 + sf * p22 * p22);
                // point block diagonal: (R^T G R)_ii with R the rotation of the pose
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const double r0 = Tk[i], r1 = Tk[4 + i], r2 = Tk[8 + i];
                    const double v = G00 * r0 * r0 + G11 * r1 * r1 + G22 * r2 * r2 + 2.0 * (G02 * r0 * r2 + G12 * r1 * r2);
                    if (i == 0) h0 = v; else if (i == 1) h1 = v; else h2 = v;
                }
                const int ka = opt[kl];
                if (ka >= 0) {
                    const double d[6] = {G11 * zc * zc - 2.0 * G12 * yc * zc + G22 * yc * yc,
                                         G00 * zc * zc - 2.0 * G02 * xc * zc + G22 * xc * xc,
                                         G00 * yc * yc + G11 * xc * xc,
                                         G00, G11, G22};
#pragma unroll
                    for (int i = 0; i < 6; ++i) lds_add(hw + 6 * ka + i, d[i]);
                }
            }
        }
        st[lane * 3] = h0;
        st[lane * 3 + 1] = h1;
        st[lane * 3 + 2] = h2;
        wave_sync();
        if (has && lane == s0) {   // the point's block diagonal
            double v0 = 0.0, v1 = 0.0, v2 = 0.0;
            for (int m = s0; m < s1; ++m) {
                v0 += st[m * 3];
                v1 += st[m * 3 + 1];
                v2 += st[m * 3 + 2];
            }
            md = fmax(md, fmax(v0, fmax(v1, v2)));
        }
        wave_sync();
        p = q;
    }

    F = wave_sum(F);
    md = wave_max(md);
    const int anyfail = __syncthreads_or(fail);
    if (lane == 0) {
        red[wave * 3] = F;
        red[wave * 3 + 1] = md;
    }
    __syncthreads();
    double *pr = a.partr + W.partr_off + (int64_t)(t - W.tile0) * n;
    for (int i = tid; i < n; i += kInitThreads) {
        double v = 0.0;
        for (int w = 0; w < kInitWaves; ++w) v += hdw[w * n + i];
        pr[i] = v;
    }
    if (tid == 0) {
        double Ft = 0.0, mt = 0.0;
        for (int w = 0; w < kInitWaves; ++w) {
            Ft += red[w * 3];
            mt = fmax(mt, red[w * 3 + 1]);
        }
        a.partd[4 * t] = Ft;
        a.partd[4 * t + 1] = mt;
        a.partd[4 * t + 2] = anyfail ? 1.0 : 0.0;
        a.partd[4 * t + 3] = 0.0;
    }
}

size_t init_static_lds() { return kernel_static_lds((const void *)k_init); }

hipError_t launch_init(const LinArgs &a, int ntiles, size_t lds, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init, dim3(ntiles), dim3(kInitThreads), lds, s, a);
    return hipGetLastError();
}

}  // namespace lba
