// Candidate search of map-point fusion (Sections III-B and IV-D): for each map point of
// the current keyframe and each neighbour keyframe, the keypoint of the neighbour that
// the point most likely duplicates.  One thread per (query, point), as the paper
// assigns them; the fuse itself stays with the caller.
//
// Each thread projects its point, applies the depth, image, distance-range and
// viewing-angle gates and predicts the octave, then visits only the 16x16-pixel cells of
// the store's index that can hold a keypoint within the search radius (one pixel of
// margin on each side, far above any rounding of the FP64 window test), so the result
// equals a scan over all keypoints of the neighbour.  The best (distance, index) is kept
// lexicographically, so the order of the visit does not matter.
#include "lmap_internal.h"

namespace lmap {

__device__ inline int hamming256(const uint32_t *a, const uint32_t *b) {
    int d = 0;
#pragma unroll
    for (int w = 0; w < 8; ++w) d += __popc(a[w] ^ b[w]);
    return d;
}

__global__ __launch_bounds__(256) void k_fuse(FuseArgs a) {
#pragma clang fp contract(off)
    const int q = blockIdx.x;
    const int n = a.nbr[q];
    const int p0 = a.p0[q], p1 = a.p1[q];
    if (n < 0 || n >= a.s.n_kf || p0 < 0 || p1 > a.n_pt || p1 < p0) return;
    const StoreView &s = a.s;
    const double *T = s.T + 12 * (size_t)n;
    // camera centre -R^T t
    double O[3];
    for (int i = 0; i < 3; ++i) {
        double acc = T[i] * T[3];
        acc = acc + T[4 + i] * T[7];
        acc = acc + T[8 + i] * T[11];
        O[i] = -acc;
    }
    const int kb = s.kp_off[n];
    const int32_t *coff = s.cell_off + (size_t)n * (s.ncells + 1);
    const int32_t *ckp = s.cell_kp + kb;
    for (int p = p0 + blockIdx.y * 256 + threadIdx.x; p < p1; p += gridDim.y * 256) {
        const int64_t o = a.out_off[q] + (p - p0);
        if (o < 0 || o >= a.n_out) continue;
        if (a.skip && a.skip[o]) continue;
        const double *Xp = a.X + 3 * (size_t)p;
        double Xc[3];
        for (int i = 0; i < 3; ++i) {
            double acc = T[i * 4] * Xp[0];
            acc = acc + T[i * 4 + 1] * Xp[1];
            acc = acc + T[i * 4 + 2] * Xp[2];
            Xc[i] = acc + T[i * 4 + 3];
        }
        if (!(Xc[2] > 0.0)) continue;
        const double iz = 1.0 / Xc[2];
        const double u = s.fx * Xc[0] * iz + s.cx;
        const double v = s.fy * Xc[1] * iz + s.cy;
        if (!(u >= 0.0 && u < (double)s.width && v >= 0.0 && v < (double)s.height)) continue;
        const double ur = u - s.bf * iz;
        const double PO[3] = {Xp[0] - O[0], Xp[1] - O[1], Xp[2] - O[2]};
        const double d2 = (PO[0] * PO[0] + PO[1] * PO[1]) + PO[2] * PO[2];
        const double lo = a.dmin[p], hi = a.dmax[p];
        if (d2 < lo * lo || d2 > hi * hi) continue;
        const double *nv = a.normal + 3 * (size_t)p;
        const double dot = (PO[0] * nv[0] + PO[1] * nv[1]) + PO[2] * nv[2];
        if (!(dot > 0.0) || dot * dot < 0.25 * d2) continue;
        int level = 0;
        while (level < s.n_levels - 1 && s.scale[level] * s.scale[level] * d2 < hi * hi) ++level;
        const double radius = a.radius_th * s.scale[level];
        uint32_t pd[8];
        for (int w = 0; w < 8; ++w) pd[w] = a.pdesc[8 * (size_t)p + w];
        // cells that can hold a keypoint with |ku - u| < radius and |kv - v| < radius
        const int cx0 = (int)fmax(0.0, floor((u - radius - 1.0) / kCell));
        const int cx1 = (int)fmin((double)(s.ncx - 1), floor((u + radius + 1.0) / kCell));
        const int cy0 = (int)fmax(0.0, floor((v - radius - 1.0) / kCell));
        const int cy1 = (int)fmin((double)(s.ncy - 1), floor((v + radius + 1.0) / kCell));
        uint32_t best = 0xffffffffu;
        for (int cy = cy0; cy <= cy1; ++cy) {
            const int e0 = coff[cy * s.ncx + cx0], e1 = coff[cy * s.ncx + cx1 + 1];
            for (int e = e0; e < e1; ++e) {
                const int jl = ckp[e];
                const int j = kb + jl;
                const double ku = s.u[j], kv = s.v[j];
                if (!(fabs(ku - u) < radius && fabs(kv - v) < radius)) continue;
                const int ko = s.oct[j];
                if (ko < level - 1 || ko > level) continue;
                const double ex = u - ku, ey = v - kv;
                const float kur = s.ur[j];
                if (kur >= 0.0f) {
                    const double er = ur - (double)kur;
                    const double e2 = (ex * ex + ey * ey) + er * er;
                    if (e2 > a.chi2_stereo * s.sigma2[ko]) continue;
                } else {
                    const double e2 = ex * ex + ey * ey;
                    if (e2 > a.chi2_mono * s.sigma2[ko]) continue;
                }
                const int d = hamming256(pd, s.desc + 8 * (size_t)j);
                if (d > a.th_low) continue;
                const uint32_t key = ((uint32_t)d << kKpBits) | (uint32_t)jl;
                best = min(best, key);
            }
        }
        if (best != 0xffffffffu) {
            a.match[o] = (int32_t)(best & kKpMask);
            a.dist[o] = (int32_t)(best >> kKpBits);
        }
    }
}

// Validation: query ranges, output offsets, the neighbour index and the point data.
__global__ __launch_bounds__(256) void k_fuse_check(FuseArgs a) {
    for (int q = blockIdx.x * 256 + threadIdx.x; q <= a.n_q; q += gridDim.x * 256) {
        const int64_t o = a.out_off[q];
        if (q == 0 && o != 0) atomicAdd(&a.err[kErrOutOff], 1);
        if (q == a.n_q) {
            if (o < 0 || o > a.n_out) atomicAdd(&a.err[kErrOutOff], 1);
        } else {
            const int n = a.nbr[q], p0 = a.p0[q], p1 = a.p1[q];
            if (n < 0 || n >= a.s.n_kf || p0 < 0 || p1 > a.n_pt || p1 < p0) atomicAdd(&a.err[kErrQuery], 1);
            else if (a.out_off[q + 1] - o != (int64_t)(p1 - p0)) atomicAdd(&a.err[kErrOutOff], 1);
        }
    }
    for (int p = blockIdx.x * 256 + threadIdx.x; p < a.n_pt; p += gridDim.x * 256) {
        bool ok = isfinite(a.dmin[p]) && isfinite(a.dmax[p]);
        for (int i = 0; i < 3; ++i) ok = ok && isfinite(a.X[3 * (size_t)p + i]) && isfinite(a.normal[3 * (size_t)p + i]);
        if (!ok) atomicAdd(&a.err[kErrPoint], 1);
    }
}

void launch_fuse_check(const FuseArgs &a, hipStream_t s) {
    const int items = std::max(a.n_q + 1, a.n_pt);
    const unsigned blocks = (unsigned)std::min(4096, (items + 255) / 256);
    prof_begin(LMAP_KCLASS_CHECK, s);
    hipLaunchKernelGGL(k_fuse_check, dim3(blocks), dim3(256), 0, s, a);
    prof_end(s);
}

void launch_fuse(const FuseArgs &a, hipStream_t s) {
    launch_fill_i32(a.match, a.n_out, -1, s);
    launch_fill_i32(a.dist, a.n_out, -1, s);
    if (a.n_q == 0) return;
    prof_begin(LMAP_KCLASS_FUSE, s);
    hipLaunchKernelGGL(k_fuse, dim3(a.n_q, a.blocks_per_q), dim3(256), 0, s, a);
    prof_end(s);
}

}  // namespace lmap
