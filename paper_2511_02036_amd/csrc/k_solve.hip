// Reduced camera system: fixed-order reduction of the per-tile partial sums, FP64 dense
// Cholesky and triangular solves for the pose step, and the per-window Levenberg-
// Marquardt decision (gain ratio, accept / reject, damping update, pose retraction).
#include "lba_internal.h"

#include <algorithm>

namespace lba {

// ------------------------------------------------------------------------------------
// partial sums -> reduced system.  Each block owns 64 entries of one window; its four
// wavefronts sum the tiles t = g, g + 4, ... (g = wavefront) and the four partial sums
// are combined in a fixed order, so the result does not depend on scheduling.
// ------------------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_reduce(ReduceArgs a) {
    __shared__ double acc4[4][64];
    const int w = blockIdx.y;
    const WinInfo W = a.win[w];
    if (!a.ctl[w].running) return;
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int i = blockIdx.x * 64 + lane;
    const int tot = W.E + W.n;
    if (blockIdx.x == 0 && g == 0) {
        // the window's point-block failure flag (written even when the system is empty)
        double fl = 0.0;
        for (int t = lane; t < W.ntiles; t += 64) fl = fmax(fl, a.partd[4 * (W.tile0 + t) + 2]);
        fl = wave_max(fl);
        if (lane == 0) a.redflag[w] = fl;
    }
    if (blockIdx.x * 64 >= tot) return;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;   // four loads in flight per step
    const double *src = nullptr;
    int64_t stride = 0;
    if (i < W.E) {
        src = a.part + W.part_off + i;
        stride = W.part_stride;
    } else if (i < tot) {
        src = a.partr + W.partr_off + (i - W.E);
        stride = W.n;
    }
    if (src) {
        int t = g;
        for (; t + 12 < W.ntiles; t += 16) {
            s0 += src[(int64_t)t * stride];
            s1 += src[(int64_t)(t + 4) * stride];
            s2 += src[(int64_t)(t + 8) * stride];
            s3 += src[(int64_t)(t + 12) * stride];
        }
        for (; t < W.ntiles; t += 4) s0 += src[(int64_t)t * stride];
    }
    acc4[g][lane] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    if (g == 0 && i < tot) a.red[W.red_off + i] = (acc4[0][lane] + acc4[1][lane]) + (acc4[2][lane] + acc4[3][lane]);
}

hipError_t launch_reduce(const ReduceArgs &a, int n_windows, hipStream_t s) {
    if (n_windows <= 0) return hipSuccess;
    dim3 grid((a.max_En + 63) / 64 > 0 ? (a.max_En + 63) / 64 : 1, n_windows), block(256);
    hipLaunchKernelGGL(k_reduce, grid, block, 0, s, a);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------
// Dense FP64 Cholesky of S + lambda I and the two triangular solves for systems too large
// for the register-tile variant below (more than 216 unknowns): one block of 512 threads
// per window, S held as a packed lower triangle in a per-window copy in HBM, which one
// block keeps hot in its XCD's L2 (kHbm; the template also keeps the LDS-resident form).
// Right-looking with 8-column panels.  Per panel every thread reads the 8x8 diagonal
// block and factors it redundantly in registers, so no lane-to-lane traffic sits on the
// serial path; each thread then solves one row of the panel below the block, and after
// one barrier all threads apply the rank-8 update to the trailing triangle in 4x4
// register tiles.  The forward solve L y = r rides along: every thread also solves the
// panel's 8 entries of y redundantly, and the thread of each row below subtracts its
// share.  The backward solve walks the panels from the last, every thread solving the
// panel's 8 entries from prefetched registers, then all threads updating the rows above.
// The right side, the pivots and the factored diagonal blocks stay in LDS.
// ------------------------------------------------------------------------------------
#ifndef LBA_CHOL_NB
#define LBA_CHOL_NB 8
#endif
constexpr int kNB = LBA_CHOL_NB;
constexpr int kCholThreads = 512;

size_t chol_lds_bytes_hbm(int n) { return sizeof(double) * (4 * (size_t)n + (size_t)kNB * n) + 64; }

__device__ __forceinline__ void tri_decode(int e, int &ii, int &jj) {
    int r = (int)((sqrtf(8.0f * (float)e + 1.0f) - 1.0f) * 0.5f);
    while (r * (r + 1) / 2 > e) --r;
    while ((r + 1) * (r + 2) / 2 <= e) ++r;
    ii = r;
    jj = e - r * (r + 1) / 2;
}

// factor the nbk x nbk diagonal block whose top-left entry is (c0, c0) into registers:
// L (lower, row-major kNB x kNB) and its reciprocal diagonal; returns false on a
// non-positive or non-finite pivot
__device__ __forceinline__ bool diag_block_factor(const double *A, int c0, int nbk, double (&L)[kNB][kNB],
                                                  double (&rd)[kNB]) {
    bool ok = true;
#pragma unroll
    for (int i = 0; i < kNB; ++i)
#pragma unroll
        for (int j = 0; j < kNB; ++j) L[i][j] = (i < nbk && j <= i) ? A[packed_lower(c0 + i, c0 + j)] : 0.0;
#pragma unroll
    for (int j = 0; j < kNB; ++j) {
        if (j < nbk) {
            double d = L[j][j];
#pragma unroll
            for (int k = 0; k < j; ++k) d -= L[j][k] * L[j][k];
            if (!(d > 0.0) || !isfinite(d)) ok = false;
            const double r = rsqrt(d);   // one reciprocal square root on the serial path
            L[j][j] = d * r;
            rd[j] = r;
#pragma unroll
            for (int i = j + 1; i < kNB; ++i) {
                double v = L[i][j];
#pragma unroll
                for (int k = 0; k < j; ++k) v -= L[i][k] * L[j][k];
                L[i][j] = v * r;
            }
        } else {
            rd[j] = 0.0;
        }
    }
    return ok;
}

template <bool kHbm>
__global__ __launch_bounds__(kCholThreads) void k_cholesky(CholArgs a) {
    extern __shared__ __align__(16) double cs[];
    __shared__ int s_fail;
    const int w = blockIdx.x;
    const WinInfo W = a.win[w];
    Ctl *ctl = a.ctl + w;
    if (!ctl->running) return;
    const int n = W.n, E = W.E;
    const int tid = threadIdx.x, lane = tid & 63;
    const int nth = blockDim.x;
    const double lambda = ctl->lambda;
    double *A = kHbm ? a.fact + W.red_off : cs;   // E, packed lower
    double *y = kHbm ? cs : cs + E;               // n: right side, then the solution
    double *rr = y + n;      // n: copy of the right side (gain-ratio denominator)
    double *rdiag = rr + n;  // n reciprocal pivots
    double *Ld = rdiag + n;  // n x kNB: factored diagonal blocks (row r holds L[r][c0 .. r])
    double *xs = Ld + (size_t)n * kNB;   // n: the solution of L^T x = y
    const double *red = a.red + W.red_off;
    // eight loads in flight per thread (one at a time, each waited on before its store,
    // took a memory round trip per 512 entries)
    for (int i0 = tid; i0 < E + n; i0 += 8 * nth) {
        double v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * nth;
            v[u] = i < E + n ? red[i] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = i0 + u * nth;
            if (i < E) {
                A[i] = v[u];
            } else if (i < E + n) {
                y[i - E] = v[u];
                rr[i - E] = v[u];
            }
        }
    }
    if (tid == 0) s_fail = a.redflag[w] != 0.0;
    __syncthreads();
    for (int i = tid; i < n; i += nth) A[packed_lower(i, i)] += lambda;
    __syncthreads();

    // ---- factorisation ----------------------------------------------------------------
    for (int c0 = 0; c0 < n; c0 += kNB) {
        const int nbk = min(kNB, n - c0);
        const int b0 = c0 + nbk;
        double L[kNB][kNB], rd[kNB];
        const bool ok = diag_block_factor(A, c0, nbk, L, rd);
        // the panel's entries of y (forward solve), redundantly in every thread
        double yp[kNB];
#pragma unroll
        for (int j = 0; j < kNB; ++j) {
            double v = j < nbk ? y[c0 + j] : 0.0;
#pragma unroll
            for (int k = 0; k < j; ++k) v -= L[j][k] * yp[k];
            yp[j] = v * rd[j];
        }
        if (!ok) {
            if (tid == 0) s_fail = 1;
        } else {
            // panel rows below the diagonal block: L[r][c0+j] = (A[r][c0+j] - sum_k L[r][c0+k] L[c0+j][c0+k]) / L[c0+j][c0+j]
            for (int r = b0 + tid; r < n; r += nth) {
                double x[kNB];
#pragma unroll
                for (int j = 0; j < kNB; ++j) x[j] = j < nbk ? A[packed_lower(r, c0 + j)] : 0.0;
#pragma unroll
                for (int j = 0; j < kNB; ++j) {
                    double v = x[j];
#pragma unroll
                    for (int k = 0; k < j; ++k) v -= x[k] * L[j][k];
                    x[j] = v * rd[j];
                }
                double dy = 0.0;
#pragma unroll
                for (int j = 0; j < kNB; ++j) {
                    if (j < nbk) A[packed_lower(r, c0 + j)] = x[j];
                    dy += x[j] * yp[j];
                }
                y[r] -= dy;   // this thread owns row r of y in this phase
            }
            // the factored diagonal block goes to Ld (A's copy is still being read by
            // other threads in this phase)
            if (tid < nbk * kNB) {
                const int i = tid / kNB, j = tid % kNB;
                double v = 0.0;
#pragma unroll
                for (int ii = 0; ii < kNB; ++ii)
#pragma unroll
                    for (int jj = 0; jj < kNB; ++jj)
                        if (ii == i && jj == j) v = L[ii][jj];
                Ld[(c0 + i) * kNB + j] = v;
            }
            if (tid < nbk) {
                double v = 0.0;
#pragma unroll
                for (int jj = 0; jj < kNB; ++jj)
                    if (jj == tid) v = rd[jj];
                rdiag[c0 + tid] = v;
            }
        }
        __syncthreads();
        if (s_fail) break;
        // the panel's solved entries of y (every thread has read the unsolved ones)
        if (tid < nbk) {
            double v = 0.0;
#pragma unroll
            for (int jj = 0; jj < kNB; ++jj)
                if (jj == tid) v = yp[jj];
            y[c0 + tid] = v;
        }
        // trailing update A[i][j] -= sum_kk L[i][c0+kk] L[j][c0+kk], b0 <= j <= i < n
        const int m = n - b0;
        const int T4 = (m + 3) / 4;
        const int ntile = T4 * (T4 + 1) / 2;
        for (int t = tid; t < ntile; t += nth) {
            int I, J;
            tri_decode(t, I, J);
            const int i0 = b0 + 4 * I, j0 = b0 + 4 * J;
            double ai[4][kNB], aj[4][kNB];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int ri = i0 + u, rj = j0 + u;
#pragma unroll
                for (int kk = 0; kk < kNB; ++kk) {
                    ai[u][kk] = (ri < n && kk < nbk) ? A[packed_lower(ri, c0 + kk)] : 0.0;
                    aj[u][kk] = (rj < n && kk < nbk) ? A[packed_lower(rj, c0 + kk)] : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int i = i0 + u, j = j0 + v;
                    if (i < n && j <= i) {
                        double acc = 0.0;
#pragma unroll
                        for (int kk = 0; kk < kNB; ++kk) acc += ai[u][kk] * aj[v][kk];
                        A[packed_lower(i, j)] -= acc;
                    }
                }
            }
        }
        __syncthreads();
    }
    const int ok = !s_fail;

    // ---- L^T x = y (y was solved with the factorisation; one barrier per panel) ------
    // Each panel's entries of x go to their own array, so the threads still reading the
    // panel's y are not overtaken by its solution; the rows above are updated in the same
    // step.
    if (ok) {
        const int last = n > 0 ? ((n - 1) / kNB) * kNB : 0;
        for (int c0 = last; c0 >= 0 && n > 0; c0 -= kNB) {
            const int nbk = min(kNB, n - c0);
            // the panel's diagonal block and right side, all loads issued before the chain
            double Lb[kNB][kNB], yb[kNB], rb[kNB], xp[kNB];
#pragma unroll
            for (int k = 0; k < kNB; ++k) {
                yb[k] = k < nbk ? y[c0 + k] : 0.0;
                rb[k] = k < nbk ? rdiag[c0 + k] : 0.0;
#pragma unroll
                for (int j = 0; j < k; ++j) Lb[k][j] = k < nbk ? Ld[(c0 + k) * kNB + j] : 0.0;
            }
#pragma unroll
            for (int j = kNB - 1; j >= 0; --j) {
                double v = yb[j];
#pragma unroll
                for (int k = j + 1; k < kNB; ++k) v -= Lb[k][j] * xp[k];
                xp[j] = v * rb[j];
            }
            if (tid < nbk) {
                double v = 0.0;
#pragma unroll
                for (int j = 0; j < kNB; ++j)
                    if (j == tid) v = xp[j];
                xs[c0 + tid] = v;
            }
            for (int j = tid; j < c0; j += nth) {
                double acc = 0.0;
#pragma unroll
                for (int kk = 0; kk < kNB; ++kk)
                    if (kk < nbk) acc += A[packed_lower(c0 + kk, j)] * xp[kk];
                y[j] -= acc;
            }
            __syncthreads();
        }
    }
    double *dp = a.dp + W.dp_off;
    if (tid < 64) {
        double den = 0.0;
        for (int i = lane; i < n; i += 64) {
            const double x = ok ? xs[i] : 0.0;
            dp[i] = x;
            den += x * (lambda * x + rr[i]);   // + point part in the update kernel
        }
        den = wave_sum(den);
        if (lane == 0) {
            ctl->solve_ok = ok;
            ctl->denom_p = den;
        }
    }
}


// ------------------------------------------------------------------------------------
// The same factorisation and solves for systems of up to 216 unknowns with the matrix in
// registers: S + lambda I is cut into 4 x 4 tiles of its lower triangle, and thread t
// owns tiles t, t + 512 and t + 1024 (packed row-major tile order) for the whole solve,
// so the trailing updates read only the panel from LDS and write nothing there.  Per
// panel of four columns:
//   1. the owner of the diagonal tile factors it (and solves the panel's entries of y),
//      and publishes the factor;
//   2. the owners of the tiles below it solve them against the factor (their rows of the
//      panel, published to LDS) and subtract their share of y;
//   3. every owner of a trailing tile subtracts the product of its two panel rows.
// The panel and the factor are double-buffered, so two barriers per panel suffice.  The
// back solve L^T x = y walks the panels from the last: the diagonal owner solves the
// panel's x, then the owners of the tiles left of the diagonal subtract their share from
// y.  Every sum is taken in a fixed order, so solves repeat bit for bit.  Rows past n are
// an identity block with a zero right side.
// ------------------------------------------------------------------------------------
constexpr int kRegMaxN = 216;                  // 54 tile rows, 1,485 tiles <= 3 x 512
constexpr int kRegThreads = 512;
constexpr int kRegSlots = 3;

int chol_reg_max_n() { return kRegMaxN; }

__global__ __launch_bounds__(kRegThreads) void k_chol_reg(CholArgs a) {
    __shared__ double P[2][kRegMaxN][4];   // panel rows: L[r][4k .. 4k + 3]
    __shared__ double Lk[2][16];           // factored diagonal tile (row-major 4 x 4)
    __shared__ double Rk[2][4];            // its reciprocal pivots
    __shared__ double y[kRegMaxN], xs[kRegMaxN], rr[kRegMaxN], rdg[kRegMaxN];
    __shared__ int s_fail;
    const int w = blockIdx.x;
    const WinInfo W = a.win[w];
    Ctl *ctl = a.ctl + w;
    if (!ctl->running) return;
    const int n = W.n, E = W.E;
    const int tid = threadIdx.x, lane = tid & 63;
    const double lambda = ctl->lambda;
    const double *red = a.red + W.red_off;
    const int NT = (n + 3) / 4, N4 = 4 * NT;
    const int ntiles = NT * (NT + 1) / 2;
    if (tid == 0) s_fail = (a.redflag[w] != 0.0) || n > kRegMaxN;
    // right side (padded with zeros)
    for (int i = tid; i < N4; i += kRegThreads) {
        const double v = i < n ? red[E + i] : 0.0;
        y[i] = v;
        rr[i] = v;
    }
    // own tiles: loads issued for all three before any is used
    int tI[kRegSlots], tJ[kRegSlots];
    double T[kRegSlots][4][4];
#pragma unroll
    for (int u = 0; u < kRegSlots; ++u) {
        const int t = tid + kRegThreads * u;
        int I = -1, J = -1;
        if (t < ntiles) tri_decode(t, I, J);
        tI[u] = I;
        tJ[u] = J;
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int i = 4 * I + r, j = 4 * J + c;
                double v = 0.0;
                if (I >= 0 && i < n && j <= i) v = red[packed_lower(i, j)] + (i == j ? lambda : 0.0);
                else if (I >= 0 && i == j) v = 1.0;   // padding rows: identity
                T[u][r][c] = v;
            }
    }
    __syncthreads();
    // (s_fail is read only right after a barrier that follows its last write: a thread
    // that read it while another sets it would leave the panel loop alone)
    const bool failed_before = s_fail != 0;

    // ---- factorisation and forward solve ----------------------------------------------
    for (int k = 0; k < NT && !failed_before; ++k) {
        const int b = k & 1;
        // 1. the diagonal tile
#pragma unroll
        for (int u = 0; u < kRegSlots; ++u) {
            if (tI[u] != k || tJ[u] != k) continue;
            double rd[4];
            bool ok = true;
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double d = T[u][c][c];
#pragma unroll
                for (int m = 0; m < c; ++m) d -= T[u][c][m] * T[u][c][m];
                if (!(d > 0.0) || !isfinite(d)) ok = false;
                const double r = rsqrt(d);
                T[u][c][c] = d * r;
                rd[c] = r;
#pragma unroll
                for (int q = c + 1; q < 4; ++q) {
                    double v = T[u][q][c];
#pragma unroll
                    for (int m = 0; m < c; ++m) v -= T[u][q][m] * T[u][c][m];
                    T[u][q][c] = v * r;
                }
            }
            double yk[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                double v = y[4 * k + c];
#pragma unroll
                for (int m = 0; m < c; ++m) v -= T[u][c][m] * yk[m];
                yk[c] = v * rd[c];
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
#pragma unroll
                for (int c = 0; c < 4; ++c) Lk[b][4 * r + c] = c <= r ? T[u][r][c] : 0.0;
                Rk[b][r] = rd[r];
                rdg[4 * k + r] = rd[r];
                y[4 * k + r] = yk[r];
            }
            if (!ok) s_fail = 1;
        }
        __syncthreads();
        if (s_fail) break;
        // 2. the tiles below the diagonal tile: L_Ik = A_Ik L_kk^-T
        double lk[16], rk[4], yk[4];
#pragma unroll
        for (int q = 0; q < 16; ++q) lk[q] = Lk[b][q];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            rk[c] = Rk[b][c];
            yk[c] = y[4 * k + c];
        }
#pragma unroll
        for (int u = 0; u < kRegSlots; ++u) {
            if (tJ[u] != k || tI[u] <= k) continue;
            const int I = tI[u];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                double dy = 0.0;
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    double v = T[u][r][c];
#pragma unroll
                    for (int m = 0; m < c; ++m) v -= T[u][r][m] * lk[4 * c + m];
                    T[u][r][c] = v * rk[c];
                    P[b][4 * I + r][c] = T[u][r][c];
                    dy += T[u][r][c] * yk[c];
                }
                y[4 * I + r] -= dy;   // the only writer of these rows in this panel
            }
        }
        __syncthreads();
        // 3. trailing tiles (J > k): A_IJ -= L_Ik L_Jk^T
#pragma unroll
        for (int u = 0; u < kRegSlots; ++u) {
            if (tJ[u] <= k) continue;
            const int I = tI[u], J = tJ[u];
            double pi[4][4], pj[4][4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c) {
                    pi[r][c] = P[b][4 * I + r][c];
                    pj[r][c] = P[b][4 * J + r][c];
                }
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    T[u][r][c] -= pi[r][0] * pj[c][0] + pi[r][1] * pj[c][1] + pi[r][2] * pj[c][2] + pi[r][3] * pj[c][3];
        }
    }
    __syncthreads();
    const int ok = !s_fail;

    // ---- back solve L^T x = y, two barriers per panel -----------------------------------
    if (ok) {
        for (int k = NT - 1; k >= 0; --k) {
#pragma unroll
            for (int u = 0; u < kRegSlots; ++u) {
                if (tI[u] != k || tJ[u] != k) continue;
                double xk[4];
#pragma unroll
                for (int c = 3; c >= 0; --c) {
                    double v = y[4 * k + c];
#pragma unroll
                    for (int m = c + 1; m < 4; ++m) v -= T[u][m][c] * xk[m];
                    xk[c] = v * rdg[4 * k + c];
                }
#pragma unroll
                for (int c = 0; c < 4; ++c) xs[4 * k + c] = xk[c];
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kRegSlots; ++u) {
                if (tI[u] != k || tJ[u] >= k) continue;
                const int J = tJ[u];
                double xk[4];
#pragma unroll
                for (int r = 0; r < 4; ++r) xk[r] = xs[4 * k + r];
#pragma unroll
                for (int c = 0; c < 4; ++c)
                    y[4 * J + c] -= T[u][0][c] * xk[0] + T[u][1][c] * xk[1] + T[u][2][c] * xk[2] + T[u][3][c] * xk[3];
            }
            __syncthreads();
        }
    }
    double *dp = a.dp + W.dp_off;
    if (tid < 64) {
        double den = 0.0;
        for (int i = lane; i < n; i += 64) {
            const double x = ok ? xs[i] : 0.0;
            dp[i] = x;
            den += x * (lambda * x + rr[i]);   // + point part in the update kernel
        }
        den = wave_sum(den);
        if (lane == 0) {
            ctl->solve_ok = ok;
            ctl->denom_p = den;
        }
    }
}

size_t chol_static_lds() { return kernel_static_lds((const void *)k_cholesky<true>); }

hipError_t launch_cholesky(const CholArgs &a, int n_windows, size_t lds, hipStream_t s) {
    if (n_windows <= 0) return hipSuccess;
    if (a.fact) hipLaunchKernelGGL(k_cholesky<true>, dim3(n_windows), dim3(kCholThreads), lds, s, a);
    else hipLaunchKernelGGL(k_chol_reg, dim3(n_windows), dim3(kRegThreads), 0, s, a);
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
    double Ft = 0.0, den = 0.0, fl = 0.0;
    const int64_t u0 = (int64_t)W.tile0 * a.split;   // the update's parts of this window's tiles
    for (int t = lane; t < W.ntiles * a.split; t += 64) {
        Ft += a.partu[4 * (u0 + t)];
        den += a.partu[4 * (u0 + t) + 1];
        fl = fmax(fl, a.partu[4 * (u0 + t) + 2]);
    }
    if (a.vi_ed)   // the inertial measurements' costs at the trial state
        for (int e = a.vi_edge_off[w] + lane; e < a.vi_edge_off[w + 1]; e += 64) Ft += a.vi_ed[(int64_t)e * kViEdgeStride + 1];
    Ft = wave_sum(Ft);
    den = wave_sum(den) + ctl->denom_p;
    fl = wave_max(fl);
    if (lane == 0) {
        const int ok = ctl->solve_ok && fl == 0.0;
        const double gain = (ctl->F - Ft) / den;
        const int acc = ok && isfinite(Ft) && isfinite(gain) && gain > 0.0;
        if (a.log && ctl->trials_total < a.log_cap) {
            TrialRec &L = a.log[(int64_t)w * a.log_cap + ctl->trials_total];
            L.round = a.round;
            L.iter = ctl->iter;
            L.trial = ctl->trial;
            L.accepted = acc;
            L.solve_ok = ok;
            L.pad = 0;
            L.lambda = ctl->lambda;
            L.F = ctl->F;
            L.F_trial = Ft;
            L.gain = gain;
        }
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
            if (a.vi_state) {   // velocity and biases move additively
                const double *d = a.vi_dp + a.vi_win[w].dp_off + 15 * ok + 6;
                double *st = a.vi_state + 9 * (int64_t)(W.kf0 + k);
#pragma unroll
                for (int q = 0; q < 9; ++q) st[q] += d[q];
            }
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
constexpr int kInitCols = 384;   // columns of one window's r (n = 6 Kopt <= 360), six per lane
constexpr int kInitRedThreads = 1024;
constexpr int kInitRedWaves = kInitRedThreads / 64;

__global__ __launch_bounds__(kInitRedThreads) void k_init_reduce(InitReduceArgs a) {
    __shared__ double smax[kInitRedWaves];
    __shared__ double colsum[kInitRedWaves][kInitCols];
    const int w = blockIdx.x;
    const WinInfo W = a.win[w];
    Ctl *ctl = a.ctl + w;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    // largest diagonal entry of Hpp (per camera, summed over the tiles): wavefront g sums
    // the tiles g, g + G, ... (G wavefronts, four tiles per step), lane l the columns l,
    // l + 64, ... (coalesced rows) ...
    constexpr int G = kInitRedWaves;
    double cs[kInitCols / 64] = {};
    const double *pr = a.partr + W.partr_off;
    for (int t0 = wave; t0 < W.ntiles; t0 += 4 * G) {
#pragma unroll
        for (int c = 0; c < kInitCols / 64; ++c) {
            const int col = lane + 64 * c;
            double v = 0.0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int t = t0 + u * G;
                if (col < W.n && t < W.ntiles) v += pr[(int64_t)t * W.n + col];
            }
            cs[c] += v;
        }
    }
#pragma unroll
    for (int c = 0; c < kInitCols / 64; ++c) colsum[wave][lane + 64 * c] = cs[c];
    __syncthreads();
    double md = 0.0;
    if (!a.vi_ed) {
        for (int i = tid; i < W.n; i += blockDim.x) {
            double v = 0.0;
            for (int g = 0; g < G; ++g) v += colsum[g][i];
            md = fmax(md, v);
        }
    } else {
        // the joint diagonal: visual pose entries plus every inertial measurement's
        // diagonal on the 15 unknowns of its two keyframes
        const int e0 = a.vi_edge_off[w], e1 = a.vi_edge_off[w + 1];
        for (int i = tid; i < 15 * W.Kopt; i += blockDim.x) {
            const int o = i / 15, c = i % 15;
            double v = 0.0;
            if (c < 6)
                for (int g = 0; g < G; ++g) v += colsum[g][6 * o + c];
            for (int e = e0; e < e1; ++e) {
                const double *rec = a.vi_ed + (int64_t)e * kViEdgeStride + kViH;
                if (a.opt_map[W.kf0 + a.vi_ei[e]] == o) v += rec[c * (c + 1) / 2 + c];
                if (a.opt_map[W.kf0 + a.vi_ej[e]] == o) v += rec[(15 + c) * (16 + c) / 2 + 15 + c];
            }
            md = fmax(md, v);
        }
    }
    // ... and of the point blocks (per tile), and the cost
    double F = 0.0;
    for (int t = tid; t < W.ntiles; t += blockDim.x) md = fmax(md, a.partd[4 * (W.tile0 + t) + 1]);
    if (wave == 0) {
        for (int t = lane; t < W.ntiles; t += 64) F += a.partd[4 * (W.tile0 + t)];
        if (a.vi_ed)
            for (int e = a.vi_edge_off[w] + lane; e < a.vi_edge_off[w + 1]; e += 64)
                F += a.vi_ed[(int64_t)e * kViEdgeStride];
    }
    md = wave_max(md);
    F = wave_sum(F);
    if (lane == 0) smax[wave] = md;
    __syncthreads();
    if (tid == 0) {
        md = 0.0;
        for (int g = 0; g < kInitRedWaves; ++g) md = fmax(md, smax[g]);
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

static_assert(6 * kMaxKoptFP64 <= kInitCols && 6 * kMaxKoptMixed <= kInitCols, "columns per lane");

hipError_t launch_init_reduce(const InitReduceArgs &a, int n_windows, hipStream_t s) {
    if (n_windows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_init_reduce, dim3(n_windows), dim3(kInitRedThreads), 0, s, a);
    return hipGetLastError();
}

}  // namespace lba
