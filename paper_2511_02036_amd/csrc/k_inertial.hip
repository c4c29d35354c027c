// Inertial measurements of the stereo-inertial solve (Section III-C: the local bundle
// adjustment of a visual-inertial system adds inertial residuals to the reprojection
// errors).  Reading: the preintegrated IMU factor of Forster, Carlone, Dellaert and
// Scaramuzza (IEEE T-RO 2017) between keyframes, plus a bias random walk; 15 unknowns per
// optimisable keyframe (camera twist, velocity, gyroscope and accelerometer biases).
//
// Kernels, all FP64:
//   k_vi_eval    one block per measurement: residual, cost and (when linearising) the
//                Jacobian with respect to both keyframes' 15 unknowns, then its Gauss-
//                Newton blocks J^T Info J (packed lower 30 x 30) and -J^T Info r, written
//                to the measurement's record; in trial mode only the cost at the trial
//                state (pose Exp(dp) T, velocity and biases plus the step);
//   k_vi_system  one block per window: the joint reduced system of 15 Kopt unknowns, the
//                visual reduced system in the pose rows and columns plus every measurement
//                of the window added in measurement order (a fixed order: results do not
//                depend on scheduling);
//   k_vi_split   the pose part of the joint step in the visual step's layout, for the
//                back-substitution and the trial poses;
//   k_vi_setup / k_vi_finish / k_vi_check   state copies and input validation.
// The damping decision adds the measurements' trial costs and applies the velocity and
// bias steps (k_decide); the round's first damping includes their diagonal
// (k_init_reduce).
#include "lba_internal.h"

namespace lba {

// ---- 3x3 helpers, row-major -------------------------------------------------------------
__device__ __forceinline__ void mm3(const double *A, const double *B, double *C) {   // C = A B
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) C[i * 3 + j] = A[i * 3] * B[j] + A[i * 3 + 1] * B[3 + j] + A[i * 3 + 2] * B[6 + j];
}
__device__ __forceinline__ void mtm3(const double *A, const double *B, double *C) {  // C = A^T B
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) C[i * 3 + j] = A[i] * B[j] + A[3 + i] * B[3 + j] + A[6 + i] * B[6 + j];
}
__device__ __forceinline__ void mv3(const double *A, const double *x, double *y) {   // y = A x
#pragma unroll
    for (int i = 0; i < 3; ++i) y[i] = A[i * 3] * x[0] + A[i * 3 + 1] * x[1] + A[i * 3 + 2] * x[2];
}
__device__ __forceinline__ void mtv3(const double *A, const double *x, double *y) {  // y = A^T x
#pragma unroll
    for (int i = 0; i < 3; ++i) y[i] = A[i] * x[0] + A[3 + i] * x[1] + A[6 + i] * x[2];
}
__device__ __forceinline__ void skew3(const double *w, double *W) {
    W[0] = 0.0;   W[1] = -w[2]; W[2] = w[1];
    W[3] = w[2];  W[4] = 0.0;   W[5] = -w[0];
    W[6] = -w[1]; W[7] = w[0];  W[8] = 0.0;
}

// SO(3) exponential through the SE(3) one (zero translation)
__device__ __forceinline__ void rot_exp(const double *w, double *R) {
    const double xi[6] = {w[0], w[1], w[2], 0.0, 0.0, 0.0};
    double t[3];
    se3_exp(xi, R, t);
}

// SO(3) logarithm: angle atan2(|sin|, cos) from the antisymmetric and trace parts; near pi
// the axis is the dominant column of the symmetric part (1 - cos t) a a^T
__device__ void rot_log(const double *R, double *w) {
    const double ax = 0.5 * (R[7] - R[5]), ay = 0.5 * (R[2] - R[6]), az = 0.5 * (R[3] - R[1]);
    const double s = sqrt(ax * ax + ay * ay + az * az);
    const double c = 0.5 * (R[0] + R[4] + R[8] - 1.0);
    const double th = atan2(s, c);
    if (th < 1e-4) {
        const double f = 1.0 + th * th * (1.0 / 6.0);
        w[0] = f * ax; w[1] = f * ay; w[2] = f * az;
        return;
    }
    if (M_PI - th > 1e-4) {
        const double f = th / s;
        w[0] = f * ax; w[1] = f * ay; w[2] = f * az;
        return;
    }
    double S[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) S[i * 3 + j] = 0.5 * (R[i * 3 + j] + R[j * 3 + i]) - (i == j ? c : 0.0);
    int k = 0;
    if (S[4] > S[k * 4]) k = 1;
    if (S[8] > S[k * 4]) k = 2;
    const double v0 = S[k], v1 = S[3 + k], v2 = S[6 + k];
    const double nv = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
    const double sg = (v0 * ax + v1 * ay + v2 * az) < 0.0 ? -1.0 : 1.0;
    w[0] = sg * th * v0 / nv; w[1] = sg * th * v1 / nv; w[2] = sg * th * v2 / nv;
}

// right Jacobian Jr(w) = I - B W + C W^2 and its inverse I + W / 2 + D W^2,
// B = (1 - cos t) / t^2, C = (t - sin t) / t^3, D = 1 / t^2 - (1 + cos t) / (2 t sin t)
__device__ void rot_jr(const double *w, double *J, bool inverse) {
    const double th2 = w[0] * w[0] + w[1] * w[1] + w[2] * w[2];
    const double th = sqrt(th2);
    double W[9], W2[9];
    skew3(w, W);
    mm3(W, W, W2);
    double a, b;
    if (inverse) {
        a = 0.5;
        b = th < 1e-2 ? 1.0 / 12.0 + th2 * (1.0 / 720.0) + th2 * th2 * (1.0 / 30240.0)
                      : 1.0 / th2 - (1.0 + cos(th)) / (2.0 * th * sin(th));
    } else {
        if (th < 1e-2) {
            a = -(0.5 - th2 * (1.0 / 24.0) + th2 * th2 * (1.0 / 720.0));
            b = 1.0 / 6.0 - th2 * (1.0 / 120.0) + th2 * th2 * (1.0 / 5040.0);
        } else {
            const double h = sin(0.5 * th);
            a = -2.0 * h * h / th2;
            b = (th - sin(th)) / (th2 * th);
        }
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) J[i] = (i % 4 == 0 ? 1.0 : 0.0) + a * W[i] + b * W2[i];
}

// body rotation R_cw^T R_cb and position R_cw^T (t_cb - t_cw) of a camera pose
__device__ __forceinline__ void body_of(const double *T, const double *Tcb, double *Rb, double *pb) {
    double Rc[9], Rcb[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Rc[i * 3 + j] = T[i * 4 + j];
            Rcb[i * 3 + j] = Tcb[i * 4 + j];
        }
    mtm3(Rc, Rcb, Rb);
    const double d[3] = {Tcb[3] - T[3], Tcb[7] - T[7], Tcb[11] - T[11]};
    mtv3(Rc, d, pb);
}

// Residual (and Jacobian when J is not null: 15 x 30, columns (w, u, v, bg, ba) of
// keyframe i then of keyframe j) of measurement e for poses Ti, Tj and states si, sj
// (v, bg, ba each).  The left camera twist (w, u) turns the body rotation by -R_cb^T w on
// the right and moves the body position by R_cw^T ([t_cb]x w - u).
__device__ void vi_residual_jacobian(const ViArgs &a, int e, const double *Ti, const double *Tj, const double *si,
                                     const double *sj, double *r, double (*J)[30]) {
    const ViEdges &E = a.E;
    const double dt = E.dt[e];
    double Ri[9], Rj[9], pi[3], pj[3];
    body_of(Ti, a.Tcb, Ri, pi);
    body_of(Tj, a.Tcb, Rj, pj);
    double dbg[3], dba[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        dbg[q] = si[3 + q] - E.bgb[3 * e + q];
        dba[q] = si[6 + q] - E.bab[3 * e + q];
    }
    const double *JRg = E.JRg + 9 * e;
    double phi[3], Eb[9], dRc[9], RiRj[9], Em[9];
    mv3(JRg, dbg, phi);
    rot_exp(phi, Eb);
    mm3(E.dR + 9 * e, Eb, dRc);
    mtm3(Ri, Rj, RiRj);
    mtm3(dRc, RiRj, Em);
    rot_log(Em, r);
    double u[3], wv[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        u[q] = sj[q] - si[q] - a.g[q] * dt;
        wv[q] = pj[q] - pi[q] - si[q] * dt - 0.5 * a.g[q] * dt * dt;
    }
    double Ru[3], Rw[3], t1[3], t2[3], t3[3], t4[3];
    mtv3(Ri, u, Ru);
    mtv3(Ri, wv, Rw);
    mv3(E.Jvg + 9 * e, dbg, t1);
    mv3(E.Jva + 9 * e, dba, t2);
    mv3(E.Jpg + 9 * e, dbg, t3);
    mv3(E.Jpa + 9 * e, dba, t4);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        r[3 + q] = Ru[q] - (E.dv[3 * e + q] + t1[q] + t2[q]);
        r[6 + q] = Rw[q] - (E.dp[3 * e + q] + t3[q] + t4[q]);
        r[9 + q] = sj[3 + q] - si[3 + q];
        r[12 + q] = sj[6 + q] - si[6 + q];
    }
    if (!J) return;
    for (int m = 0; m < 15; ++m)
        for (int c = 0; c < 30; ++c) J[m][c] = 0.0;
    auto put = [&](int row, int col, const double *M, double scale) {
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) J[row + i][col + j] = scale * M[i * 3 + j];
    };
    // twist maps of both keyframes: rotation -R_cb^T, position R_cw^T [t_cb]x and -R_cw^T
    double A[9], Pw[2][9], Pu[2][9];
    {
        double Rcb[9], tx[9];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                Rcb[i * 3 + j] = a.Tcb[i * 4 + j];
                A[j * 3 + i] = -a.Tcb[i * 4 + j];
            }
        const double tcb[3] = {a.Tcb[3], a.Tcb[7], a.Tcb[11]};
        skew3(tcb, tx);
        for (int side = 0; side < 2; ++side) {
            const double *T = side ? Tj : Ti;
            double Rc[9];
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) Rc[i * 3 + j] = T[i * 4 + j];
            mtm3(Rc, tx, Pw[side]);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) Pu[side][i * 3 + j] = -Rc[j * 3 + i];
        }
        (void)Rcb;
    }
    double RiT[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) RiT[i * 3 + j] = Ri[j * 3 + i];
    // rotation rows
    double Jri[9], RjRi[9], M[9], M2[9];
    rot_jr(r, Jri, true);
    mtm3(Rj, Ri, RjRi);
    mm3(Jri, RjRi, M);          // d r_R / d th_i = -M
    mm3(M, A, M2);
    put(0, 0, M2, -1.0);
    mm3(Jri, A, M2);            // d r_R / d th_j = Jri
    put(0, 15, M2, 1.0);
    {
        double Jr[9], EJ[9], T1[9], T2[9];
        rot_jr(phi, Jr, false);
        mtm3(Em, Jr, EJ);      // E^T Jr
        mm3(Jri, EJ, T1);
        mm3(T1, JRg, T2);
        put(0, 9, T2, -1.0);
    }
    // velocity rows
    double H[9];
    skew3(Ru, H);
    mm3(H, A, M2);
    put(3, 0, M2, 1.0);
    put(3, 6, RiT, -1.0);
    put(3, 21, RiT, 1.0);
    put(3, 9, E.Jvg + 9 * e, -1.0);
    put(3, 12, E.Jva + 9 * e, -1.0);
    // position rows: rotation and position of i, position of j, velocity of i, biases
    skew3(Rw, H);
    mm3(H, A, M);
    mm3(RiT, Pw[0], M2);
    for (int q = 0; q < 9; ++q) M[q] -= M2[q];
    put(6, 0, M, 1.0);
    mm3(RiT, Pu[0], M2);
    put(6, 3, M2, -1.0);
    mm3(RiT, Pw[1], M2);
    put(6, 15, M2, 1.0);
    mm3(RiT, Pu[1], M2);
    put(6, 18, M2, 1.0);
    put(6, 6, RiT, -dt);
    put(6, 9, E.Jpg + 9 * e, -1.0);
    put(6, 12, E.Jpa + 9 * e, -1.0);
    // bias random walks
    for (int q = 0; q < 3; ++q) {
        J[9 + q][9 + q] = -1.0;
        J[9 + q][24 + q] = 1.0;
        J[12 + q][12 + q] = -1.0;
        J[12 + q][27 + q] = 1.0;
    }
}

// ---- per measurement ---------------------------------------------------------------------
__global__ __launch_bounds__(64) void k_vi_eval(ViArgs a) {
    __shared__ double J[15][30], OJ[15][30], r[15], Or[15];
    const int e = blockIdx.x, lane = threadIdx.x;
    const int w = a.edge_win[e];
    if (a.trial && !a.ctl[w].running) return;
    const WinInfo W = a.win[w];
    const int ki = W.kf0 + a.E.ei[e], kj = W.kf0 + a.E.ej[e];
    const int oi = a.opt_map[ki], oj = a.opt_map[kj];
    const ViEdges &E = a.E;
    if (lane == 0) {
        double Ti[12], Tj[12], si[9], sj[9];
        for (int q = 0; q < 9; ++q) {
            si[q] = a.state[9 * (int64_t)ki + q];
            sj[q] = a.state[9 * (int64_t)kj + q];
        }
        if (a.trial) {
            const WinInfo V = a.vwin[w];
            if (oi >= 0) {
                se3_left_update(a.dp + W.dp_off + 6 * oi, a.T + 12 * (int64_t)ki, Ti);
                for (int q = 0; q < 9; ++q) si[q] += a.vdp[V.dp_off + 15 * oi + 6 + q];
            } else {
                for (int q = 0; q < 12; ++q) Ti[q] = a.T[12 * (int64_t)ki + q];
            }
            if (oj >= 0) {
                se3_left_update(a.dp + W.dp_off + 6 * oj, a.T + 12 * (int64_t)kj, Tj);
                for (int q = 0; q < 9; ++q) sj[q] += a.vdp[V.dp_off + 15 * oj + 6 + q];
            } else {
                for (int q = 0; q < 12; ++q) Tj[q] = a.T[12 * (int64_t)kj + q];
            }
            vi_residual_jacobian(a, e, Ti, Tj, si, sj, r, nullptr);
        } else {
            for (int q = 0; q < 12; ++q) {
                Ti[q] = a.T[12 * (int64_t)ki + q];
                Tj[q] = a.T[12 * (int64_t)kj + q];
            }
            vi_residual_jacobian(a, e, Ti, Tj, si, sj, r, J);
        }
    }
    __syncthreads();
    // Info r and Info J: the 9 x 9 block, then the two bias blocks (multiples of I)
    const double *inf = E.info + 81 * (int64_t)e;
    const double ibg = E.ibg[e], iba = E.iba[e];
    if (lane < 15) {
        double v;
        if (lane < 9) {
            v = 0.0;
            for (int k = 0; k < 9; ++k) v += inf[lane * 9 + k] * r[k];
        } else {
            v = (lane < 12 ? ibg : iba) * r[lane];
        }
        Or[lane] = v;
    }
    if (!a.trial && lane < 30) {
        for (int m = 0; m < 15; ++m) {
            double v;
            if (m < 9) {
                v = 0.0;
                for (int k = 0; k < 9; ++k) v += inf[m * 9 + k] * J[k][lane];
            } else {
                v = (m < 12 ? ibg : iba) * J[m][lane];
            }
            OJ[m][lane] = v;
        }
    }
    __syncthreads();
    double *rec = a.ed + (int64_t)e * kViEdgeStride;
    if (lane == 0) {
        double c = 0.0;
        for (int m = 0; m < 15; ++m) c += r[m] * Or[m];
        rec[a.trial ? 1 : 0] = c;
    }
    if (a.trial) return;
    const bool si_opt = oi >= 0, sj_opt = oj >= 0;
    if (lane < 30) {
        double g = 0.0;
        for (int m = 0; m < 15; ++m) g += J[m][lane] * Or[m];
        rec[kViB + lane] = -g;
    }
    for (int idx = lane; idx < 465; idx += 64) {
        int row = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
        while (row * (row + 1) / 2 > idx) --row;
        while ((row + 1) * (row + 2) / 2 <= idx) ++row;
        const int col = idx - row * (row + 1) / 2;
        const bool need = (row < 15 ? si_opt : sj_opt) && (col < 15 ? si_opt : sj_opt);
        double h = 0.0;
        if (need)
            for (int m = 0; m < 15; ++m) h += J[m][row] * OJ[m][col];
        rec[kViH + idx] = h;
    }
}

// ---- per window: the joint reduced system ---------------------------------------------------
__global__ __launch_bounds__(256) void k_vi_system(ViArgs a) {
    const int w = blockIdx.x, tid = threadIdx.x;
    if (!a.ctl[w].running) return;
    const WinInfo W = a.win[w], V = a.vwin[w];
    double *S = a.vred + V.red_off;
    const double *Sv = a.red + W.red_off;
    const int n = V.n, E = V.E;
    for (int idx = tid; idx < E + n; idx += 256) {
        double v = 0.0;
        if (idx < E) {
            int row = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
            while (row * (row + 1) / 2 > idx) --row;
            while ((row + 1) * (row + 2) / 2 <= idx) ++row;
            const int col = idx - row * (row + 1) / 2;
            if (row % 15 < 6 && col % 15 < 6)
                v = Sv[packed_lower(6 * (row / 15) + row % 15, 6 * (col / 15) + col % 15)];
        } else {
            const int i = idx - E;
            if (i % 15 < 6) v = Sv[W.E + 6 * (i / 15) + i % 15];
        }
        S[idx] = v;
    }
    __syncthreads();
    for (int e = a.edge_off[w]; e < a.edge_off[w + 1]; ++e) {
        const int oi = a.opt_map[W.kf0 + a.E.ei[e]], oj = a.opt_map[W.kf0 + a.E.ej[e]];
        const double *rec = a.ed + (int64_t)e * kViEdgeStride;
        for (int idx = tid; idx < 465; idx += 256) {
            int la = (int)((sqrt(8.0 * idx + 1.0) - 1.0) * 0.5);
            while (la * (la + 1) / 2 > idx) --la;
            while ((la + 1) * (la + 2) / 2 <= idx) ++la;
            const int lc = idx - la * (la + 1) / 2;
            const int oa = la < 15 ? oi : oj, oc = lc < 15 ? oi : oj;
            if (oa < 0 || oc < 0) continue;
            const int ga = 15 * oa + la % 15, gc = 15 * oc + lc % 15;
            S[ga >= gc ? packed_lower(ga, gc) : packed_lower(gc, ga)] += rec[kViH + idx];
        }
        if (tid < 30) {
            const int o = tid < 15 ? oi : oj;
            if (o >= 0) S[E + 15 * o + tid % 15] += rec[kViB + tid];
        }
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void k_vi_split(ViArgs a) {
    const int w = blockIdx.x;
    if (!a.ctl[w].running) return;
    const WinInfo W = a.win[w], V = a.vwin[w];
    for (int i = threadIdx.x; i < V.n; i += 64)
        if (i % 15 < 6) a.dpv[W.dp_off + 6 * (i / 15) + i % 15] = a.vdp[V.dp_off + i];
}

__global__ __launch_bounds__(256) void k_vi_setup(ViArgs a) {
    for (int k = blockIdx.x * 256 + threadIdx.x; k < a.n_kf; k += gridDim.x * 256)
        for (int q = 0; q < 3; ++q) {
            a.state[9 * (int64_t)k + q] = a.v0[3 * (int64_t)k + q];
            a.state[9 * (int64_t)k + 3 + q] = a.bg0[3 * (int64_t)k + q];
            a.state[9 * (int64_t)k + 6 + q] = a.ba0[3 * (int64_t)k + q];
        }
}

__global__ __launch_bounds__(256) void k_vi_finish(ViArgs a) {
    for (int k = blockIdx.x * 256 + threadIdx.x; k < a.n_kf; k += gridDim.x * 256)
        for (int q = 0; q < 3; ++q) {
            a.v_out[3 * (int64_t)k + q] = a.state[9 * (int64_t)k + q];
            a.bg_out[3 * (int64_t)k + q] = a.state[9 * (int64_t)k + 3 + q];
            a.ba_out[3 * (int64_t)k + q] = a.state[9 * (int64_t)k + 6 + q];
        }
}

// Validation: endpoints inside their window and distinct, dt > 0, every value finite.
constexpr int32_t kErrInertial = 1 << 10;

__global__ __launch_bounds__(256) void k_vi_check(ViArgs a) {
    const ViEdges &E = a.E;
    for (int e = blockIdx.x * 256 + threadIdx.x; e < E.n; e += gridDim.x * 256) {
        const WinInfo W = a.win[a.edge_win[e]];
        const int i = E.ei[e], j = E.ej[e];
        bool ok = i >= 0 && i < W.K && j >= 0 && j < W.K && i != j && E.dt[e] > 0.0 && isfinite(E.dt[e]);
        for (int q = 0; q < 9 && ok; ++q)
            ok = isfinite(E.dR[9 * e + q]) && isfinite(E.JRg[9 * e + q]) && isfinite(E.Jvg[9 * e + q]) &&
                 isfinite(E.Jva[9 * e + q]) && isfinite(E.Jpg[9 * e + q]) && isfinite(E.Jpa[9 * e + q]);
        for (int q = 0; q < 3 && ok; ++q)
            ok = isfinite(E.dv[3 * e + q]) && isfinite(E.dp[3 * e + q]) && isfinite(E.bgb[3 * e + q]) &&
                 isfinite(E.bab[3 * e + q]);
        for (int q = 0; q < 81 && ok; ++q) ok = isfinite(E.info[81 * (int64_t)e + q]);
        ok = ok && isfinite(E.ibg[e]) && isfinite(E.iba[e]);
        if (!ok) atomicOr(a.err, kErrInertial);
    }
    for (int k = blockIdx.x * 256 + threadIdx.x; k < a.n_kf; k += gridDim.x * 256) {
        bool ok = true;
        for (int q = 0; q < 3; ++q)
            ok = ok && isfinite(a.v0[3 * (int64_t)k + q]) && isfinite(a.bg0[3 * (int64_t)k + q]) &&
                 isfinite(a.ba0[3 * (int64_t)k + q]);
        if (!ok) atomicOr(a.err, kErrInertial);
    }
}

hipError_t launch_vi_setup(const ViArgs &a, hipStream_t s) {
    if (a.n_kf > 0) hipLaunchKernelGGL(k_vi_setup, dim3((a.n_kf + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_vi_finish(const ViArgs &a, hipStream_t s) {
    if (a.n_kf > 0) hipLaunchKernelGGL(k_vi_finish, dim3((a.n_kf + 255) / 256), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_vi_check(const ViArgs &a, hipStream_t s) {
    const int items = std::max(a.E.n, a.n_kf);
    if (items > 0) hipLaunchKernelGGL(k_vi_check, dim3(std::min(1024, (items + 255) / 256)), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_vi_eval(const ViArgs &a, hipStream_t s) {
    if (a.E.n > 0) hipLaunchKernelGGL(k_vi_eval, dim3(a.E.n), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_vi_system(const ViArgs &a, int n_windows, hipStream_t s) {
    if (n_windows > 0) hipLaunchKernelGGL(k_vi_system, dim3(n_windows), dim3(256), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_vi_split(const ViArgs &a, int n_windows, hipStream_t s) {
    if (n_windows > 0) hipLaunchKernelGGL(k_vi_split, dim3(n_windows), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace lba
