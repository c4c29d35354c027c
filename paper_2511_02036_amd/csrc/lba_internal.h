// Internal definitions shared by the HIP translation units of liblba.so: the launch
// plan records, the per-window LM control block, kernel argument packs and the device
// geometry helpers (projection, SE(3) exponential, 3x3 Cholesky).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lba {

constexpr int kWave = 64;
constexpr int kMaxObsPerPoint = 64;   // a point's observations fit one wavefront
constexpr int kMaxKf = 128;           // keyframes per window (poses are staged in LDS)
constexpr int kMaxLevels = 32;
constexpr int kMaxKoptFP64 = 60;
constexpr int kMaxKoptMixed = 60;   // reduced systems of up to 360 unknowns (in HBM above 180)
constexpr int kLinThreads = 512;      // linearisation block (owner-computes reduced system)
constexpr int kUpdThreads = 256;      // update block: 4 wavefronts

// ------------------------------------------------------------------------------------
// launch plan (built on the host, uploaded once per solve)
// ------------------------------------------------------------------------------------
struct WinInfo {
    int32_t kf0, K, pt0, M, ob0, N;   // ranges in the concatenated arrays
    int32_t Kopt, n, E;               // optimisable kfs, n = 6 Kopt, E = n (n + 1) / 2
    int32_t tile0, ntiles;            // tiles of this window in the tile list
    int32_t red_off;                  // doubles: reduced system (E + n) of this window
    int32_t dp_off;                   // doubles: pose step (n) of this window
    int32_t pad;
    int64_t part_off;                 // doubles: partial S (E per tile) of tile 0
    int64_t part_stride;              // doubles per tile: E
    int64_t partr_off;                // doubles: partial r (n per tile) of tile 0
};

struct Tile {
    int32_t win, p0, p1, pad;         // global point range [p0, p1) of one window
};

// per-window Levenberg-Marquardt state, lives in device memory for the whole solve
struct Ctl {
    double lambda, nu, F, F_trial, denom_p;
    double F_initial, F_end_r1, F_start_r2;
    int32_t running, iter, trial, trials_total;
    int32_t cur, solve_ok, iters_r1, iters_r2;
    int32_t term_r1, term_r2, n_outliers, round;
};

// one LM trial as k_decide records it (layout of lba_trial_record)
struct TrialRec {
    int32_t round, iter, trial, accepted, solve_ok, pad;
    double lambda, F, F_trial, gain;
};

struct CamParams {
    double fx, fy, cx, cy, bf;
};

// device view of the observations
struct ObsView {
    const int32_t *kf;      // window-local keyframe
    const int32_t *pt;      // window-local point
    const void *z;          // planar u / v / uR, stride n_obs
    const uint8_t *type;
    const uint8_t *oct;
    int32_t n_obs;
    int32_t z_f32;
};

struct SolveConsts {
    CamParams cam;
    double huber2[2];        // mono, stereo
    double chi2[2];
    double tau;
    double inv_sigma2[kMaxLevels];
    int32_t iters[2];        // per round
    int32_t max_trials;
    int32_t n_windows;
};

struct LinArgs {
    const WinInfo *win;
    const Tile *tiles;
    const int32_t *order;        // launch order: block b processes tile order[b]
    const int32_t *opt_map;      // global kf -> window-local optimisable index or -1
    const int32_t *pt_start;     // global point -> first global observation (n_pt + 1)
    const int4 *pinfo;           // per position of the linearisation order (points sorted by
                                 // keyframes within each window): point, first observation,
                                 // observation count, place of the first observation in
                                 // the observation order that follows the points' order
    ObsView sobs;                // the observations in places (n_obs, same layout as obs)
    const uint8_t *smask;        // round-2 outlier flags in places, or nullptr
    const double *T;             // working poses
    const double *X0, *X1;       // point double buffer
    const Ctl *ctl;
    ObsView obs;
    const uint8_t *mask;         // round-2 outlier flags (1 = inactive) or nullptr
    double *part;                // partial S per tile (packed lower, FP64)
    double *partr;               // FP64 partial r per tile (INIT: diagonal of Hpp)
    double *partd;               // 4 doubles per tile: F, max diag, fail, unused
    double *pf;                  // per point: L^-1 of V (6), t = L^-1 bl (3), bl (3)
    int robust;
    int waves;
    int acc32;                   // mixed precision: sum S and the self terms in FP32
    int self_copies;             // copies of the camera sums of the self terms: one per
                                 // wavefront (bitwise-repeatable sums), or 1
    // chunk records of the pair structure, kept for the rest of an LM round (the pairs of
    // a chunk depend only on which observations are active, which changes only between
    // rounds): a pool of 32-bit words, its size in words and its fill counter, and per
    // tile and pass the word offset of the first record (-1: none, built by the next
    // launch).  plan_head == nullptr: the structure is rebuilt at every step.
    uint32_t *plan;
    unsigned long long *plan_ctr;
    int32_t *plan_head;
    int64_t plan_cap;
    SolveConsts c;
};

// point order of the linearisation (k_order)
struct OrderArgs {
    const WinInfo *win;
    const int32_t *pt_start;     // global point -> first global observation (n_pt + 1)
    const int32_t *opt_map;      // global kf -> window-local optimisable index or -1
    const int32_t *obs_kf;       // window-local keyframe of each observation
    uint16_t *keys;              // per point: lowest | highest << 5 optimisable keyframe (n_pt)
    int32_t *tmp;                // per window, window-local order after the first pass (n_pt)
    int4 *pinfo;                 // result, per position of the order: point, first observation,
                                 // observation count, place of the first observation (n_pt)
    int by_keyframes;            // 1: sort the windows with many optimisable keyframes by
                                 // keyframes; 0: index order everywhere
    int32_t n_pt;
    // observations copied into places (k_order_gather): the order that follows the points'
    ObsView obs;                 // source, in index order
    int32_t *sobs_kf;            // n_obs
    uint8_t *sobs_type, *sobs_oct;
    void *sobs_z;                // 3 x n_obs planar, the type of obs.z
    const uint8_t *mask;         // k_order_gather_mask: outlier flags in index order ...
    uint8_t *smask;              // ... and in places
};

// stereo-inertial measurements (device view of lba_inertial)
struct ViEdges {
    const int32_t *ei, *ej;
    const double *dt, *dR, *dv, *dp, *JRg, *Jvg, *Jva, *Jpg, *Jpa, *bgb, *bab, *info, *ibg, *iba;
    int32_t n, pad;
};

constexpr int kViEdgeStride = 512;   // doubles per measurement: cost, trial cost, b (30), H (465)
constexpr int kViB = 2, kViH = 32;   // offsets of b and of the packed lower H in a record
constexpr int kMaxKoptInertial = 12; // 15 Kopt <= 180

struct ReduceArgs {
    const WinInfo *win;
    const Ctl *ctl;
    const double *part;
    const double *partr;
    const double *partd;
    double *red;                 // per window: E packed-lower S, then n r
    double *redflag;             // per window fail flag
    int max_En;
};

struct CholArgs {
    const WinInfo *win;
    Ctl *ctl;
    const double *red;
    const double *redflag;
    double *dp;
    double *fact;   // systems too large for LDS: per window E doubles at red_off, factored in
                    // place (nullptr: the system is factored in LDS)
};

struct UpdArgs {
    const WinInfo *win;
    const Tile *tiles;
    const int32_t *order;        // launch order: block b processes tile order[b]
    const int32_t *opt_map;
    const int32_t *pt_start;
    const double *T;
    double *X0, *X1;
    const Ctl *ctl;
    const double *dp;
    const double *pf;            // per point factors written by the linearisation of this step
    ObsView obs;
    const uint8_t *mask;
    double *partu;               // 4 doubles per part of a tile: F', denominator part, fail, unused
    int split;                   // parts per tile (one block each)
    int robust;
    int waves;
    SolveConsts c;
};

struct DecideArgs {
    const WinInfo *win;
    Ctl *ctl;
    const int32_t *opt_map;
    double *T;
    const double *dp;
    const double *partu;         // 4 doubles per part of a tile (split parts per tile)
    TrialRec *log;               // per window log_cap records of its trials, or nullptr
    int log_cap;
    int split;
    int round;                   // 1 or 2
    SolveConsts c;
    // stereo-inertial solve (null otherwise)
    const double *vi_ed;         // measurement records: trial costs
    const int32_t *vi_edge_off;
    const double *vi_dp;         // joint step
    const WinInfo *vi_win;
    double *vi_state;
};

struct InitReduceArgs {
    const WinInfo *win;
    Ctl *ctl;
    const double *partr;
    const double *partd;
    int round;
    SolveConsts c;
    // stereo-inertial solve (null otherwise): measurement records, their windows and
    // keyframes
    const double *vi_ed;
    const int32_t *vi_edge_off;
    const int32_t *vi_ei, *vi_ej;
    const int32_t *opt_map;
};

struct MiscArgs {
    const WinInfo *win;
    const int32_t *obs_off_dev;  // n_windows + 1
    const int32_t *pt_off_dev;   // n_windows + 1
    const int32_t *kf_off_dev;
    const double *T_in;
    const double *X_in;
    double *T;
    double *X0, *X1;
    Ctl *ctl;
    int32_t *pt_start;
    ObsView obs;
    uint8_t *flags;
    double *T_out, *X_out;
    double *stats;
    int32_t *err;
    int32_t n_kf, n_pt, n_levels;
    int32_t round;
    int32_t count;               // k_flags: add the flagged observations to Ctl::n_outliers
    const float *xi;             // cost layer: pose perturbations (n_kf x 6, or null: none)
    float *Pf;                   // cost layer: Exp(xi_k) T_k in FP32 (n_kf x 12); null: skip
    SolveConsts c;
};

// differentiation form: one window of the robust-cost layer
struct CostWin {
    int32_t kf0, K, pt0, M, ob0, N;   // ranges in the concatenated arrays
    int32_t tile0, ntiles;            // tiles of this window in the tile list
    int64_t g_off;                    // doubles: per-tile pose-gradient partials (ntiles x K x 6)
};

struct CostArgs {
    const CostWin *win;
    const Tile *tiles;
    const int32_t *pt_start;     // global point -> first global observation (n_pt + 1)
    const double *T;             // base poses, n_kf x 12
    const float *xi;             // left perturbations, n_kf x 6, or nullptr (zero)
    const float *Pf;             // Exp(xi_k) T_k in FP32, n_kf x 12 (formed by k_setup)
    const float *X;              // points, n_pt x 3
    const float *z;              // measurements, 3 x n_obs planar
    const int32_t *obs_kf, *obs_pt;
    const uint8_t *obs_type, *obs_oct;
    const uint8_t *mask;         // 1 = observation left out, or nullptr
    const double *grad_cost;     // backward: dL/dcost per window
    float *g_xi, *g_X, *g_z;     // backward outputs
    double *cost;                // forward output, per window
    double *partF;               // per tile cost
    double *partG;               // per tile pose-gradient partials (left-trivialised)
    int32_t *err;                // set when a tile meets an observation it cannot place
    int32_t n_obs;
    CamParams cam;
    double huber2[2];
    double inv_sigma2[kMaxLevels];
};

// ------------------------------------------------------------------------------------
// launchers (one per translation unit that owns the kernel)
// ------------------------------------------------------------------------------------
struct ViArgs {
    ViEdges E;
    const WinInfo *win;          // visual records
    const WinInfo *vwin;         // records of the joint reduced system: n = 15 Kopt, E, red_off, dp_off
    const int32_t *edge_win;     // window of each measurement
    const int32_t *edge_off;     // n_windows + 1
    const int32_t *opt_map;
    Ctl *ctl;
    const double *T;             // current poses
    double *state;               // per keyframe: v (3), bg (3), ba (3)
    const double *v0, *bg0, *ba0;
    double *v_out, *bg_out, *ba_out;
    const double *dp;            // visual pose step (6 per optimisable keyframe)
    double *dpv;                 // visual pose step written from the joint one
    const double *vdp;           // joint step (15 per optimisable keyframe)
    const double *red;           // visual reduced system (packed lower S, then r)
    double *vred;                // joint reduced system
    double *ed;                  // per measurement record (kViEdgeStride doubles)
    int32_t *err;
    double Tcb[12];
    double g[3];
    int trial;                   // k_vi_eval: 0 = linearise at the current state, 1 = trial cost
    int n_kf;
};

hipError_t launch_vi_setup(const ViArgs &a, hipStream_t s);
hipError_t launch_vi_check(const ViArgs &a, hipStream_t s);
hipError_t launch_vi_eval(const ViArgs &a, hipStream_t s);
hipError_t launch_vi_system(const ViArgs &a, int n_windows, hipStream_t s);
hipError_t launch_vi_split(const ViArgs &a, int n_windows, hipStream_t s);
hipError_t launch_vi_finish(const ViArgs &a, hipStream_t s);

hipError_t launch_linearize(const LinArgs &a, int ntiles, int passes, size_t lds, bool mixed, hipStream_t s);
hipError_t launch_plan_reset(const LinArgs &a, int slots, hipStream_t s);   // forget the chunk records
int lin_passes(int kopt);   // passes over the camera blocks of a window with kopt optimisable keyframes
hipError_t launch_update(const UpdArgs &a, int ntiles, size_t lds, bool mixed, hipStream_t s);
hipError_t launch_init(const LinArgs &a, int ntiles, size_t lds, hipStream_t s);
hipError_t launch_reduce(const ReduceArgs &a, int n_windows, hipStream_t s);
hipError_t launch_cholesky(const CholArgs &a, int n_windows, size_t lds, hipStream_t s);
size_t chol_lds_bytes_hbm(int n);   // LDS of the variant whose matrix is in HBM
int chol_reg_max_n();               // largest system the register-tile variant factors
hipError_t launch_decide(const DecideArgs &a, int n_windows, hipStream_t s);
hipError_t launch_init_reduce(const InitReduceArgs &a, int n_windows, hipStream_t s);
hipError_t launch_setup(const MiscArgs &a, int n_windows, hipStream_t s);
hipError_t launch_order(const OrderArgs &a, int n_windows, int max_points, int max_kopt, hipStream_t s);
hipError_t launch_order_gather(const OrderArgs &a, bool mask, hipStream_t s);
hipError_t launch_validate(const MiscArgs &a, int n_windows, int64_t max_obs, hipStream_t s);
hipError_t launch_flags(const MiscArgs &a, int n_windows, int64_t max_obs, hipStream_t s);
hipError_t launch_finalize(const MiscArgs &a, int n_windows, hipStream_t s);
hipError_t launch_cost(const CostArgs &a, int ntiles, int max_k, bool backward, hipStream_t s);
hipError_t launch_cost_reduce(const CostArgs &a, int n_windows, bool backward, hipStream_t s);

// LDS bytes of the linearisation / update blocks for a window shape
// The static LDS of a kernel (the runtime's block reductions behind __syncthreads_count
// and the like take some): it comes on top of the dynamic LDS a launch asks for.
inline size_t kernel_static_lds(const void *f) {
    hipFuncAttributes fa;
    return hipFuncGetAttributes(&fa, f) == hipSuccess ? fa.sharedSizeBytes : 1024;
}
size_t lin_static_lds();
size_t init_static_lds();
size_t chol_static_lds();
size_t cost_static_lds();
size_t lin_lds_bytes(int K, int kopt, int copies, bool mixed);
int lin_self_copies(bool mixed);   // copies of the camera sums for bitwise-repeatable solves
size_t upd_lds_bytes(int K, int n, int waves, bool mixed);
size_t cost_lds_bytes(int K, bool backward);
size_t init_lds_bytes(int K, int n);

#if defined(__HIPCC__)
// ------------------------------------------------------------------------------------
// device helpers
// ------------------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T>
__device__ __forceinline__ void lds_add(T *p, T v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ int wave_exclusive_scan(int v, int lane) {
    int x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        int y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    return x - v;
}

// exact SE(3) exponential of the twist (w, v): R = I + A W + B W^2, t = (I + B W + C W^2) v,
// A = sin(t)/t, B = (1 - cos t)/t^2, C = (t - sin t)/t^3; power series below 1e-2
__device__ inline void se3_exp(const double *xi, double *R, double *t) {
    const double w0 = xi[0], w1 = xi[1], w2 = xi[2];
    const double th2 = w0 * w0 + w1 * w1 + w2 * w2;
    const double th = sqrt(th2);
    double A, B, C;
    if (th < 1e-2) {
        const double t4 = th2 * th2, t6 = t4 * th2;
        A = 1.0 - th2 * (1.0 / 6.0) + t4 * (1.0 / 120.0) - t6 * (1.0 / 5040.0);
        B = 0.5 - th2 * (1.0 / 24.0) + t4 * (1.0 / 720.0) - t6 * (1.0 / 40320.0);
        C = 1.0 / 6.0 - th2 * (1.0 / 120.0) + t4 * (1.0 / 5040.0) - t6 * (1.0 / 362880.0);
    } else {
        const double s = sin(th), h = sin(0.5 * th);
        A = s / th;
        B = 2.0 * h * h / th2;
        C = (th - s) / (th2 * th);
    }
    // W^2 = w w^T - th2 I
    const double W[9] = {0.0, -w2, w1, w2, 0.0, -w0, -w1, w0, 0.0};
    const double ww[9] = {w0 * w0 - th2, w0 * w1, w0 * w2, w1 * w0, w1 * w1 - th2, w1 * w2,
                          w2 * w0, w2 * w1, w2 * w2 - th2};
    double V[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) {
        const double I = (i % 4 == 0) ? 1.0 : 0.0;
        R[i] = I + A * W[i] + B * ww[i];
        V[i] = I + B * W[i] + C * ww[i];
    }
    const double v0 = xi[3], v1 = xi[4], v2 = xi[5];
    t[0] = V[0] * v0 + V[1] * v1 + V[2] * v2;
    t[1] = V[3] * v0 + V[4] * v1 + V[5] * v2;
    t[2] = V[6] * v0 + V[7] * v1 + V[8] * v2;
}

// Tout = Exp(xi) * Tin (3x4 row-major)
__device__ inline void se3_left_update(const double *xi, const double *Tin, double *Tout) {
    double R[9], t[3];
    se3_exp(xi, R, t);
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
        for (int c = 0; c < 4; ++c)
            Tout[r * 4 + c] = R[r * 3] * Tin[c] + R[r * 3 + 1] * Tin[4 + c] + R[r * 3 + 2] * Tin[8 + c] +
                              (c == 3 ? t[r] : 0.0);
    }
}

__device__ __forceinline__ void huber(double s, double d2, int robust, double &rho, double &w) {
    if (!robust || s <= d2) {
        rho = s;
        w = 1.0;
    } else {
        const double rs = sqrt(s), d = sqrt(d2);
        rho = 2.0 * d * rs - d2;
        w = d / rs;
    }
}

template <typename ZT>
__device__ __forceinline__ void load_z(const ObsView &ob, int o, double &u, double &v, double &ur) {
    const ZT *z = static_cast<const ZT *>(ob.z);
    u = (double)z[o];
    v = (double)z[(int64_t)ob.n_obs + o];
    ur = (double)z[2 * (int64_t)ob.n_obs + o];
}

// residual of one observation at pose T (3x4) and point X; returns s, the camera point and
// the residual (er = 0 for mono)
__device__ __forceinline__ double residual(const CamParams &cam, const double *T, double X0, double X1,
                                           double X2, double zu, double zv, double zr, int stereo,
                                           double &xc, double &yc, double &zc, double &eu, double &ev,
                                           double &er) {
    xc = T[0] * X0 + T[1] * X1 + T[2] * X2 + T[3];
    yc = T[4] * X0 + T[5] * X1 + T[6] * X2 + T[7];
    zc = T[8] * X0 + T[9] * X1 + T[10] * X2 + T[11];
    const double iz = 1.0 / zc;
    const double u = cam.fx * xc * iz + cam.cx;
    const double v = cam.fy * yc * iz + cam.cy;
    eu = zu - u;
    ev = zv - v;
    er = stereo ? zr - (u - cam.bf * iz) : 0.0;
    return eu * eu + ev * ev + er * er;
}

// 3x3 SPD Cholesky V = L L^T and the inverse factor Li = L^-1 (both lower, 6 entries in
// order 00 10 11 20 21 22).  Returns false if a pivot is not positive.
template <typename Real>
__device__ __forceinline__ bool chol3_inv(const Real *V /*00 01 02 11 12 22*/, Real *Li) {
    const Real v00 = V[0], v01 = V[1], v02 = V[2], v11 = V[3], v12 = V[4], v22 = V[5];
    if (!(v00 > Real(0))) return false;
    const Real l00 = sqrt(v00);
    const Real l10 = v01 / l00, l20 = v02 / l00;
    const Real d1 = v11 - l10 * l10;
    if (!(d1 > Real(0))) return false;
    const Real l11 = sqrt(d1);
    const Real l21 = (v12 - l20 * l10) / l11;
    const Real d2 = v22 - l20 * l20 - l21 * l21;
    if (!(d2 > Real(0))) return false;
    const Real l22 = sqrt(d2);
    const Real i00 = Real(1) / l00, i11 = Real(1) / l11, i22 = Real(1) / l22;
    const Real i10 = -l10 * i00 * i11;
    const Real i21 = -l21 * i11 * i22;
    const Real i20 = -(l20 * i00 + l21 * i10) * i22;
    Li[0] = i00; Li[1] = i10; Li[2] = i11; Li[3] = i20; Li[4] = i21; Li[5] = i22;
    return true;
}

// y = Li x (lower triangular)
template <typename Real>
__device__ __forceinline__ void lmul(const Real *Li, Real x0, Real x1, Real x2, Real &y0, Real &y1,
                                     Real &y2) {
    y0 = Li[0] * x0;
    y1 = Li[1] * x0 + Li[2] * x1;
    y2 = Li[3] * x0 + Li[4] * x1 + Li[5] * x2;
}

// y = Li^T x
template <typename Real>
__device__ __forceinline__ void ltmul(const Real *Li, Real x0, Real x1, Real x2, Real &y0, Real &y1,
                                      Real &y2) {
    y0 = Li[0] * x0 + Li[1] * x1 + Li[3] * x2;
    y1 = Li[2] * x1 + Li[4] * x2;
    y2 = Li[5] * x2;
}

// Gauss-Newton blocks of one observation, in the factored form
//   G = om P^T P (3x3),  g = om P^T e,  M = G R,
//   Hll = R^T G R,  bl = R^T g,  W = [x]x M ; M  (6x3),  bp = (x cross g ; g),
//   Hpp = [[ [x]x G [x]x^T, [x]x G ], [ . , G ]]
// where P = d pi / d Xc, x = Xc and R the pose rotation.
template <typename Real>
struct ObsBlocks {
    Real G[6];      // 00 01 02 11 12 22
    Real g[3];
    Real M[9];      // row-major
    Real x[3];
    Real R[9];
};

template <typename Real>
__device__ __forceinline__ void obs_blocks(const CamParams &cam, const double *T, double xc, double yc,
                                           double zc, double eu, double ev, double er, int stereo,
                                           Real om, ObsBlocks<Real> &B) {
    const Real x = (Real)xc, y = (Real)yc, z = (Real)zc;
    const Real iz = Real(1) / z;
    const Real fx = (Real)cam.fx, fy = (Real)cam.fy, bf = (Real)cam.bf;
    const Real p00 = fx * iz, p02 = -fx * x * iz * iz;
    const Real p11 = fy * iz, p12 = -fy * y * iz * iz;
    const Real st = stereo ? Real(1) : Real(0);
    const Real p22 = -(fx * x - bf) * iz * iz;
    const Real e0 = (Real)eu, e1 = (Real)ev, e2 = (Real)er;
    B.G[0] = om * (p00 * p00 * (Real(1) + st));
    B.G[1] = Real(0);
    B.G[2] = om * (p00 * p02 + st * p00 * p22);
    B.G[3] = om * (p11 * p11);
    B.G[4] = om * (p11 * p12);
    B.G[5] = om * (p02 * p02 + p12 * p12 + st * p22 * p22);
    B.g[0] = om * (p00 * e0 + st * p00 * e2);
    B.g[1] = om * (p11 * e1);
    B.g[2] = om * (p02 * e0 + p12 * e1 + st * p22 * e2);
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int c = 0; c < 3; ++c) B.R[r * 3 + c] = (Real)T[r * 4 + c];
    const Real G00 = B.G[0], G01 = B.G[1], G02 = B.G[2], G11 = B.G[3], G12 = B.G[4], G22 = B.G[5];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const Real r0 = B.R[c], r1 = B.R[3 + c], r2 = B.R[6 + c];
        B.M[0 * 3 + c] = G00 * r0 + G01 * r1 + G02 * r2;
        B.M[1 * 3 + c] = G01 * r0 + G11 * r1 + G12 * r2;
        B.M[2 * 3 + c] = G02 * r0 + G12 * r1 + G22 * r2;
    }
    B.x[0] = x; B.x[1] = y; B.x[2] = z;
}

// gradient piece g = om P^T e of an observation in FP64 (P = d pi / d Xc)
__device__ __forceinline__ void obs_gradient(const CamParams &cam, double xc, double yc, double zc, double eu,
                                             double ev, double er, int stereo, double om, double *g) {
    const double iz = 1.0 / zc, st = stereo ? 1.0 : 0.0;
    const double p00 = cam.fx * iz, p02 = -cam.fx * xc * iz * iz;
    const double p11 = cam.fy * iz, p12 = -cam.fy * yc * iz * iz;
    const double p22 = -(cam.fx * xc - cam.bf) * iz * iz;
    g[0] = om * (p00 * eu + st * p00 * er);
    g[1] = om * (p11 * ev);
    g[2] = om * (p02 * eu + p12 * ev + st * p22 * er);
}

// point block of an observation in FP64: Hll = R^T G R (6 upper entries) and bl = R^T g,
// G = om P^T P, g = om P^T e.  The 3x3 point blocks are factored in FP64 in every
// precision: a point left with one monocular observation has a rank-2 Hll, so V = Hll +
// lambda I is conditioned like max(Hll) / lambda and loses its small pivot in FP32.
__device__ __forceinline__ void point_block_fp64(const CamParams &cam, const double *T, double xc, double yc,
                                                 double zc, double eu, double ev, double er, int stereo,
                                                 double om, double *Hll, double *bl) {
    const double iz = 1.0 / zc, st = stereo ? 1.0 : 0.0;
    const double p00 = cam.fx * iz, p02 = -cam.fx * xc * iz * iz;
    const double p11 = cam.fy * iz, p12 = -cam.fy * yc * iz * iz;
    const double p22 = -(cam.fx * xc - cam.bf) * iz * iz;
    const double G00 = om * (p00 * p00 * (1.0 + st)), G02 = om * (p00 * p02 + st * p00 * p22);
    const double G11 = om * (p11 * p11), G12 = om * (p11 * p12);
    const double G22 = om * (p02 * p02 + p12 * p12 + st * p22 * p22);
    const double g0 = om * (p00 * eu + st * p00 * er), g1 = om * (p11 * ev);
    const double g2 = om * (p02 * eu + p12 * ev + st * p22 * er);
    double M[9];   // G R
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double r0 = T[c], r1 = T[4 + c], r2 = T[8 + c];
        M[c] = G00 * r0 + G02 * r2;
        M[3 + c] = G11 * r1 + G12 * r2;
        M[6 + c] = G02 * r0 + G12 * r1 + G22 * r2;
    }
    Hll[0] = T[0] * M[0] + T[4] * M[3] + T[8] * M[6];
    Hll[1] = T[0] * M[1] + T[4] * M[4] + T[8] * M[7];
    Hll[2] = T[0] * M[2] + T[4] * M[5] + T[8] * M[8];
    Hll[3] = T[1] * M[1] + T[5] * M[4] + T[9] * M[7];
    Hll[4] = T[1] * M[2] + T[5] * M[5] + T[9] * M[8];
    Hll[5] = T[2] * M[2] + T[6] * M[5] + T[10] * M[8];
#pragma unroll
    for (int i = 0; i < 3; ++i) bl[i] = T[i] * g0 + T[4 + i] * g1 + T[8 + i] * g2;
}

// q = W_a^T dp = R^T G c of an observation in FP64, for the camera-frame motion
// c = dw x Xc + dv of a pose step dp = (dw, dv), G = om P^T P (P = d pi / d Xc)
__device__ __forceinline__ void obs_step_q(const CamParams &cam, const double *T, double xc, double yc, double zc,
                                           int stereo, double om, double c0, double c1, double c2, double *q) {
    const double iz = 1.0 / zc, st = stereo ? 1.0 : 0.0;
    const double p00 = cam.fx * iz, p02 = -cam.fx * xc * iz * iz;
    const double p11 = cam.fy * iz, p12 = -cam.fy * yc * iz * iz;
    const double p22 = -(cam.fx * xc - cam.bf) * iz * iz;
    const double G00 = om * (p00 * p00 * (1.0 + st)), G02 = om * (p00 * p02 + st * p00 * p22);
    const double G11 = om * (p11 * p11), G12 = om * (p11 * p12);
    const double G22 = om * (p02 * p02 + p12 * p12 + st * p22 * p22);
    const double g0 = G00 * c0 + G02 * c2, g1 = G11 * c1 + G12 * c2, g2 = G02 * c0 + G12 * c1 + G22 * c2;
#pragma unroll
    for (int i = 0; i < 3; ++i) q[i] = T[i] * g0 + T[4 + i] * g1 + T[8 + i] * g2;
}

// Hll (6 upper entries) and bl of an observation
template <typename Real>
__device__ __forceinline__ void point_terms(const ObsBlocks<Real> &B, Real *Hll, Real *bl) {
    // Hll = R^T M
    Real H[9];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int c = 0; c < 3; ++c)
            H[a * 3 + c] = B.R[a] * B.M[c] + B.R[3 + a] * B.M[3 + c] + B.R[6 + a] * B.M[6 + c];
    Hll[0] = H[0]; Hll[1] = H[1]; Hll[2] = H[2]; Hll[3] = H[4]; Hll[4] = H[5]; Hll[5] = H[8];
#pragma unroll
    for (int a = 0; a < 3; ++a) bl[a] = B.R[a] * B.g[0] + B.R[3 + a] * B.g[1] + B.R[6 + a] * B.g[2];
}

template <typename Real>
__device__ __forceinline__ void cross3(const Real *a, Real b0, Real b1, Real b2, Real &c0, Real &c1,
                                       Real &c2) {
    c0 = a[1] * b2 - a[2] * b1;
    c1 = a[2] * b0 - a[0] * b2;
    c2 = a[0] * b1 - a[1] * b0;
}

// W (6x3 row-major) = [x]x M ; M
template <typename Real>
__device__ __forceinline__ void pose_point_block(const ObsBlocks<Real> &B, Real *W) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Real c0, c1, c2;
        cross3(B.x, B.M[c], B.M[3 + c], B.M[6 + c], c0, c1, c2);
        W[0 * 3 + c] = c0; W[1 * 3 + c] = c1; W[2 * 3 + c] = c2;
        W[3 * 3 + c] = B.M[c]; W[4 * 3 + c] = B.M[3 + c]; W[5 * 3 + c] = B.M[6 + c];
    }
}

// full 6x6 Hpp (row-major) and bp
template <typename Real>
__device__ __forceinline__ void pose_terms(const ObsBlocks<Real> &B, Real *H, Real *bp) {
    const Real Gf[9] = {B.G[0], B.G[1], B.G[2], B.G[1], B.G[3], B.G[4], B.G[2], B.G[4], B.G[5]};
    Real Cm[9];   // [x]x G
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        Real c0, c1, c2;
        cross3(B.x, Gf[c], Gf[3 + c], Gf[6 + c], c0, c1, c2);
        Cm[c] = c0; Cm[3 + c] = c1; Cm[6 + c] = c2;
    }
#pragma unroll
    for (int r = 0; r < 3; ++r) {
        Real q0, q1, q2;   // row r of [x]x G [x]x^T = x cross (row r of Cm)
        cross3(B.x, Cm[r * 3], Cm[r * 3 + 1], Cm[r * 3 + 2], q0, q1, q2);
        H[r * 6 + 0] = q0; H[r * 6 + 1] = q1; H[r * 6 + 2] = q2;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            H[r * 6 + 3 + c] = Cm[r * 3 + c];
            H[(3 + c) * 6 + r] = Cm[r * 3 + c];
            H[(3 + r) * 6 + 3 + c] = Gf[r * 3 + c];
        }
    }
    Real c0, c1, c2;
    cross3(B.x, B.g[0], B.g[1], B.g[2], c0, c1, c2);
    bp[0] = c0; bp[1] = c1; bp[2] = c2; bp[3] = B.g[0]; bp[4] = B.g[1]; bp[5] = B.g[2];
}

__device__ __forceinline__ int packed_lower(int row, int col) { return row * (row + 1) / 2 + col; }
#endif  // __HIPCC__

}  // namespace lba
