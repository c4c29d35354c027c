// C ABI of liblba.so: argument validation, launch planning, workspace layout and the
// host-side sequencing of the Levenberg-Marquardt rounds.  All numerical work runs in
// the kernels of the other translation units; this file only decides what to launch.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <unordered_map>
#include <vector>

#include "lba.h"
#include "lba_internal.h"

using namespace lba;

static_assert(sizeof(TrialRec) == sizeof(lba_trial_record), "trial record layout");

struct lba_ctx {
    lba_options opt;
    int device = 0;
    int max_lds = 65536;
    std::string err;
    void *pinned = nullptr;
    size_t pinned_bytes = 0;
    hipEvent_t upload_ev = nullptr;   // recorded after the last copy out of `pinned`
    bool upload_pending = false;
    // LM-step graphs: captured on a private stream, replayed on the caller's
    hipStream_t cap_stream = nullptr;
    struct GraphEntry {
        hipGraph_t graph;
        hipGraphExec_t exec;
        uint64_t used;   // value of graph_clock at the last use
    };
    std::unordered_map<std::string, GraphEntry> graphs;
    uint64_t graph_clock = 0;
    // tile tuner: points per tile by window class (optimisable keyframes x points, see
    // window_class); tuned_sig[0] == -2 marks a table installed by lba_tune_set, which
    // applies to every problem
    int64_t tuned_sig[5] = {-1, -1, -1, -1, -1};
    int tuned_ppt[LBA_TUNE_CLASSES] = {};
    const int *ppt_override = nullptr;   // set while the tuner measures a candidate
    // kernel timing
    bool prof = false;
    std::vector<hipEvent_t> ev_pool;
    std::vector<int> pending_cls;    // class of each recorded pair, pair i = events 2i, 2i+1
    double prof_ms[LBA_KCLASS_COUNT] = {};
    int64_t prof_n[LBA_KCLASS_COUNT] = {};
};

namespace {

lba_status set_error(lba_ctx *ctx, lba_status st, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    if (ctx) ctx->err = buf;
    return st;
}

#define HIPCHK(call)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (call);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return set_error(ctx, LBA_ERR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

constexpr size_t kGraphCache = 1024;

struct Plan {
    int nw = 0;
    int64_t max_obs = 0;
    int max_pts = 0;
    int max_kopt = 0;
    int upd_split = 1;
    bool mixed = false;
    int waves = 4;
    std::vector<WinInfo> win;
    std::vector<Tile> tiles;
    std::vector<int32_t> order;   // launch order of the tiles: estimated heaviest first
    std::vector<int32_t> opt_map;
    std::vector<int32_t> kf_off, pt_off, obs_off;
    size_t lin_lds = 0, upd_lds = 0, chol_lds = 0, init_lds = 0;
    bool chol_hbm = false;   // reduced systems factored in HBM (too large for LDS)
    int lin_passes = 1;      // linearisation passes over the camera blocks
    int lin_copies = 1;   // copies of the linearisation's camera sums
    int max_En = 0;
    int64_t part_elems = 0;
    int64_t partr_elems = 0;
    int64_t red_elems = 0;
    int64_t dp_elems = 0;
    // workspace byte offsets
    size_t o_win, o_tiles, o_order, o_opt, o_kfoff, o_ptoff, o_obsoff, o_upload_end;
    size_t o_ptstart, o_ctl, o_T, o_X0, o_X1, o_part, o_partr, o_partd, o_partu, o_red, o_fact, o_redflag, o_dp, o_pf,
        o_pkey, o_ptmp, o_pinfo, o_skf, o_stype, o_soct, o_sz, o_smask, o_stats, o_err, o_log, o_planhead, o_planctr,
        o_plan, total;
    int64_t plan_cap = 0;   // words of the pool of chunk records (0: rebuilt at every step)
    int log_cap = 0;
    // stereo-inertial solve
    bool vi = false;
    std::vector<WinInfo> vwin;         // joint reduced systems (n = 15 Kopt)
    std::vector<int32_t> edge_win, edge_off;
    size_t o_vwin = 0, o_edgewin = 0, o_edgeoff = 0, o_vred = 0, o_vdp = 0, o_state = 0, o_ed = 0;
};

int choose_points_per_tile(const lba_options &opt, int64_t total_points) {
    if (opt.points_per_tile > 0) return opt.points_per_tile;
    // about four blocks per compute unit over the whole batch, each block large enough
    // that its partial reduced system is small next to the observations it reads
    const int64_t target_blocks = 1024;
    int64_t p = (total_points + target_blocks - 1) / target_blocks;
    p = (p + 31) / 32 * 32;
    p = std::max<int64_t>(64, std::min<int64_t>(4096, p));
    return (int)p;
}

// The cost layer has no per-tile reduced system, so its tiles are small: about 448
// observations each (two mostly full 256-observation chunks), which gives a few
// thousand blocks over a batch.  Measured on 64 windows of 2,000 points and about 6.7
// observations per point: tiles of 64 points beat 16, 24, 33, 48 and 128 (one chunk per
// tile pays the block's fixed costs too often; four chunks leave too few blocks).
int choose_cost_points_per_tile(const lba_options &opt, int64_t total_points, int64_t total_obs) {
    if (opt.points_per_tile > 0) return opt.points_per_tile;
    if (total_points <= 0 || total_obs <= 0) return 64;
    int64_t p = (int64_t)(448.0 * (double)total_points / (double)total_obs);
    return (int)std::max<int64_t>(1, std::min<int64_t>(4096, p));
}

int kopt_class(int kopt) { return kopt <= 10 ? 0 : (kopt <= 20 ? 1 : 2); }

// tuner class of a window: optimisable keyframes (<= 10, <= 20, > 20) x points (< 2,000,
// < 8,000, >= 8,000)
int window_class(int kopt, int points) {
    return 3 * kopt_class(kopt) + (points < 2000 ? 0 : (points < 8000 ? 1 : 2));
}

void tune_signature(const lba_problem *P, int nw, bool mixed, int64_t *sig) {
    sig[0] = P->n_kf;
    sig[1] = P->n_pt;
    sig[2] = P->n_obs;
    sig[3] = nw;
    sig[4] = mixed ? 1 : 0;
}

bool tune_signature_matches(const lba_ctx *ctx, const lba_problem *P, int nw, bool mixed) {
    if (ctx->tuned_sig[0] == -2) return true;
    int64_t sig[5];
    tune_signature(P, nw, mixed, sig);
    for (int i = 0; i < 5; ++i)
        if (sig[i] != ctx->tuned_sig[i]) return false;
    return true;
}

lba_status build_plan(lba_ctx *ctx, const lba_problem *P, const lba_batch *B, Plan &pl,
                      const lba_inertial *I = nullptr) {
    if (!P) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "problem is NULL");
    if (P->n_kf < 0 || P->n_pt < 0 || P->n_obs < 0)
        return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "negative size");
    if (P->n_levels < 1 || P->n_levels > kMaxLevels)
        return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "n_levels must be in [1, %d]", kMaxLevels);
    if (!P->sigma2) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "sigma2 (host) is NULL");
    for (int i = 0; i < P->n_levels; ++i)
        if (!(P->sigma2[i] > 0.0) || !std::isfinite(P->sigma2[i]))
            return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "sigma2[%d] must be positive", i);
    if (P->n_kf > 0 && (!P->T_cw || !P->fixed))
        return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "T_cw / fixed is NULL");
    if (P->n_pt > 0 && !P->X_w) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "X_w is NULL");
    if (P->n_obs > 0 && (!P->obs_kf || !P->obs_pt || !P->obs_z || !P->obs_type || !P->obs_oct))
        return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "an observation array is NULL");
    if (!(P->cam.fx > 0.0) || !(P->cam.fy > 0.0) || !std::isfinite(P->cam.cx) ||
        !std::isfinite(P->cam.cy) || !std::isfinite(P->cam.bf))
        return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "invalid intrinsics");
    const lba_options &opt = ctx->opt;
    pl.mixed = opt.precision == LBA_PREC_MIXED;

    if (B) {
        if (B->n_windows < 1 || !B->kf_off || !B->pt_off || !B->obs_off)
            return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "invalid batch description");
        pl.nw = B->n_windows;
        pl.kf_off.assign(B->kf_off, B->kf_off + pl.nw + 1);
        pl.pt_off.assign(B->pt_off, B->pt_off + pl.nw + 1);
        pl.obs_off.assign(B->obs_off, B->obs_off + pl.nw + 1);
    } else {
        pl.nw = 1;
        pl.kf_off = {0, P->n_kf};
        pl.pt_off = {0, P->n_pt};
        pl.obs_off = {0, P->n_obs};
    }
    const int nw = pl.nw;
    if (pl.kf_off[0] != 0 || pl.pt_off[0] != 0 || pl.obs_off[0] != 0 || pl.kf_off[nw] != P->n_kf ||
        pl.pt_off[nw] != P->n_pt || pl.obs_off[nw] != P->n_obs)
        return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "batch offsets must start at 0 and end at the totals");

    int64_t total_points = P->n_pt;
    const int ppt_default = choose_points_per_tile(opt, total_points);
    const int *class_ppt = nullptr;
    if (opt.points_per_tile <= 0) {
        if (ctx->ppt_override) class_ppt = ctx->ppt_override;
        else if (tune_signature_matches(ctx, P, nw, pl.mixed)) class_ppt = ctx->tuned_ppt;
    }
    const int kopt_max = pl.mixed ? kMaxKoptMixed : kMaxKoptFP64;
    pl.win.resize(nw);
    pl.opt_map.assign(P->n_kf, -1);
    pl.tiles.clear();
    int64_t part = 0, partr = 0, red = 0, dpo = 0;
    int maxK = 1, maxn = 0;
    for (int w = 0; w < nw; ++w) {
        WinInfo &W = pl.win[w];
        W.kf0 = pl.kf_off[w];
        W.K = pl.kf_off[w + 1] - pl.kf_off[w];
        W.pt0 = pl.pt_off[w];
        W.M = pl.pt_off[w + 1] - pl.pt_off[w];
        W.ob0 = pl.obs_off[w];
        W.N = pl.obs_off[w + 1] - pl.obs_off[w];
        if (W.K < 0 || W.M < 0 || W.N < 0)
            return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "batch offsets decrease at window %d", w);
        if (W.K > kMaxKf)
            return set_error(ctx, LBA_ERR_UNSUPPORTED, "window %d has %d keyframes (limit %d)", w, W.K, kMaxKf);
        int kopt = 0;
        for (int k = 0; k < W.K; ++k) {
            const uint8_t f = P->fixed[W.kf0 + k];
            if (f > 1) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "fixed[%d] is not 0/1", W.kf0 + k);
            pl.opt_map[W.kf0 + k] = f ? -1 : kopt++;
        }
        if (kopt > kopt_max)
            return set_error(ctx, LBA_ERR_UNSUPPORTED, "window %d has %d optimisable keyframes (limit %d for this precision)",
                             w, kopt, kopt_max);
        if (I && kopt > kMaxKoptInertial)
            return set_error(ctx, LBA_ERR_UNSUPPORTED,
                             "window %d has %d optimisable keyframes (limit %d with inertial measurements)", w, kopt,
                             kMaxKoptInertial);
        W.Kopt = kopt;
        W.n = 6 * kopt;
        W.E = W.n * (W.n + 1) / 2;
        const int ppt = class_ppt ? class_ppt[window_class(kopt, W.M)] : ppt_default;
        W.tile0 = (int)pl.tiles.size();
        W.ntiles = (W.M + ppt - 1) / ppt;
        for (int t = 0; t < W.ntiles; ++t) {
            Tile T;
            T.win = w;
            T.p0 = W.pt0 + t * ppt;
            T.p1 = W.pt0 + std::min(W.M, (t + 1) * ppt);
            T.pad = 0;
            pl.tiles.push_back(T);
        }
        W.part_stride = W.E;
        W.part_off = part;
        part += W.part_stride * W.ntiles;
        W.partr_off = partr;
        partr += (int64_t)W.n * W.ntiles;
        W.red_off = (int32_t)red;
        red += W.E + W.n;
        W.dp_off = (int32_t)dpo;
        dpo += W.n;
        W.pad = 0;
        maxK = std::max(maxK, W.K);
        maxn = std::max(maxn, W.n);
        pl.max_En = std::max(pl.max_En, W.E + W.n);
        pl.max_obs = std::max<int64_t>(pl.max_obs, W.N);
        pl.max_pts = std::max(pl.max_pts, W.M);
        pl.max_kopt = std::max(pl.max_kopt, W.Kopt);
    }
    if (red > INT32_MAX) return set_error(ctx, LBA_ERR_UNSUPPORTED, "batch too large");
    // launch the tiles heaviest first (estimated observations times a cost growing with
    // the window's reduced system), so that the light ones fill the end of the launch
    {
        std::vector<double> wgt(pl.tiles.size());
        for (size_t t = 0; t < pl.tiles.size(); ++t) {
            const Tile &T = pl.tiles[t];
            const WinInfo &W = pl.win[T.win];
            const double obs = W.M > 0 ? (double)W.N * (T.p1 - T.p0) / W.M : 0.0;
            wgt[t] = obs * (W.Kopt + 8);
        }
        pl.order.resize(pl.tiles.size());
        for (size_t t = 0; t < pl.order.size(); ++t) pl.order[t] = (int32_t)t;
        std::stable_sort(pl.order.begin(), pl.order.end(), [&](int32_t x, int32_t y) { return wgt[x] > wgt[y]; });
    }
    pl.part_elems = std::max<int64_t>(part, 1);
    pl.partr_elems = std::max<int64_t>(partr, 1);
    pl.red_elems = std::max<int64_t>(red, 1);
    pl.dp_elems = std::max<int64_t>(dpo, 1);

    // LDS: the update block uses four wavefronts if its staging fits, fewer otherwise
    pl.waves = 0;
    for (int wv = 4; wv >= 1; wv /= 2) {
        if (upd_lds_bytes(maxK, maxn, wv, pl.mixed) <= (size_t)ctx->max_lds) {
            pl.waves = wv;
            break;
        }
    }
    // the linearisation keeps one copy of its camera sums per wavefront (bitwise-repeatable
    // solves) where LDS allows, else one copy for the block
    pl.lin_copies = lin_self_copies(pl.mixed);
    const size_t lin_room = (size_t)ctx->max_lds - std::min((size_t)ctx->max_lds, lin_static_lds());
    if (lin_lds_bytes(maxK, pl.max_kopt, pl.lin_copies, pl.mixed) > lin_room) pl.lin_copies = 1;
    if (!pl.waves || lin_lds_bytes(maxK, pl.max_kopt, pl.lin_copies, pl.mixed) > lin_room ||
        init_lds_bytes(maxK, maxn) + init_static_lds() > (size_t)ctx->max_lds)
        return set_error(ctx, LBA_ERR_UNSUPPORTED, "window of %d keyframes does not fit in LDS", maxK);
    pl.lin_lds = lin_lds_bytes(maxK, pl.max_kopt, pl.lin_copies, pl.mixed);
    pl.init_lds = init_lds_bytes(maxK, maxn);
    pl.upd_lds = upd_lds_bytes(maxK, maxn, pl.waves, pl.mixed);
    // the inertial measurements: per window their range, the joint reduced system
    pl.vi = I != nullptr;
    int64_t vred = 0, vdp = 0;
    if (pl.vi) {
        if (I->n_edges < 0) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "negative n_edges");
        if (I->n_edges > 0 &&
            (!I->edge_i || !I->edge_j || !I->dt || !I->dR || !I->dv || !I->dp || !I->J_Rg || !I->J_vg || !I->J_va ||
             !I->J_pg || !I->J_pa || !I->bg_bar || !I->ba_bar || !I->info || !I->info_bg || !I->info_ba))
            return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "an inertial measurement array is NULL");
        if (P->n_kf > 0 && (!I->v || !I->bg || !I->ba))
            return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "initial velocities / biases are NULL");
        for (int q = 0; q < 12; ++q)
            if (!std::isfinite(I->T_cb[q])) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "T_cb not finite");
        for (int q = 0; q < 3; ++q)
            if (!std::isfinite(I->g[q])) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "gravity not finite");
        if (B && !I->edge_off) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "edge_off is NULL for a batch");
        if (B) pl.edge_off.assign(I->edge_off, I->edge_off + nw + 1);
        else pl.edge_off = {0, I->n_edges};
        if (pl.edge_off[0] != 0 || pl.edge_off[nw] != I->n_edges)
            return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "edge offsets must start at 0 and end at n_edges");
        pl.edge_win.assign(std::max(I->n_edges, 1), 0);
        pl.vwin = pl.win;
        for (int w = 0; w < nw; ++w) {
            if (pl.edge_off[w + 1] < pl.edge_off[w])
                return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "edge offsets decrease at window %d", w);
            for (int e = pl.edge_off[w]; e < pl.edge_off[w + 1]; ++e) pl.edge_win[e] = w;
            WinInfo &V = pl.vwin[w];
            V.n = 15 * pl.win[w].Kopt;
            V.E = V.n * (V.n + 1) / 2;
            V.red_off = (int32_t)vred;
            vred += V.E + V.n;
            V.dp_off = (int32_t)vdp;
            vdp += V.n;
            maxn = std::max(maxn, V.n);
        }
        if (vred > INT32_MAX) return set_error(ctx, LBA_ERR_UNSUPPORTED, "batch too large");
    }
    // the reduced system is factored in LDS when it fits, else in a per-window copy in HBM
    // (systems of up to chol_reg_max_n() unknowns are factored with the matrix in registers
    // and static LDS only; larger ones in a per-window copy in HBM)
    pl.chol_hbm = maxn > chol_reg_max_n();
    pl.chol_lds = pl.chol_hbm ? chol_lds_bytes_hbm(maxn) : 0;
    if (pl.chol_lds + chol_static_lds() > (size_t)ctx->max_lds || (pl.chol_hbm && pl.vi))
        return set_error(ctx, LBA_ERR_UNSUPPORTED, "reduced system of %d unknowns does not fit in LDS", maxn);
    pl.lin_passes = lin_passes(pl.max_kopt);

    // workspace layout (plan records first: they are uploaded in one copy)
    size_t o = 0;
    pl.o_win = o;    o = align256(o + sizeof(WinInfo) * nw);
    pl.o_tiles = o;  o = align256(o + sizeof(Tile) * std::max<size_t>(pl.tiles.size(), 1));
    pl.o_order = o;  o = align256(o + sizeof(int32_t) * std::max<size_t>(pl.tiles.size(), 1));
    pl.o_opt = o;    o = align256(o + sizeof(int32_t) * std::max(P->n_kf, 1));
    pl.o_kfoff = o;  o = align256(o + sizeof(int32_t) * (nw + 1));
    pl.o_ptoff = o;  o = align256(o + sizeof(int32_t) * (nw + 1));
    pl.o_obsoff = o; o = align256(o + sizeof(int32_t) * (nw + 1));
    if (pl.vi) {
        pl.o_vwin = o;    o = align256(o + sizeof(WinInfo) * nw);
        pl.o_edgewin = o; o = align256(o + sizeof(int32_t) * pl.edge_win.size());
        pl.o_edgeoff = o; o = align256(o + sizeof(int32_t) * (nw + 1));
    }
    pl.o_upload_end = o;
    pl.o_ptstart = o; o = align256(o + sizeof(int32_t) * ((size_t)P->n_pt + 1));
    pl.o_ctl = o;     o = align256(o + sizeof(Ctl) * nw);
    pl.o_T = o;       o = align256(o + sizeof(double) * 12 * std::max(P->n_kf, 1));
    pl.o_X0 = o;      o = align256(o + sizeof(double) * 3 * std::max(P->n_pt, 1));
    pl.o_X1 = o;      o = align256(o + sizeof(double) * 3 * std::max(P->n_pt, 1));
    pl.o_part = o;    o = align256(o + sizeof(double) * pl.part_elems);
    pl.o_partr = o;   o = align256(o + sizeof(double) * pl.partr_elems);
    pl.o_partd = o;   o = align256(o + sizeof(double) * 4 * std::max<size_t>(pl.tiles.size(), 1));
    // the update splits each tile into parts of about 512 points (one block each): it
    // reads a tile's observations once, so smaller blocks balance the launch better
    {
        int max_tile = 1;
        for (const Tile &T : pl.tiles) max_tile = std::max(max_tile, T.p1 - T.p0);
        pl.upd_split = std::max(1, std::min(8, max_tile / 512));
    }
    pl.o_partu = o;   o = align256(o + sizeof(double) * 4 * pl.upd_split * std::max<size_t>(pl.tiles.size(), 1));
    pl.o_red = o;     o = align256(o + sizeof(double) * pl.red_elems);
    pl.o_fact = o;    o = align256(o + (pl.chol_hbm ? sizeof(double) * pl.red_elems : 0));
    pl.o_redflag = o; o = align256(o + sizeof(double) * nw);
    pl.o_dp = o;      o = align256(o + sizeof(double) * pl.dp_elems);
    pl.o_pf = o;      o = align256(o + sizeof(double) * 12 * std::max(P->n_pt, 1));
    pl.o_pkey = o;    o = align256(o + sizeof(uint16_t) * std::max(P->n_pt, 1));
    pl.o_ptmp = o;    o = align256(o + sizeof(int32_t) * std::max(P->n_pt, 1));
    pl.o_pinfo = o;   o = align256(o + sizeof(int4) * std::max(P->n_pt, 1));
    // the observations copied into the linearisation order
    const size_t nob = (size_t)std::max(P->n_obs, 1);
    pl.o_skf = o;     o = align256(o + sizeof(int32_t) * nob);
    pl.o_stype = o;   o = align256(o + nob);
    pl.o_soct = o;    o = align256(o + nob);
    pl.o_sz = o;      o = align256(o + 3 * nob * (P->obs_z_f32 ? sizeof(float) : sizeof(double)));
    pl.o_smask = o;   o = align256(o + nob);
    pl.o_stats = o;   o = align256(o + sizeof(double) * LBA_STATS_LEN * nw);
    pl.o_err = o;     o = align256(o + sizeof(int32_t) * 16);
    if (opt.trial_log < 0 || opt.trial_log > 4096)
        return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "trial_log must be in [0, 4096]");
    pl.log_cap = opt.trial_log;
    pl.o_log = o;     o = align256(o + sizeof(TrialRec) * (size_t)pl.log_cap * nw);
    // chunk records of the linearisation (kept for the rest of an LM round): about 3 words
    // per observation on the batched workload (pairs, piece starts) plus up to 243 per
    // chunk (header, piece offsets of the blocks); the pool is sized at 8 per observation
    // plus 256 per 256 observations and per tile and pass.  A tile whose records do not
    // fit forms them at every step instead.
    if (opt.pair_cache != 0 && opt.pair_cache != 1)
        return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "pair_cache must be 0 or 1");
    // one slot per block of the linearisation's grid (tiles x passes; a batch without
    // optimisable keyframes has no pass but still launches one row of blocks)
    const int64_t slots = (int64_t)std::max<size_t>(pl.tiles.size(), 1) * std::max(pl.lin_passes, 1);
    pl.plan_cap = opt.pair_cache ? 8 * (int64_t)P->n_obs + 256 * ((int64_t)P->n_obs / 256 + slots) : 0;
    pl.plan_cap = std::min<int64_t>(pl.plan_cap, INT32_MAX - 4);   // word offsets are 32-bit
    pl.o_planhead = o; o = align256(o + sizeof(int32_t) * slots);
    pl.o_planctr = o;  o = align256(o + sizeof(unsigned long long));
    pl.o_plan = o;     o = align256(o + sizeof(uint32_t) * (size_t)pl.plan_cap);
    if (pl.vi) {
        pl.o_vred = o;  o = align256(o + sizeof(double) * std::max<int64_t>(vred, 1));
        pl.o_vdp = o;   o = align256(o + sizeof(double) * std::max<int64_t>(vdp, 1));
        pl.o_state = o; o = align256(o + sizeof(double) * 9 * std::max(P->n_kf, 1));
        pl.o_ed = o;    o = align256(o + sizeof(double) * kViEdgeStride * std::max(I->n_edges, 1));
    }
    pl.total = o;
    return LBA_OK;
}

// the pinned staging buffer is reused by every call: wait until the copy that the
// previous call enqueued from it has been executed
lba_status wait_upload(lba_ctx *ctx) {
    if (ctx->upload_pending) {
        HIPCHK(hipEventSynchronize(ctx->upload_ev));
        ctx->upload_pending = false;
    }
    return LBA_OK;
}

lba_status record_upload(lba_ctx *ctx, hipStream_t s) {
    if (!ctx->upload_ev) HIPCHK(hipEventCreateWithFlags(&ctx->upload_ev, hipEventDisableTiming));
    HIPCHK(hipEventRecord(ctx->upload_ev, s));
    ctx->upload_pending = true;
    return LBA_OK;
}

lba_status ensure_pinned(lba_ctx *ctx, size_t bytes) {
    lba_status st = wait_upload(ctx);
    if (st != LBA_OK) return st;
    if (ctx->pinned_bytes >= bytes) return LBA_OK;
    if (ctx->pinned) HIPCHK(hipHostFree(ctx->pinned));
    ctx->pinned = nullptr;
    ctx->pinned_bytes = 0;
    size_t want = std::max<size_t>(bytes, 1 << 16);
    HIPCHK(hipHostMalloc(&ctx->pinned, want, hipHostMallocDefault));
    ctx->pinned_bytes = want;
    return LBA_OK;
}

struct DeviceGuard {
    int prev = -1;
    bool changed = false;
    hipError_t enter(int dev) {
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != dev) {
            changed = true;
            return hipSetDevice(dev);
        }
        return hipSuccess;
    }
    ~DeviceGuard() {
        if (changed) (void)hipSetDevice(prev);
    }
};

std::string describe_input_error(int32_t e) {
    std::string s;
    const char *names[] = {"observation keyframe index out of range", "observation point index out of range",
                           "octave >= n_levels", "observation type not 0/1",
                           "observations not grouped by point (obs_pt decreasing within a window)",
                           "non-finite measurement", "non-finite pose", "non-finite point",
                           "a point has more than 64 observations", "stereo observation with bf <= 0",
                           "inertial measurement invalid (keyframe outside its window or repeated, dt <= 0, or a "
                           "non-finite value) or non-finite initial velocity / bias"};
    for (int b = 0; b < 11; ++b)
        if (e & (1 << b)) {
            if (!s.empty()) s += "; ";
            s += names[b];
        }
    return s;
}

// Launch `fn` (returning hipError_t) as kernel class `cls`, bracketed by events when
// profiling is on.
template <typename Fn>
hipError_t timed(lba_ctx *ctx, int cls, hipStream_t s, Fn &&fn) {
    if (!ctx->prof) return fn();
    const size_t i = ctx->pending_cls.size();
    while (ctx->ev_pool.size() < 2 * (i + 1)) {
        hipEvent_t e;
        hipError_t err = hipEventCreate(&e);
        if (err != hipSuccess) return err;
        ctx->ev_pool.push_back(e);
    }
    hipError_t e = hipEventRecord(ctx->ev_pool[2 * i], s);
    if (e != hipSuccess) return e;
    e = fn();
    if (e != hipSuccess) return e;
    e = hipEventRecord(ctx->ev_pool[2 * i + 1], s);
    if (e != hipSuccess) return e;
    ctx->pending_cls.push_back(cls);
    return hipSuccess;
}

// fold the recorded event pairs into the counters (the stream has been synchronised)
hipError_t collect_timing(lba_ctx *ctx) {
    for (size_t i = 0; i < ctx->pending_cls.size(); ++i) {
        float ms = 0.0f;
        hipError_t e = hipEventElapsedTime(&ms, ctx->ev_pool[2 * i], ctx->ev_pool[2 * i + 1]);
        if (e != hipSuccess) return e;
        ctx->prof_ms[ctx->pending_cls[i]] += ms;
        ctx->prof_n[ctx->pending_cls[i]] += 1;
    }
    ctx->pending_cls.clear();
    return hipSuccess;
}

// executable graph of one LM step for the launch arguments `key`: captured from `step` on
// the context's private stream the first time (nothing runs during a capture) and kept in
// a cache of at most kGraphCache entries; the least recently used one makes room
template <typename Fn>
lba_status step_graph(lba_ctx *ctx, const std::string &key, Fn &&step, hipGraphExec_t *out) {
    auto &G = ctx->graphs;
    auto it = G.find(key);
    if (it != G.end()) {
        it->second.used = ++ctx->graph_clock;
        *out = it->second.exec;
        return LBA_OK;
    }
    if (!ctx->cap_stream) HIPCHK(hipStreamCreateWithFlags(&ctx->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal));
    const hipError_t le = step(ctx->cap_stream);
    const hipError_t ce = hipStreamEndCapture(ctx->cap_stream, &graph);
    if (le != hipSuccess || ce != hipSuccess) {
        if (graph) (void)hipGraphDestroy(graph);
        return set_error(ctx, LBA_ERR_HIP, "capture of the LM step failed: %s",
                         hipGetErrorString(le != hipSuccess ? le : ce));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ie = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (ie != hipSuccess) {
        (void)hipGraphDestroy(graph);
        return set_error(ctx, LBA_ERR_HIP, "hipGraphInstantiate failed: %s", hipGetErrorString(ie));
    }
    if (G.size() >= kGraphCache) {
        // every solve synchronises its stream before it returns, so only the current
        // solve's graphs (the most recently used) can still be pending
        auto old = G.begin();
        for (auto i = G.begin(); i != G.end(); ++i)
            if (i->second.used < old->second.used) old = i;
        (void)hipGraphExecDestroy(old->second.exec);
        (void)hipGraphDestroy(old->second.graph);
        G.erase(old);
    }
    G.emplace(key, lba_ctx::GraphEntry{graph, exec, ++ctx->graph_clock});
    *out = exec;
    return LBA_OK;
}

lba_status solve_impl(lba_ctx *ctx, const lba_problem *P, const lba_batch *B, lba_result *R, void *ws,
                      size_t ws_bytes, void *stream_ptr, const lba_inertial *I = nullptr, double *v_out = nullptr,
                      double *bg_out = nullptr, double *ba_out = nullptr) {
    if (!ctx) return LBA_ERR_INVALID_ARGUMENT;
    ctx->err.clear();
    if (!R) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "result is NULL");
    Plan pl;
    lba_status st = build_plan(ctx, P, B, pl, I);
    if (st != LBA_OK) return st;
    if (I && P->n_kf > 0 && (!v_out || !bg_out || !ba_out))
        return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "v_out / bg_out / ba_out is NULL");
    if (P->n_kf > 0 && !R->T_out) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "T_out is NULL");
    if (P->n_pt > 0 && !R->X_out) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "X_out is NULL");
    if (P->n_obs > 0 && !R->outlier) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "outlier is NULL");
    if (!ws || ws_bytes < pl.total)
        return set_error(ctx, LBA_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes given, %zu needed", ws_bytes,
                         pl.total);
    if (((uintptr_t)ws) & 255) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "workspace not 256-byte aligned");
    const lba_options &opt = ctx->opt;
    if (opt.iters_round1 < 0 || opt.iters_round2 < 0 || opt.max_trials < 1)
        return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "invalid iteration counts");

    DeviceGuard dg;
    HIPCHK(dg.enter(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream_ptr);
    unsigned char *wsb = static_cast<unsigned char *>(ws);
    const int nw = pl.nw;

    // ---- upload the plan ------------------------------------------------------------
    const size_t down_bytes = std::max(sizeof(Ctl) * nw, sizeof(double) * LBA_STATS_LEN * nw) + 256;
    st = ensure_pinned(ctx, pl.o_upload_end + down_bytes);
    if (st != LBA_OK) return st;
    unsigned char *up = static_cast<unsigned char *>(ctx->pinned);
    unsigned char *down = up + pl.o_upload_end;
    memcpy(up + pl.o_win, pl.win.data(), sizeof(WinInfo) * nw);
    if (!pl.tiles.empty()) {
        memcpy(up + pl.o_tiles, pl.tiles.data(), sizeof(Tile) * pl.tiles.size());
        memcpy(up + pl.o_order, pl.order.data(), sizeof(int32_t) * pl.order.size());
    }
    if (P->n_kf > 0) memcpy(up + pl.o_opt, pl.opt_map.data(), sizeof(int32_t) * P->n_kf);
    memcpy(up + pl.o_kfoff, pl.kf_off.data(), sizeof(int32_t) * (nw + 1));
    memcpy(up + pl.o_ptoff, pl.pt_off.data(), sizeof(int32_t) * (nw + 1));
    memcpy(up + pl.o_obsoff, pl.obs_off.data(), sizeof(int32_t) * (nw + 1));
    if (pl.vi) {
        memcpy(up + pl.o_vwin, pl.vwin.data(), sizeof(WinInfo) * nw);
        memcpy(up + pl.o_edgewin, pl.edge_win.data(), sizeof(int32_t) * pl.edge_win.size());
        memcpy(up + pl.o_edgeoff, pl.edge_off.data(), sizeof(int32_t) * (nw + 1));
    }
    HIPCHK(hipMemcpyAsync(wsb, up, pl.o_upload_end, hipMemcpyHostToDevice, s));
    st = record_upload(ctx, s);
    if (st != LBA_OK) return st;

    // ---- constants and argument packs ----------------------------------------------------
    SolveConsts c;
    memset(&c, 0, sizeof(c));
    c.cam = {P->cam.fx, P->cam.fy, P->cam.cx, P->cam.cy, P->cam.bf};
    c.huber2[0] = opt.huber2_mono;
    c.huber2[1] = opt.huber2_stereo;
    c.chi2[0] = opt.chi2_mono;
    c.chi2[1] = opt.chi2_stereo;
    c.tau = opt.tau;
    for (int i = 0; i < P->n_levels; ++i) c.inv_sigma2[i] = 1.0 / P->sigma2[i];
    c.iters[0] = opt.iters_round1;
    c.iters[1] = opt.iters_round2;
    c.max_trials = opt.max_trials;
    c.n_windows = nw;

    auto W_ = [&](size_t off) { return reinterpret_cast<void *>(wsb + off); };
    const WinInfo *d_win = static_cast<const WinInfo *>(W_(pl.o_win));
    const Tile *d_tiles = static_cast<const Tile *>(W_(pl.o_tiles));
    const int32_t *d_opt = static_cast<const int32_t *>(W_(pl.o_opt));
    int32_t *d_ptstart = static_cast<int32_t *>(W_(pl.o_ptstart));
    Ctl *d_ctl = static_cast<Ctl *>(W_(pl.o_ctl));
    double *d_T = static_cast<double *>(W_(pl.o_T));
    double *d_X0 = static_cast<double *>(W_(pl.o_X0));
    double *d_X1 = static_cast<double *>(W_(pl.o_X1));
    double *d_partd = static_cast<double *>(W_(pl.o_partd));
    double *d_partu = static_cast<double *>(W_(pl.o_partu));
    double *d_red = static_cast<double *>(W_(pl.o_red));
    double *d_redflag = static_cast<double *>(W_(pl.o_redflag));
    double *d_dp = static_cast<double *>(W_(pl.o_dp));
    double *d_stats = static_cast<double *>(W_(pl.o_stats));
    int32_t *d_err = static_cast<int32_t *>(W_(pl.o_err));

    ObsView ob;
    ob.kf = P->obs_kf;
    ob.pt = P->obs_pt;
    ob.z = P->obs_z;
    ob.type = P->obs_type;
    ob.oct = P->obs_oct;
    ob.n_obs = P->n_obs;
    ob.z_f32 = P->obs_z_f32 ? 1 : 0;

    MiscArgs m;
    memset(&m, 0, sizeof(m));
    m.win = d_win;
    m.kf_off_dev = static_cast<const int32_t *>(W_(pl.o_kfoff));
    m.pt_off_dev = static_cast<const int32_t *>(W_(pl.o_ptoff));
    m.obs_off_dev = static_cast<const int32_t *>(W_(pl.o_obsoff));
    m.T_in = P->T_cw;
    m.X_in = P->X_w;
    m.T = d_T;
    m.X0 = d_X0;
    m.X1 = d_X1;
    m.ctl = d_ctl;
    m.pt_start = d_ptstart;
    m.obs = ob;
    m.flags = R->outlier;
    m.T_out = R->T_out;
    m.X_out = R->X_out;
    m.stats = d_stats;
    m.err = d_err;
    m.n_kf = P->n_kf;
    m.n_pt = P->n_pt;
    m.n_levels = P->n_levels;
    m.c = c;

    // the inertial measurements (stereo-inertial solve)
    ViArgs va;
    memset(&va, 0, sizeof(va));
    if (pl.vi) {
        va.E = {I->edge_i, I->edge_j, I->dt, I->dR, I->dv, I->dp, I->J_Rg, I->J_vg, I->J_va, I->J_pg, I->J_pa,
                I->bg_bar, I->ba_bar, I->info, I->info_bg, I->info_ba, I->n_edges, 0};
        va.win = d_win;
        va.vwin = static_cast<const WinInfo *>(W_(pl.o_vwin));
        va.edge_win = static_cast<const int32_t *>(W_(pl.o_edgewin));
        va.edge_off = static_cast<const int32_t *>(W_(pl.o_edgeoff));
        va.opt_map = static_cast<const int32_t *>(W_(pl.o_opt));
        va.ctl = d_ctl;
        va.T = d_T;
        va.state = static_cast<double *>(W_(pl.o_state));
        va.v0 = I->v;
        va.bg0 = I->bg;
        va.ba0 = I->ba;
        va.v_out = v_out;
        va.bg_out = bg_out;
        va.ba_out = ba_out;
        va.dp = d_dp;
        va.dpv = d_dp;
        va.vdp = static_cast<double *>(W_(pl.o_vdp));
        va.red = d_red;
        va.vred = static_cast<double *>(W_(pl.o_vred));
        va.ed = static_cast<double *>(W_(pl.o_ed));
        va.err = d_err;
        for (int q = 0; q < 12; ++q) va.Tcb[q] = I->T_cb[q];
        for (int q = 0; q < 3; ++q) va.g[q] = I->g[q];
        va.n_kf = P->n_kf;
    }
    ViArgs va_trial = va;
    va_trial.trial = 1;

    HIPCHK(timed(ctx, LBA_KCLASS_SETUP, s, [&] { return launch_setup(m, nw, s); }));
    HIPCHK(timed(ctx, LBA_KCLASS_VALIDATE, s, [&] { return launch_validate(m, nw, pl.max_obs, s); }));
    if (pl.vi) {
        HIPCHK(timed(ctx, LBA_KCLASS_VALIDATE, s, [&] { return launch_vi_check(va, s); }));
        HIPCHK(timed(ctx, LBA_KCLASS_SETUP, s, [&] { return launch_vi_setup(va, s); }));
    }
    HIPCHK(hipMemcpyAsync(down, d_err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    int32_t in_err;
    memcpy(&in_err, down, sizeof(int32_t));
    HIPCHK(collect_timing(ctx));
    if (in_err) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "invalid input: %s", describe_input_error(in_err).c_str());

    // point order of the linearisation (the observation structure is fixed for the solve),
    // and the observations copied into it
    int4 *d_pinfo = static_cast<int4 *>(W_(pl.o_pinfo));
    ObsView sob = ob;
    sob.pt = nullptr;
    sob.kf = static_cast<const int32_t *>(W_(pl.o_skf));
    sob.type = static_cast<const uint8_t *>(W_(pl.o_stype));
    sob.oct = static_cast<const uint8_t *>(W_(pl.o_soct));
    sob.z = W_(pl.o_sz);
    OrderArgs oa;
    memset(&oa, 0, sizeof(oa));
    {
        oa.win = d_win;
        oa.pt_start = d_ptstart;
        oa.opt_map = d_opt;
        oa.obs_kf = P->obs_kf;
        oa.keys = static_cast<uint16_t *>(W_(pl.o_pkey));
        oa.tmp = static_cast<int32_t *>(W_(pl.o_ptmp));
        oa.pinfo = d_pinfo;
        oa.by_keyframes = 1;
        oa.n_pt = P->n_pt;
        oa.obs = ob;
        oa.sobs_kf = static_cast<int32_t *>(W_(pl.o_skf));
        oa.sobs_type = static_cast<uint8_t *>(W_(pl.o_stype));
        oa.sobs_oct = static_cast<uint8_t *>(W_(pl.o_soct));
        oa.sobs_z = W_(pl.o_sz);
        oa.smask = static_cast<uint8_t *>(W_(pl.o_smask));
        HIPCHK(timed(ctx, LBA_KCLASS_ORDER, s, [&] {
            hipError_t e = launch_order(oa, nw, pl.max_pts, pl.max_kopt, s);
            return e != hipSuccess ? e : launch_order_gather(oa, false, s);
        }));
    }

    const int ntiles = (int)pl.tiles.size();
    LinArgs la;
    memset(&la, 0, sizeof(la));
    la.win = d_win;
    la.tiles = d_tiles;
    la.order = static_cast<const int32_t *>(W_(pl.o_order));
    la.opt_map = d_opt;
    la.pt_start = d_ptstart;
    la.pinfo = d_pinfo;
    la.sobs = sob;
    la.T = d_T;
    la.X0 = d_X0;
    la.X1 = d_X1;
    la.ctl = d_ctl;
    la.obs = ob;
    la.part = static_cast<double *>(W_(pl.o_part));
    la.partr = static_cast<double *>(W_(pl.o_partr));
    la.partd = d_partd;
    la.pf = static_cast<double *>(W_(pl.o_pf));
    la.waves = pl.waves;
    la.acc32 = (pl.mixed && opt.schur_fp32_accum) ? 1 : 0;
    la.self_copies = pl.lin_copies;
    if (pl.plan_cap > 0) {
        la.plan = static_cast<uint32_t *>(W_(pl.o_plan));
        la.plan_ctr = static_cast<unsigned long long *>(W_(pl.o_planctr));
        la.plan_head = static_cast<int32_t *>(W_(pl.o_planhead));
        la.plan_cap = pl.plan_cap;
    }
    la.c = c;

    ReduceArgs ra;
    memset(&ra, 0, sizeof(ra));
    ra.win = d_win;
    ra.ctl = d_ctl;
    ra.part = static_cast<const double *>(W_(pl.o_part));
    ra.partr = static_cast<const double *>(W_(pl.o_partr));
    ra.partd = d_partd;
    ra.red = d_red;
    ra.redflag = d_redflag;
    ra.max_En = pl.max_En;

    CholArgs ca;
    memset(&ca, 0, sizeof(ca));
    ca.win = d_win;
    ca.ctl = d_ctl;
    ca.red = d_red;
    ca.redflag = d_redflag;
    ca.dp = d_dp;
    ca.fact = pl.chol_hbm ? static_cast<double *>(W_(pl.o_fact)) : nullptr;
    if (pl.vi) {   // the joint reduced system of 15 Kopt unknowns per window
        ca.win = va.vwin;
        ca.red = va.vred;
        ca.dp = static_cast<double *>(W_(pl.o_vdp));
    }

    UpdArgs ua;
    memset(&ua, 0, sizeof(ua));
    ua.win = d_win;
    ua.tiles = d_tiles;
    ua.order = static_cast<const int32_t *>(W_(pl.o_order));
    ua.opt_map = d_opt;
    ua.pt_start = d_ptstart;
    ua.T = d_T;
    ua.X0 = d_X0;
    ua.X1 = d_X1;
    ua.ctl = d_ctl;
    ua.dp = d_dp;
    ua.obs = ob;
    ua.partu = d_partu;
    ua.split = pl.upd_split;
    ua.pf = static_cast<const double *>(W_(pl.o_pf));
    ua.waves = pl.waves;
    ua.c = c;

    DecideArgs da;
    memset(&da, 0, sizeof(da));
    da.win = d_win;
    da.ctl = d_ctl;
    da.opt_map = d_opt;
    da.T = d_T;
    da.dp = d_dp;
    da.partu = d_partu;
    da.log = pl.log_cap > 0 ? static_cast<TrialRec *>(W_(pl.o_log)) : nullptr;
    da.log_cap = pl.log_cap;
    da.split = pl.upd_split;
    da.c = c;
    if (pl.vi) {
        da.vi_ed = va.ed;
        da.vi_edge_off = va.edge_off;
        da.vi_dp = va.vdp;
        da.vi_win = va.vwin;
        da.vi_state = va.state;
    }

    InitReduceArgs ia;
    memset(&ia, 0, sizeof(ia));
    ia.win = d_win;
    ia.ctl = d_ctl;
    ia.partr = static_cast<const double *>(W_(pl.o_partr));
    ia.partd = d_partd;
    ia.c = c;
    if (pl.vi) {
        ia.vi_ed = va.ed;
        ia.vi_edge_off = va.edge_off;
        ia.vi_ei = I->edge_i;
        ia.vi_ej = I->edge_j;
        ia.opt_map = va.opt_map;
    }

    std::vector<Ctl> hctl(nw);
    for (int round = 1; round <= 2; ++round) {
        const int iters = round == 1 ? opt.iters_round1 : opt.iters_round2;
        const uint8_t *mask = nullptr;
        if (round == 2) {
            m.count = 0;
            oa.mask = R->outlier;
            HIPCHK(timed(ctx, LBA_KCLASS_FLAGS, s, [&] {
                hipError_t e = launch_flags(m, nw, pl.max_obs, s);
                return e != hipSuccess ? e : launch_order_gather(oa, true, s);   // the flags in places
            }));
            mask = R->outlier;
        }
        const int robust = round == 1 ? 1 : (opt.round2_robust ? 1 : 0);
        la.mask = mask;
        la.smask = mask ? oa.smask : nullptr;
        la.robust = robust;
        ua.mask = mask;
        ua.robust = robust;
        da.round = round;
        ia.round = round;
        // the active observations change between rounds: the chunk records are formed again
        HIPCHK(timed(ctx, LBA_KCLASS_LINEARIZE_INIT, s, [&] {
            hipError_t e = launch_plan_reset(la, ntiles * std::max(pl.lin_passes, 1), s);
            return e != hipSuccess ? e : launch_init(la, ntiles, pl.init_lds, s);
        }));
        if (pl.vi) HIPCHK(timed(ctx, LBA_KCLASS_INERTIAL, s, [&] { return launch_vi_eval(va, s); }));
        HIPCHK(timed(ctx, LBA_KCLASS_INIT_REDUCE, s, [&] { return launch_init_reduce(ia, nw, s); }));
        int steps_done = 0;
        int nsteps = iters;
        const int max_steps = iters * opt.max_trials;
        // one LM step over every window: [linearise, reduce, factor + solve, update, decide]
        auto step = [&](hipStream_t q) -> hipError_t {
            hipError_t e;
            if ((e = timed(ctx, LBA_KCLASS_LINEARIZE, q,
                           [&] { return launch_linearize(la, ntiles, pl.lin_passes, pl.lin_lds, pl.mixed, q); })) != hipSuccess)
                return e;
            if ((e = timed(ctx, LBA_KCLASS_REDUCE, q, [&] { return launch_reduce(ra, nw, q); })) != hipSuccess) return e;
            if (pl.vi) {
                if ((e = timed(ctx, LBA_KCLASS_INERTIAL, q, [&] { return launch_vi_eval(va, q); })) != hipSuccess) return e;
                if ((e = timed(ctx, LBA_KCLASS_INERTIAL, q, [&] { return launch_vi_system(va, nw, q); })) != hipSuccess)
                    return e;
            }
            if ((e = timed(ctx, LBA_KCLASS_CHOLESKY, q, [&] { return launch_cholesky(ca, nw, pl.chol_lds, q); })) !=
                hipSuccess)
                return e;
            if (pl.vi && (e = timed(ctx, LBA_KCLASS_INERTIAL, q, [&] { return launch_vi_split(va, nw, q); })) != hipSuccess)
                return e;
            if ((e = timed(ctx, LBA_KCLASS_UPDATE, q,
                           [&] { return launch_update(ua, ntiles, pl.upd_lds, pl.mixed, q); })) != hipSuccess)
                return e;
            if (pl.vi && (e = timed(ctx, LBA_KCLASS_INERTIAL, q, [&] { return launch_vi_eval(va_trial, q); })) !=
                             hipSuccess)
                return e;
            return timed(ctx, LBA_KCLASS_DECIDE, q, [&] { return launch_decide(da, nw, q); });
        };
        hipGraphExec_t exec = nullptr;
        if (opt.use_graphs && !ctx->prof && iters > 0) {
            std::string key;
            auto add = [&](const void *p, size_t n) { key.append(static_cast<const char *>(p), n); };
            add(&la, sizeof(la));
            add(&ra, sizeof(ra));
            add(&ca, sizeof(ca));
            add(&ua, sizeof(ua));
            add(&da, sizeof(da));
            add(&va, sizeof(va));
            const int64_t dims[6] = {ntiles, nw, (int64_t)pl.lin_lds, (int64_t)pl.chol_lds, (int64_t)pl.upd_lds,
                                     pl.mixed ? 1 : 0};
            add(dims, sizeof(dims));
            st = step_graph(ctx, key, step, &exec);
            if (st != LBA_OK) return st;
        }
        while (nsteps > 0 && steps_done < max_steps) {
            for (int k = 0; k < nsteps; ++k) {
                if (exec) HIPCHK(hipGraphLaunch(exec, s));
                else HIPCHK(step(s));
            }
            steps_done += nsteps;
            HIPCHK(hipMemcpyAsync(down, d_ctl, sizeof(Ctl) * nw, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            memcpy(hctl.data(), down, sizeof(Ctl) * nw);
            int need = 0;
            for (int w = 0; w < nw; ++w)
                if (hctl[w].running) need = std::max(need, std::max(1, iters - hctl[w].iter));
            nsteps = std::min(need, max_steps - steps_done);
        }
    }
    m.count = 1;
    HIPCHK(timed(ctx, LBA_KCLASS_FLAGS, s, [&] { return launch_flags(m, nw, pl.max_obs, s); }));
    HIPCHK(timed(ctx, LBA_KCLASS_FINALIZE, s, [&] { return launch_finalize(m, nw, s); }));
    if (pl.vi) HIPCHK(timed(ctx, LBA_KCLASS_FINALIZE, s, [&] { return launch_vi_finish(va, s); }));
    if (R->log && pl.log_cap > 0)
        HIPCHK(hipMemcpyAsync(R->log, W_(pl.o_log), sizeof(TrialRec) * (size_t)pl.log_cap * nw,
                              hipMemcpyDeviceToHost, s));
    if (R->stats) {
        HIPCHK(hipMemcpyAsync(down, d_stats, sizeof(double) * LBA_STATS_LEN * nw, hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        memcpy(R->stats, down, sizeof(double) * LBA_STATS_LEN * nw);
    } else {
        HIPCHK(hipStreamSynchronize(s));
    }
    HIPCHK(collect_timing(ctx));
    return LBA_OK;
}


// ------------------------------------------------------------------------------------
// differentiation form
// ------------------------------------------------------------------------------------
struct CostPlan {
    int nw = 0;
    int64_t max_obs = 0;
    int maxK = 0;
    std::vector<CostWin> win;
    std::vector<Tile> tiles;
    std::vector<int32_t> kf_off, pt_off, obs_off;
    size_t o_win, o_tiles, o_kfoff, o_ptoff, o_obsoff, o_upload_end, o_ptstart, o_partF, o_partG, o_pf, o_err,
        total;
};

lba_status build_cost_plan(lba_ctx *ctx, const lba_problem *P, const lba_batch *B, CostPlan &cp) {
    if (!P) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "problem is NULL");
    if (P->n_kf < 0 || P->n_pt < 0 || P->n_obs < 0)
        return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "negative size");
    if (P->n_levels < 1 || P->n_levels > kMaxLevels)
        return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "n_levels must be in [1, %d]", kMaxLevels);
    if (!P->sigma2) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "sigma2 (host) is NULL");
    for (int i = 0; i < P->n_levels; ++i)
        if (!(P->sigma2[i] > 0.0) || !std::isfinite(P->sigma2[i]))
            return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "sigma2[%d] must be positive", i);
    if (P->n_kf > 0 && !P->T_cw) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "T_cw is NULL");
    if (P->n_obs > 0 && (!P->obs_kf || !P->obs_pt || !P->obs_type || !P->obs_oct))
        return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "an observation array is NULL");
    if (!(P->cam.fx > 0.0) || !(P->cam.fy > 0.0) || !std::isfinite(P->cam.cx) ||
        !std::isfinite(P->cam.cy) || !std::isfinite(P->cam.bf))
        return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "invalid intrinsics");
    if (B) {
        if (B->n_windows < 1 || !B->kf_off || !B->pt_off || !B->obs_off)
            return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "invalid batch description");
        cp.nw = B->n_windows;
        cp.kf_off.assign(B->kf_off, B->kf_off + cp.nw + 1);
        cp.pt_off.assign(B->pt_off, B->pt_off + cp.nw + 1);
        cp.obs_off.assign(B->obs_off, B->obs_off + cp.nw + 1);
    } else {
        cp.nw = 1;
        cp.kf_off = {0, P->n_kf};
        cp.pt_off = {0, P->n_pt};
        cp.obs_off = {0, P->n_obs};
    }
    const int nw = cp.nw;
    if (cp.kf_off[0] != 0 || cp.pt_off[0] != 0 || cp.obs_off[0] != 0 || cp.kf_off[nw] != P->n_kf ||
        cp.pt_off[nw] != P->n_pt || cp.obs_off[nw] != P->n_obs)
        return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "batch offsets must start at 0 and end at the totals");
    const int ppt = choose_cost_points_per_tile(ctx->opt, P->n_pt, P->n_obs);
    int64_t g = 0;
    cp.win.resize(nw);
    cp.tiles.clear();
    for (int w = 0; w < nw; ++w) {
        CostWin &W = cp.win[w];
        W.kf0 = cp.kf_off[w];
        W.K = cp.kf_off[w + 1] - cp.kf_off[w];
        W.pt0 = cp.pt_off[w];
        W.M = cp.pt_off[w + 1] - cp.pt_off[w];
        W.ob0 = cp.obs_off[w];
        W.N = cp.obs_off[w + 1] - cp.obs_off[w];
        if (W.K < 0 || W.M < 0 || W.N < 0)
            return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "batch offsets decrease at window %d", w);
        if (W.K > kMaxKf)
            return set_error(ctx, LBA_ERR_UNSUPPORTED, "window %d has %d keyframes (at most %d)", w, W.K, kMaxKf);
        if (W.N > 0 && (W.M == 0 || W.K == 0))
            return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "window %d has observations but no points or keyframes", w);
        W.tile0 = (int)cp.tiles.size();
        W.ntiles = (W.M + ppt - 1) / ppt;
        for (int t = 0; t < W.ntiles; ++t) {
            Tile T;
            T.win = w;
            T.p0 = W.pt0 + t * ppt;
            T.p1 = W.pt0 + std::min(W.M, (t + 1) * ppt);
            T.pad = 0;
            cp.tiles.push_back(T);
        }
        W.g_off = g;
        cp.max_obs = std::max<int64_t>(cp.max_obs, W.N);
        g += (int64_t)W.ntiles * W.K * 6;
        cp.maxK = std::max(cp.maxK, W.K);
    }
    size_t o = 0;
    cp.o_win = o;    o = align256(o + sizeof(CostWin) * nw);
    cp.o_tiles = o;  o = align256(o + sizeof(Tile) * std::max<size_t>(cp.tiles.size(), 1));
    cp.o_kfoff = o;  o = align256(o + sizeof(int32_t) * (nw + 1));
    cp.o_ptoff = o;  o = align256(o + sizeof(int32_t) * (nw + 1));
    cp.o_obsoff = o; o = align256(o + sizeof(int32_t) * (nw + 1));
    cp.o_upload_end = o;
    cp.o_ptstart = o; o = align256(o + sizeof(int32_t) * ((size_t)P->n_pt + 1));
    cp.o_partF = o;   o = align256(o + sizeof(double) * std::max<size_t>(cp.tiles.size(), 1));
    cp.o_partG = o;   o = align256(o + sizeof(double) * std::max<int64_t>(g, 1));
    cp.o_pf = o;      o = align256(o + sizeof(float) * 12 * std::max<size_t>((size_t)P->n_kf, 1));
    cp.o_err = o;     o = align256(o + sizeof(int32_t) * 16);
    cp.total = o;
    return LBA_OK;
}

lba_status cost_impl(lba_ctx *ctx, const lba_problem *P, const lba_batch *B, bool bwd, const float *xi,
                     const float *X, const float *z, const uint8_t *mask, const double *grad_cost, double *cost,
                     float *g_xi, float *g_X, float *g_z, void *ws, size_t ws_bytes, void *stream_ptr) {
    if (!ctx) return LBA_ERR_INVALID_ARGUMENT;
    ctx->err.clear();
    CostPlan cp;
    lba_status st = build_cost_plan(ctx, P, B, cp);
    if (st != LBA_OK) return st;
    if (P->n_pt > 0 && !X) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "X is NULL");
    if (P->n_obs > 0 && !z) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "z is NULL");
    if (!bwd && !cost) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "cost is NULL");
    if (bwd) {
        if (!grad_cost) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "grad_cost is NULL");
        if ((P->n_kf > 0 && !g_xi) || (P->n_pt > 0 && !g_X) || (P->n_obs > 0 && !g_z))
            return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "a gradient output is NULL");
    }
    if (!ws || ws_bytes < cp.total)
        return set_error(ctx, LBA_ERR_WORKSPACE_TOO_SMALL, "workspace of %zu bytes given, %zu needed", ws_bytes,
                         cp.total);
    if (((uintptr_t)ws) & 255) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "workspace not 256-byte aligned");
    if (cost_lds_bytes(cp.maxK, bwd) + cost_static_lds() > (size_t)ctx->max_lds)
        return set_error(ctx, LBA_ERR_UNSUPPORTED, "window of %d keyframes does not fit in LDS", cp.maxK);

    DeviceGuard dg;
    HIPCHK(dg.enter(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream_ptr);
    unsigned char *wsb = static_cast<unsigned char *>(ws);
    const int nw = cp.nw;

    st = ensure_pinned(ctx, cp.o_upload_end + 256);
    if (st != LBA_OK) return st;
    unsigned char *up = static_cast<unsigned char *>(ctx->pinned);
    unsigned char *down = up + cp.o_upload_end;
    memcpy(up + cp.o_win, cp.win.data(), sizeof(CostWin) * nw);
    if (!cp.tiles.empty()) memcpy(up + cp.o_tiles, cp.tiles.data(), sizeof(Tile) * cp.tiles.size());
    memcpy(up + cp.o_kfoff, cp.kf_off.data(), sizeof(int32_t) * (nw + 1));
    memcpy(up + cp.o_ptoff, cp.pt_off.data(), sizeof(int32_t) * (nw + 1));
    memcpy(up + cp.o_obsoff, cp.obs_off.data(), sizeof(int32_t) * (nw + 1));
    HIPCHK(hipMemcpyAsync(wsb, up, cp.o_upload_end, hipMemcpyHostToDevice, s));
    st = record_upload(ctx, s);
    if (st != LBA_OK) return st;

    auto W_ = [&](size_t off) { return reinterpret_cast<void *>(wsb + off); };
    int32_t *d_ptstart = static_cast<int32_t *>(W_(cp.o_ptstart));
    int32_t *d_err = static_cast<int32_t *>(W_(cp.o_err));

    ObsView ob;
    ob.kf = P->obs_kf;
    ob.pt = P->obs_pt;
    ob.z = z;
    ob.type = P->obs_type;
    ob.oct = P->obs_oct;
    ob.n_obs = P->n_obs;
    ob.z_f32 = 1;

    MiscArgs m;
    memset(&m, 0, sizeof(m));
    m.kf_off_dev = static_cast<const int32_t *>(W_(cp.o_kfoff));
    m.pt_off_dev = static_cast<const int32_t *>(W_(cp.o_ptoff));
    m.obs_off_dev = static_cast<const int32_t *>(W_(cp.o_obsoff));
    m.T_in = P->T_cw;
    m.pt_start = d_ptstart;
    m.obs = ob;
    m.err = d_err;
    m.n_kf = P->n_kf;
    m.n_pt = P->n_pt;
    m.n_levels = P->n_levels;
    m.c.cam = {P->cam.fx, P->cam.fy, P->cam.cx, P->cam.cy, P->cam.bf};
    m.c.n_windows = nw;
    m.xi = xi;
    m.Pf = static_cast<float *>(W_(cp.o_pf));

    HIPCHK(timed(ctx, LBA_KCLASS_SETUP, s, [&] { return launch_setup(m, nw, s); }));
    if (ctx->opt.check_inputs) {
        HIPCHK(timed(ctx, LBA_KCLASS_VALIDATE, s, [&] { return launch_validate(m, nw, cp.max_obs, s); }));
        HIPCHK(hipMemcpyAsync(down, d_err, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        int32_t in_err;
        memcpy(&in_err, down, sizeof(int32_t));
        if (in_err)
            return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "invalid input: %s", describe_input_error(in_err).c_str());
    }

    CostArgs ca;
    memset(&ca, 0, sizeof(ca));
    ca.win = static_cast<const CostWin *>(W_(cp.o_win));
    ca.tiles = static_cast<const Tile *>(W_(cp.o_tiles));
    ca.pt_start = d_ptstart;
    ca.T = P->T_cw;
    ca.xi = xi;
    ca.Pf = m.Pf;
    ca.X = X;
    ca.z = z;
    ca.obs_kf = P->obs_kf;
    ca.obs_pt = P->obs_pt;
    ca.obs_type = P->obs_type;
    ca.obs_oct = P->obs_oct;
    ca.mask = mask;
    ca.grad_cost = grad_cost;
    ca.g_xi = g_xi;
    ca.g_X = g_X;
    ca.g_z = g_z;
    ca.cost = cost;
    ca.partF = static_cast<double *>(W_(cp.o_partF));
    ca.partG = static_cast<double *>(W_(cp.o_partG));
    ca.err = d_err + 1;
    ca.n_obs = P->n_obs;
    ca.cam = m.c.cam;
    ca.huber2[0] = ctx->opt.huber2_mono;
    ca.huber2[1] = ctx->opt.huber2_stereo;
    for (int i = 0; i < P->n_levels; ++i) ca.inv_sigma2[i] = 1.0 / P->sigma2[i];
    const int ntiles = (int)cp.tiles.size();
    const int cls = bwd ? LBA_KCLASS_COST_BACKWARD : LBA_KCLASS_COST_FORWARD;
    HIPCHK(timed(ctx, cls, s, [&] { return launch_cost(ca, ntiles, cp.maxK, bwd, s); }));
    HIPCHK(launch_cost_reduce(ca, nw, bwd, s));
    if (ctx->prof) {
        HIPCHK(hipStreamSynchronize(s));
        HIPCHK(collect_timing(ctx));
    }
    return LBA_OK;
}

}  // namespace

extern "C" {

int32_t lba_abi_version(void) { return LBA_ABI_VERSION; }

const char *lba_status_string(lba_status status) {
    switch (status) {
        case LBA_OK: return "ok";
        case LBA_ERR_INVALID_ARGUMENT: return "invalid argument";
        case LBA_ERR_OUT_OF_MEMORY: return "out of memory";
        case LBA_ERR_HIP: return "HIP runtime error";
        case LBA_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case LBA_ERR_UNSUPPORTED: return "unsupported problem size";
    }
    return "unknown status";
}

void lba_default_options(lba_options *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->precision = LBA_PREC_FP64;
    o->iters_round1 = 5;
    o->iters_round2 = 10;
    o->max_trials = 10;
    o->round2_robust = 1;
    o->check_inputs = 1;
    o->huber2_mono = 5.991;
    o->huber2_stereo = 7.815;
    o->chi2_mono = 5.991;
    o->chi2_stereo = 7.815;
    o->tau = 1e-5;
    o->points_per_tile = 0;
    o->use_graphs = 1;
    o->pair_cache = 1;
}

lba_status lba_create(const lba_options *opt, int32_t device, lba_ctx **out) {
    if (!out) return LBA_ERR_INVALID_ARGUMENT;
    *out = nullptr;
    lba_ctx *ctx = new (std::nothrow) lba_ctx();
    if (!ctx) return LBA_ERR_OUT_OF_MEMORY;
    if (opt) ctx->opt = *opt;
    else lba_default_options(&ctx->opt);
    ctx->device = device;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        delete ctx;
        return LBA_ERR_INVALID_ARGUMENT;
    }
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
        ctx->max_lds = lds;
    *out = ctx;
    return LBA_OK;
}

void lba_destroy(lba_ctx *ctx) {
    if (!ctx) return;
    if (ctx->upload_pending) (void)hipEventSynchronize(ctx->upload_ev);
    for (auto &g : ctx->graphs) {
        (void)hipGraphExecDestroy(g.second.exec);
        (void)hipGraphDestroy(g.second.graph);
    }
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    if (ctx->upload_ev) (void)hipEventDestroy(ctx->upload_ev);
    if (ctx->pinned) (void)hipHostFree(ctx->pinned);
    for (hipEvent_t e : ctx->ev_pool) (void)hipEventDestroy(e);
    delete ctx;
}

lba_status lba_profile_enable(lba_ctx *ctx, int32_t enable) {
    if (!ctx) return LBA_ERR_INVALID_ARGUMENT;
    ctx->prof = enable != 0;
    ctx->pending_cls.clear();
    for (int i = 0; i < LBA_KCLASS_COUNT; ++i) {
        ctx->prof_ms[i] = 0.0;
        ctx->prof_n[i] = 0;
    }
    return LBA_OK;
}

lba_status lba_profile_read(const lba_ctx *ctx, int32_t kernel_class, int64_t *launches, double *total_ms) {
    if (!ctx || kernel_class < 0 || kernel_class >= LBA_KCLASS_COUNT) return LBA_ERR_INVALID_ARGUMENT;
    if (launches) *launches = ctx->prof_n[kernel_class];
    if (total_ms) *total_ms = ctx->prof_ms[kernel_class];
    return LBA_OK;
}

const char *lba_last_error(const lba_ctx *ctx) { return ctx ? ctx->err.c_str() : "NULL context"; }

lba_status lba_set_options(lba_ctx *ctx, const lba_options *opt) {
    if (!ctx || !opt) return LBA_ERR_INVALID_ARGUMENT;
    ctx->opt = *opt;
    return LBA_OK;
}

lba_status lba_workspace_size(lba_ctx *ctx, const lba_problem *problem, const lba_batch *batch, size_t *bytes) {
    if (!ctx || !bytes) return LBA_ERR_INVALID_ARGUMENT;
    ctx->err.clear();
    Plan pl;
    lba_status st = build_plan(ctx, problem, batch, pl);
    if (st != LBA_OK) return st;
    *bytes = pl.total;
    return LBA_OK;
}

lba_status lba_solve(lba_ctx *ctx, const lba_problem *problem, lba_result *result, void *workspace,
                     size_t workspace_bytes, void *stream) {
    return solve_impl(ctx, problem, nullptr, result, workspace, workspace_bytes, stream);
}

lba_status lba_cost_workspace_size(lba_ctx *ctx, const lba_problem *problem, const lba_batch *batch,
                                   size_t *bytes) {
    if (!ctx || !bytes) return LBA_ERR_INVALID_ARGUMENT;
    ctx->err.clear();
    CostPlan cp;
    lba_status st = build_cost_plan(ctx, problem, batch, cp);
    if (st != LBA_OK) return st;
    *bytes = cp.total;
    return LBA_OK;
}

lba_status lba_cost_forward(lba_ctx *ctx, const lba_problem *problem, const lba_batch *batch, const float *xi,
                            const float *X, const float *z, const uint8_t *mask, double *cost, void *workspace,
                            size_t workspace_bytes, void *stream) {
    return cost_impl(ctx, problem, batch, false, xi, X, z, mask, nullptr, cost, nullptr, nullptr, nullptr,
                     workspace, workspace_bytes, stream);
}

lba_status lba_cost_backward(lba_ctx *ctx, const lba_problem *problem, const lba_batch *batch, const float *xi,
                             const float *X, const float *z, const uint8_t *mask, const double *grad_cost,
                             float *g_xi, float *g_X, float *g_z, void *workspace, size_t workspace_bytes,
                             void *stream) {
    return cost_impl(ctx, problem, batch, true, xi, X, z, mask, grad_cost, nullptr, g_xi, g_X, g_z, workspace,
                     workspace_bytes, stream);
}

lba_status lba_tune(lba_ctx *ctx, const lba_problem *problem, const lba_batch *batch, void *stream,
                    int32_t *points_per_tile) {
    if (!ctx) return LBA_ERR_INVALID_ARGUMENT;
    ctx->err.clear();
    Plan pl0;
    lba_status st = build_plan(ctx, problem, batch, pl0);
    if (st != LBA_OK) return st;
    bool present[LBA_TUNE_CLASSES] = {};
    for (const WinInfo &W : pl0.win) present[window_class(W.Kopt, W.M)] = true;
    static const int cand[] = {64, 128, 256, 512, 1024, 2048, 4096};

    DeviceGuard dg;
    HIPCHK(dg.enter(ctx->device));
    hipStream_t s = static_cast<hipStream_t>(stream);
    void *ws = nullptr, *T = nullptr, *X = nullptr, *fl = nullptr;
    size_t ws_bytes = 0;
    auto release = [&] {
        (void)hipStreamSynchronize(s);
        for (auto &g : ctx->graphs) {
            (void)hipGraphExecDestroy(g.second.exec);
            (void)hipGraphDestroy(g.second.graph);
        }
        ctx->graphs.clear();
        if (ws) (void)hipFree(ws);
        if (T) (void)hipFree(T);
        if (X) (void)hipFree(X);
        if (fl) (void)hipFree(fl);
    };
    if (hipMalloc(&T, sizeof(double) * 12 * std::max(problem->n_kf, 1)) != hipSuccess ||
        hipMalloc(&X, sizeof(double) * 3 * std::max(problem->n_pt, 1)) != hipSuccess ||
        hipMalloc(&fl, std::max(problem->n_obs, 1)) != hipSuccess) {
        release();
        return set_error(ctx, LBA_ERR_HIP, "lba_tune: device allocation failed");
    }
    const lba_options saved = ctx->opt;
    const bool saved_prof = ctx->prof;
    ctx->opt.iters_round1 = 3;
    ctx->opt.iters_round2 = 0;
    ctx->opt.points_per_tile = 0;
    ctx->prof = false;
    lba_result R = {static_cast<double *>(T), static_cast<double *>(X), static_cast<uint8_t *>(fl), nullptr,
                    nullptr};
    int cfg[LBA_TUNE_CLASSES];
    double best = 0.0;
    // time of one short solve (three LM steps on every window) with the tile table c: the
    // workspace grows to the candidate's plan when it needs more (a table's size depends
    // on its tiles and on the update's parts per tile); the first run captures the step
    // graph, the least of the next three is taken
    auto measure = [&](const int *c, double *sec) -> lba_status {
        ctx->ppt_override = c;
        Plan pc;
        lba_status e = build_plan(ctx, problem, batch, pc);
        if (e != LBA_OK) return e;
        if (pc.total > ws_bytes) {
            if (hipStreamSynchronize(s) != hipSuccess) return set_error(ctx, LBA_ERR_HIP, "stream sync failed");
            for (auto &g : ctx->graphs) {   // captured graphs hold the old workspace's address
                (void)hipGraphExecDestroy(g.second.exec);
                (void)hipGraphDestroy(g.second.graph);
            }
            ctx->graphs.clear();
            if (ws) (void)hipFree(ws);
            ws = nullptr;
            if (hipMalloc(&ws, pc.total) != hipSuccess)
                return set_error(ctx, LBA_ERR_HIP, "lba_tune: device allocation of %zu bytes failed", pc.total);
            ws_bytes = pc.total;
        }
        *sec = 0.0;
        for (int rep = 0; rep < 4; ++rep) {
            if (hipStreamSynchronize(s) != hipSuccess) return set_error(ctx, LBA_ERR_HIP, "stream sync failed");
            const auto t0 = std::chrono::steady_clock::now();
            e = solve_impl(ctx, problem, batch, &R, ws, ws_bytes, stream);
            if (e != LBA_OK) return e;
            if (hipStreamSynchronize(s) != hipSuccess) return set_error(ctx, LBA_ERR_HIP, "stream sync failed");
            const double t = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            if (rep == 1 || (rep > 1 && t < *sec)) *sec = t;
        }
        return LBA_OK;
    };
    const int start = choose_points_per_tile(saved, problem->n_pt);
    for (int c = 0; c < LBA_TUNE_CLASSES; ++c) cfg[c] = start;
    st = measure(cfg, &best);
    // coordinate descent over the classes present; a change must gain 1%
    for (int c = 0; c < LBA_TUNE_CLASSES && st == LBA_OK; ++c) {
        if (!present[c]) continue;
        for (int v : cand) {
            if (v == cfg[c]) continue;
            int trial[LBA_TUNE_CLASSES];
            for (int q = 0; q < LBA_TUNE_CLASSES; ++q) trial[q] = cfg[q];
            trial[c] = v;
            double t = 0.0;
            st = measure(trial, &t);
            if (st != LBA_OK) break;
            if (t < 0.99 * best) {
                best = t;
                cfg[c] = v;
            }
        }
    }
    ctx->ppt_override = nullptr;
    ctx->opt = saved;
    ctx->prof = saved_prof;
    release();
    if (st != LBA_OK) return st;
    tune_signature(problem, pl0.nw, pl0.mixed, ctx->tuned_sig);
    for (int c = 0; c < LBA_TUNE_CLASSES; ++c) ctx->tuned_ppt[c] = cfg[c];
    if (points_per_tile)
        for (int c = 0; c < LBA_TUNE_CLASSES; ++c) points_per_tile[c] = cfg[c];
    return LBA_OK;
}

lba_status lba_tune_get(const lba_ctx *ctx, int32_t *points_per_tile) {
    if (!ctx || !points_per_tile) return LBA_ERR_INVALID_ARGUMENT;
    if (ctx->tuned_sig[0] == -1) return LBA_ERR_INVALID_ARGUMENT;
    for (int c = 0; c < LBA_TUNE_CLASSES; ++c) points_per_tile[c] = ctx->tuned_ppt[c];
    return LBA_OK;
}

lba_status lba_tune_set(lba_ctx *ctx, const int32_t *points_per_tile) {
    if (!ctx) return LBA_ERR_INVALID_ARGUMENT;
    ctx->err.clear();
    if (!points_per_tile) {   // forget the table
        ctx->tuned_sig[0] = -1;
        return LBA_OK;
    }
    for (int c = 0; c < LBA_TUNE_CLASSES; ++c)
        if (points_per_tile[c] < 1 || points_per_tile[c] > 65536)
            return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "points per tile of class %d must be in [1, 65536]", c);
    for (int c = 0; c < LBA_TUNE_CLASSES; ++c) ctx->tuned_ppt[c] = points_per_tile[c];
    ctx->tuned_sig[0] = -2;
    return LBA_OK;
}

lba_status lba_inertial_workspace_size(lba_ctx *ctx, const lba_problem *problem, const lba_batch *batch,
                                       const lba_inertial *inertial, size_t *bytes) {
    if (!ctx) return LBA_ERR_INVALID_ARGUMENT;
    ctx->err.clear();
    if (!bytes || !inertial) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "bytes / inertial is NULL");
    Plan pl;
    lba_status st = build_plan(ctx, problem, batch, pl, inertial);
    if (st != LBA_OK) return st;
    *bytes = pl.total;
    return LBA_OK;
}

lba_status lba_solve_inertial(lba_ctx *ctx, const lba_problem *problem, const lba_batch *batch,
                              const lba_inertial *inertial, lba_result *result, double *v_out, double *bg_out,
                              double *ba_out, void *workspace, size_t workspace_bytes, void *stream) {
    if (!ctx) return LBA_ERR_INVALID_ARGUMENT;
    if (!inertial) return set_error(ctx, LBA_ERR_INVALID_ARGUMENT, "inertial is NULL");
    return solve_impl(ctx, problem, batch, result, workspace, workspace_bytes, stream, inertial, v_out, bg_out,
                      ba_out);
}

lba_status lba_solve_batch(lba_ctx *ctx, const lba_problem *problem, const lba_batch *batch, lba_result *result,
                           void *workspace, size_t workspace_bytes, void *stream) {
    if (!batch) {
        if (ctx) ctx->err = "batch is NULL";
        return LBA_ERR_INVALID_ARGUMENT;
    }
    return solve_impl(ctx, problem, batch, result, workspace, workspace_bytes, stream);
}

}  // extern "C"
