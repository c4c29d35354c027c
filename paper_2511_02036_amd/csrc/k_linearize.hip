// Linearisation + Schur complement kernel (owner-computes).
//
// One 512-thread block per tile of one window's points, taken in the window's
// linearisation order (in windows with many optimisable keyframes, points sorted by the
// keyframes that observe them, so that a chunk's points share keyframes; the order and
// the observations copied into it are built once per solve).  The block's share of the
// reduced camera system
//     S = Hpp + lambda I - sum_j sum_{a,b in obs(j)} W_a V_j^-1 W_b^T,
//     r = bp - sum_j sum_{a in obs(j)} W_a V_j^-1 bl_j,
// is assembled on chip for the whole tile.  The tile is walked in chunks of whole points
// holding at most CO observations (512 for FP32 arithmetic, 256 for FP64); per chunk:
//   1. one thread per observation forms the residual (FP64), the robust weight and the
//      FP64 point block Hll_a and gradient bl_a, and marks its point in its camera's bit
//      mask;
//   2. the threads of each point sum Hll and bl through LDS, factor
//      V = Hll + lambda I = L L^T and stage Z_a = W_a L^-T (so W_a V^-1 W_b^T = Z_a Z_b^T);
//      the observation's own terms D_a = Hpp_a - Z_a Z_a^T and r_a = bp_a - Z_a L^-1 bl go
//      into FP64 per-camera sums in LDS, one copy per wavefront where LDS allows (LDS
//      atomics from the lanes of one wavefront only, which the hardware applies in a fixed
//      order), else one copy for the block;
//   3. every pair (a, b), a < b, of optimisable observations of one point is placed into
//      a list sorted by camera block: the count of block (kA, kB) is the popcount of the
//      two camera masks, and a pair's place is the number of the block's points before
//      its own; the threads of a point share its pairs round-robin (a chunk with two
//      observations of one point on one camera falls back to LDS integer atomics);
//   4. each block's run of the list is cut into pieces of at most kPiece pairs (8 in
//      FP32, or 6 when the chunk's pieces of 6 fit one batch; 4 in FP64); in batches of
//      PB pieces, two neighbouring threads per piece
//      (three rows each, sharing Z_b through a lane swap) sum the piece's -Z_a Z_b^T
//      (lower triangle of Z_a Z_b^T + Z_b Z_a^T for two observations on one camera) in
//      registers and write it to LDS in list order; 14 groups of 36 threads each own one
//      entry of every 14th camera block and add up the contiguous run of their block's
//      pieces in FP64 registers (no two threads add into the same entry, no atomics
//      touch S).
// At the end of the tile each owner writes its entry, plus the per-camera sums of the
// wavefronts in wavefront order on the diagonal blocks, to the tile's partial system; a
// separate kernel sums the partials of a window in a fixed order (no global atomics).
// With one copy of the camera sums per wavefront every sum is taken in a fixed order and
// two runs agree bit for bit, except in chunks with two observations of one point on one
// camera, whose pairs are placed by atomics of several wavefronts.
// The gradient bp itself is not needed: the gain-ratio denominator uses
// dp^T bp = dp^T r + sum_j q_j^T V_j^-1 bl_j (q_j = sum_a W_a^T dp), whose point part
// the update kernel forms.
#include "lba_internal.h"

#include <algorithm>

namespace lba {

constexpr int kNT = kLinThreads;           // 512
constexpr int kGroups = kLinThreads / 36;  // 14 groups of 36 threads, one block entry each
constexpr int kSlots = 34;                 // blocks per group and pass
constexpr int kPassBlocks = kGroups * kSlots;   // camera blocks per pass (476: Kopt <= 30 in one)

template <typename Real>
struct LinCfg {
    static constexpr int CO = sizeof(Real) == 4 ? 512 : 256;   // observations per chunk
    static constexpr int PCAP = sizeof(Real) == 4 ? 3072 : 2080;   // pairs per chunk (>= 64*65/2)
    static constexpr int PB = 256;                             // pieces per batch
    static constexpr int kPiece = sizeof(Real) == 4 ? 8 : 4;   // pairs per piece (measured best)
    // An FP32 chunk takes the smallest piece of 4, 5 or 6 pairs whose pieces fit one batch
    // (else pieces of kPiece): a batch costs each lane kp pair products, and every thread
    // pair of the block then holds a piece
    static constexpr bool kAdaptive = sizeof(Real) == 4;
    static constexpr int PS = 37;                              // product row stride (odd)
    // Z row stride in values: 19 (odd) rather than 18, so that the rows the lanes of a
    // wavefront gather by pair start in twice as many distinct LDS banks
    static constexpr int ZS = 19;
    static constexpr int RPT = 6 * PB / kNT;                   // product rows per thread
    static_assert(RPT == 3, "two neighbouring threads per piece");
    static_assert(PCAP < 65536, "packed scan of pair and piece counts");
};

template <typename Real>
struct LinSmem {
    double *T;       // K x 12 poses, then 34 weights: 1 / sigma2 per octave (32), Huber
                     // thresholds mono, stereo
    int *opt;        // K
    Real *Z;         // (CO + 1) x ZS (18 values per observation; row CO stays zero)
    double *hs;      // CO x 9    FP64 Hll_a (6) and bl_a (3) for the point sums
    int *ints;       // the chunk's observation ranges and points (phases 1-2)
    double *dacc;    // copies x Kopt x 27: per copy (wavefront, or one for the block) and
                     // camera, sum of D_a (lower triangle, 21) and r_a (6)
    unsigned *pairs; // PCAP pairs
    unsigned short *pcs;   // PCAP + 1 piece starts (list positions)
    Real *prod;      // PB x PS: signed 6 x 6 sum of each piece of the current batch
    int *cnt;        // pass blocks + 1 pair counts (then list offsets), then pass blocks + 1
                     // piece offsets
    int *cur;        // pass blocks
    int *oka;        // CO: optimisable camera of the chunk observation (-1: none)
    int *scan;       // 16: per-wavefront totals
    unsigned long long *touch;   // 2 x kGroups: per group, blocks with pairs in the batch, then
                                 // Kopt x 8: per camera, bit mask of the chunk's points it observes
    double *red;     // 8 x 2, then 4 ints: word offset of the chunk's record in the pool
                     // (-1: not stored)
};

// value of the neighbouring lane: lanes 2k and 2k + 1 exchange (DPP quad permutation
// [1, 0, 3, 2], no LDS traffic); both lanes must be active
template <typename Real>
__device__ __forceinline__ Real lane_pair_swap(Real v) {
    if constexpr (sizeof(Real) == 4) {
        return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
    } else {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), 0xB1, 0xF, 0xF, false);
        const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0xB1, 0xF, 0xF, false);
        return __longlong_as_double((long long)(unsigned)lo | ((long long)hi << 32));
    }
}

// The signed 6 x 6 sum over the pairs [r0, r1) of one piece (all of one camera block, so
// all with the same flag), by two neighbouring lanes: lane h of the pair forms rows 3h ..
// 3h + 2, summed in registers.  For two cameras (the common case) each lane loads only
// rows 3h .. 3h + 2 of Z_a and Z_b and takes the other half of Z_b from its neighbour;
// the list entries of the piece load at once and the pairs are unrolled without branches
// (a missing pair repeats the last with weight 0).
template <typename Real, int NP>
__device__ __forceinline__ void piece_product(const LinSmem<Real> &sm, int r0, int r1, int fl, int h, Real *out) {
    const int R0 = 3 * h, R1 = 3 - R0;   // own rows, the neighbour's rows
    if (fl == 0) {   // Z_a Z_b^T, camera of a before camera of b
        Real own[9], oth[9];   // [i][jj]: row R0 + i of the sum, column R0 + jj / R1 + jj
#pragma unroll
        for (int c = 0; c < 9; ++c) own[c] = oth[c] = (Real)0;
        // a piece of fewer than NP pairs is filled up with the zero row (row CO of Z)
        constexpr unsigned kZeroPair = (unsigned)LinCfg<Real>::CO | ((unsigned)LinCfg<Real>::CO << 10);
        unsigned e[NP];
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            const unsigned ev = sm.pairs[min(r0 + u, r1 - 1)];
            e[u] = r0 + u < r1 ? ev : kZeroPair;
        }
#pragma unroll
        for (int u = 0; u < NP; ++u) {
            constexpr int ZS = LinCfg<Real>::ZS;
            const Real *za = sm.Z + (e[u] & 1023) * ZS + R0 * 3, *zb = sm.Z + ((e[u] >> 10) & 1023) * ZS + R0 * 3;
            Real ai[9], bh[9], bo[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                ai[c] = za[c];
                bh[c] = zb[c];
            }
#pragma unroll
            for (int c = 0; c < 9; ++c) bo[c] = lane_pair_swap(bh[c]);
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int jj = 0; jj < 3; ++jj) {
                    own[i * 3 + jj] += ai[i * 3] * bh[jj * 3] + ai[i * 3 + 1] * bh[jj * 3 + 1] + ai[i * 3 + 2] * bh[jj * 3 + 2];
                    oth[i * 3 + jj] += ai[i * 3] * bo[jj * 3] + ai[i * 3 + 1] * bo[jj * 3 + 1] + ai[i * 3 + 2] * bo[jj * 3 + 2];
                }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int jj = 0; jj < 3; ++jj) {
                out[(R0 + i) * 6 + R0 + jj] = -own[i * 3 + jj];
                out[(R0 + i) * 6 + R1 + jj] = -oth[i * 3 + jj];
            }
    } else {         // one camera twice: Z_a Z_b^T + Z_b Z_a^T, lower triangle
        Real acc[18];
#pragma unroll
        for (int c = 0; c < 18; ++c) acc[c] = (Real)0;
        for (int r = r0; r < r1; ++r) {
            const unsigned e = sm.pairs[r];
            const Real *za = sm.Z + (e & 1023) * LinCfg<Real>::ZS, *zb = sm.Z + ((e >> 10) & 1023) * LinCfg<Real>::ZS;
            Real ai[9], bi[9];
#pragma unroll
            for (int c = 0; c < 9; ++c) {
                ai[c] = za[R0 * 3 + c];
                bi[c] = zb[R0 * 3 + c];
            }
#pragma unroll
            for (int j = 0; j < 6; ++j) {
                const Real b0 = zb[j * 3], b1 = zb[j * 3 + 1], b2 = zb[j * 3 + 2];
                const Real a0 = za[j * 3], a1 = za[j * 3 + 1], a2 = za[j * 3 + 2];
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    acc[i * 6 + j] += ai[i * 3] * b0 + ai[i * 3 + 1] * b1 + ai[i * 3 + 2] * b2 + bi[i * 3] * a0 +
                                      bi[i * 3 + 1] * a1 + bi[i * 3 + 2] * a2;
            }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 6; ++j)
                if (j <= R0 + i) out[(R0 + i) * 6 + j] = -acc[i * 6 + j];
    }
}

static __host__ __device__ inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// camera blocks one pass handles (every pass but the last takes kPassBlocks)
__host__ __device__ inline int pass_blocks(int Kopt) {
    const int nblk = Kopt * (Kopt + 1) / 2;
    return nblk < kPassBlocks ? nblk : kPassBlocks;
}

int lin_passes(int kopt) { return (kopt * (kopt + 1) / 2 + kPassBlocks - 1) / kPassBlocks; }

// LDS layout.  A window with fewer keyframes or optimisable keyframes than the launch was
// sized for takes less.
template <typename Real>
__host__ __device__ inline size_t lin_carve(unsigned char *base, int K, int Kopt, int copies, LinSmem<Real> *s) {
    using C = LinCfg<Real>;
    size_t o = 0;
    auto take = [&](size_t bytes) { void *p = base ? (void *)(base + o) : nullptr; o = align_up(o + bytes, 16); return p; };
    void *T = take(sizeof(double) * (12 * K + kMaxLevels + 2));
    void *opt = take(sizeof(int) * K);
    void *Z = take(sizeof(Real) * (C::CO + 1) * C::ZS);   // row CO: zeros
    // the staging of phases 1-2 (point-sum terms, then the chunk's observation ranges
    // (513), first observations and indices of its points (512 each) and the point of
    // each observation slot (CO), see the kernel) and the piece products of phase 4 share
    // space
    constexpr size_t kHs = sizeof(double) * C::CO * 9;
    constexpr size_t kStage = kHs + sizeof(int) * (kNT + 1 + 2 * kNT + C::CO);
    constexpr size_t kProd = sizeof(Real) * C::PB * C::PS;
    void *prod = take(kStage > kProd ? kStage : kProd);
    void *hs = prod;
    void *ints = base ? static_cast<void *>(static_cast<unsigned char *>(prod) + kHs) : nullptr;
    void *pairs = take(sizeof(unsigned) * C::PCAP);
    void *pcs = take(sizeof(unsigned short) * (C::PCAP + 1));
    const int nloc = pass_blocks(Kopt);
    void *cnt = take(sizeof(int) * 2 * (nloc + 1));
    void *cur = take(sizeof(int) * (nloc > 0 ? nloc : 1));
    void *touch = take(sizeof(unsigned long long) * (2 * kGroups + 8 * (Kopt > 0 ? Kopt : 1)));
    void *oka = take(sizeof(int) * C::CO);
    void *scan = take(sizeof(int) * 16);
    void *red = take(sizeof(double) * 2 * (kNT / 64) + sizeof(int) * 4);
    void *dacc = take(sizeof(double) * copies * Kopt * 27);
    if (s) {
        s->T = (double *)T; s->opt = (int *)opt; s->Z = (Real *)Z; s->hs = (double *)hs; s->ints = (int *)ints;
        s->dacc = (double *)dacc; s->pairs = (unsigned *)pairs; s->pcs = (unsigned short *)pcs; s->prod = (Real *)prod;
        s->cnt = (int *)cnt; s->cur = (int *)cur; s->touch = (unsigned long long *)touch; s->oka = (int *)oka;
        s->scan = (int *)scan; s->red = (double *)red;
    }
    return o;
}

size_t lin_lds_bytes(int K, int kopt, int copies, bool mixed) {
    return mixed ? lin_carve<float>(nullptr, K, kopt, copies, nullptr) : lin_carve<double>(nullptr, K, kopt, copies, nullptr);
}

int lin_self_copies(bool mixed) { return mixed ? LinCfg<float>::CO / 64 : LinCfg<double>::CO / 64; }

// index of block (ka <= kb) of the upper block triangle, row-major
__device__ __forceinline__ int block_id(int ka, int kb, int Kopt) { return ka * Kopt - ka * (ka - 1) / 2 + (kb - ka); }

// block row ka of block index B (0 <= B < Kopt (Kopt + 1) / 2): the largest ka with
// block_id(ka, ka) <= B, from the quadratic's root and one correction step each way
__device__ __forceinline__ int block_row(int B, int Kopt) {
    const float c = 2.0f * Kopt + 1.0f;
    int ka = (int)((c - sqrtf(fmaxf(c * c - 8.0f * B, 0.0f))) * 0.5f);
    ka = min(max(ka, 0), max(Kopt - 1, 0));
    if (ka > 0 && block_id(ka, ka, Kopt) > B) --ka;
    if (ka + 1 < Kopt && block_id(ka + 1, ka + 1, Kopt) <= B) ++ka;
    return ka;
}

// inclusive scan of one 64-bit value per thread over the block (512 threads).  The
// caller places a barrier between this and the next writer of scan[].
__device__ __forceinline__ long long block_inclusive_scan64(long long v, int *scan, int tid) {
    const int lane = tid & 63, wave = tid >> 6;
    long long x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const long long y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    long long *sc = reinterpret_cast<long long *>(scan);
    if (lane == 63) sc[wave] = x;
    __syncthreads();
    long long add = 0;
#pragma unroll
    for (int w = 0; w < kNT / 64; ++w) {
        const long long u = sc[w];
        add += w < wave ? u : 0;
    }
    return x + add;
}

// inclusive scan of one 64-bit value per thread over the block (512 threads), and the
// block's total.  The caller places a barrier between this and the next writer of scan[].
__device__ __forceinline__ unsigned long long block_inclusive_scan64_total(unsigned long long v, int *scan, int tid,
                                                                           unsigned long long &total) {
    const int lane = tid & 63, wave = tid >> 6;
    unsigned long long x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    unsigned long long *sc = reinterpret_cast<unsigned long long *>(scan);
    if (lane == 63) sc[wave] = x;
    __syncthreads();
    unsigned long long add = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kNT / 64; ++w) {
        const unsigned long long u = sc[w];
        add += w < wave ? u : 0ull;
        tot += u;
    }
    total = tot;
    return x + add;
}

// piece of the pair of rank rk in its block (constant divisors)
__device__ __forceinline__ int piece_of(int rk, int kp) {
    switch (kp) {
        case 4: return rk / 4;
        case 5: return rk / 5;
        case 6: return rk / 6;
        default: return rk / 8;
    }
}

// inclusive scan of one int per thread over the block (512 threads).  The caller places a
// barrier between this and the next writer of scan[].
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
#pragma unroll
    for (int w = 0; w < kNT / 64; ++w) {   // independent loads, one wait
        const int v = scan[w];
        add += w < wave ? v : 0;
    }
    return x + add;
}

// inclusive scan of one unsigned value per thread over the block (512 threads), and the
// block's total.  The caller places a barrier between this and the next writer of scan[].
__device__ __forceinline__ unsigned block_inclusive_scan_total(unsigned v, int *scan, int tid, unsigned &total) {
    const int lane = tid & 63, wave = tid >> 6;
    unsigned x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    unsigned *sc = reinterpret_cast<unsigned *>(scan);
    if (lane == 63) sc[wave] = x;
    __syncthreads();
    unsigned add = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kNT / 64; ++w) {
        const unsigned u = sc[w];
        add += w < wave ? u : 0u;
        tot += u;
    }
    total = tot;
    return x + add;
}

template <typename Real, typename ZT, typename Acc>
__global__ __launch_bounds__(kNT) void k_linearize(LinArgs a) {
    using C = LinCfg<Real>;
    extern __shared__ __align__(16) unsigned char smem[];
    const int t = a.order[blockIdx.x];
    const Tile tile = a.tiles[t];
    const WinInfo W = a.win[tile.win];
    const Ctl ctl = a.ctl[tile.win];
    if (!ctl.running) return;
    const int K = W.K, n = W.n, E = W.E, Kopt = W.Kopt;
    // pass blockIdx.y owns the camera blocks [bbase, bbase + nblk) of the upper block
    // triangle (row-major); its lists, offsets and owner slots use block indices local to
    // the pass
    const int bbase = blockIdx.y * kPassBlocks;
    const int nall = Kopt * (Kopt + 1) / 2;
    if (bbase > 0 && bbase >= nall) return;
    const int nblk = nall - bbase < kPassBlocks ? nall - bbase : kPassBlocks;
    const bool first_pass = blockIdx.y == 0;
    LinSmem<Real> sm;
    lin_carve<Real>(smem, K, Kopt, a.self_copies, &sm);
    unsigned long long *const cm = sm.touch + 2 * kGroups;
    double *const wt = sm.T + 12 * K;                                   // weights
    int *const rec = reinterpret_cast<int *>(sm.red + 2 * (kNT / 64));  // record offset
    int *const pst = sm.ints;                           // chunk-local observation starts
    int *const gst = pst + kNT + 1;                     // place of each point's first observation
    int *const pid = gst + kNT;                         // global index of each point
    int *const seg = pid + kNT;                         // chunk point of each observation slot
    int *const pco = sm.cnt + pass_blocks(Kopt) + 1;    // piece offsets per block
    unsigned short *const pcs = sm.pcs;                 // first list position of each piece
    const double lambda = ctl.lambda;
    const double *Xs = ctl.cur ? a.X1 : a.X0;
    const int tid = threadIdx.x;
    // Chunk records.  The pairs of a chunk, their pieces and the blocks' piece offsets
    // depend only on which observations are active, which is fixed within an LM round.
    // The first launch of a round forms them (phases 1-3 below) and stores one record per
    // chunk in the pool while it has room; later launches of the round load the records
    // instead of forming them.  A record: next record (word offset, ~0 for none), end
    // point of the chunk, pairs | pieces << 12 | code << 22 (pieces of 3 + code pairs, or
    // of kPiece for code 0), place of
    // the chunk's first observation; then the pairs, the piece starts (16-bit) and the
    // blocks' piece offsets (16-bit).
    const int slot = t * (int)gridDim.y + (int)blockIdx.y;
    const int head = a.plan_head ? a.plan_head[slot] : -1;
    const bool use = head >= 0 && (int64_t)head + 4 <= a.plan_cap;
    bool store = !use && a.plan_head != nullptr;   // uniform over the block
    uint4 hdr = make_uint4(0xffffffffu, 0u, 0u, 0u);
    if (use) hdr = *reinterpret_cast<const uint4 *>(a.plan + head);
    uint32_t recw = (uint32_t)head;   // record of the current chunk (use)
    uint32_t first_rec = 0xffffffffu, prev_rec = 0xffffffffu;   // thread 0, building

    for (int i = tid; i < 12 * K; i += kNT) sm.T[i] = a.T[(int64_t)W.kf0 * 12 + i];
    for (int i = tid; i < K; i += kNT) sm.opt[i] = a.opt_map[W.kf0 + i];
    // the weights by octave and type, read per observation: from LDS rather than from the
    // kernel arguments (one dependent memory round trip less per chunk)
    if (tid < kMaxLevels + 2) wt[tid] = tid < kMaxLevels ? a.c.inv_sigma2[tid] : a.c.huber2[tid - kMaxLevels];

    // ---- owned entries: thread g * 36 + q (g < 14) owns entry q = 6 i + j of the 6 x 6
    // blocks bbase + g + 14 k (kA <= kB).  In a diagonal block the entries j <= i are S, the
    // six upper positions 1 2 3 4 5 8 accumulate r of that camera, the rest are unused.
    const int grp = tid / 36, qe = tid - 36 * grp;
    const int nent = nblk;
    Acc acc[kSlots];
#pragma unroll
    for (int k = 0; k < kSlots; ++k) acc[k] = (Acc)0;
    unsigned long long m_r = 0, m_skip = 0;   // per slot: accumulates r / owns nothing
    {
        const int ie = qe / 6, je = qe - 6 * (qe / 6);
        const bool rpos = qe == 8 || (qe >= 1 && qe <= 5);
        for (int k = 0; k < kSlots; ++k) {
            const int B = grp + kGroups * k;
            const int kA = block_row(bbase + B, Kopt);
            const bool diag = bbase + B == block_id(kA, kA, Kopt);
            if (grp >= kGroups || B >= nent || (diag && je > ie && !rpos)) m_skip |= 1ull << k;
            else if (diag && rpos) m_r |= 1ull << k;
        }
    }
    // camera sums of the self terms, one copy per wavefront that holds observation slots
    // (CO / 64 copies) or one for the block, in the accumulation type (sized for FP64)
    const int ncopy = a.self_copies;
    Acc *const dacc = reinterpret_cast<Acc *>(sm.dacc);
    for (int i = tid; i < ncopy * Kopt * 27; i += kNT) dacc[i] = (Acc)0;
    if (tid < C::ZS) sm.Z[C::CO * C::ZS + tid] = (Real)0;   // the zero row that fills pieces
    __syncthreads();

    const CamParams cam = a.c.cam;
    double Facc = 0.0;
    int fail = 0;

    // the point records of the next chunk are loaded one chunk ahead (thread t: point p + t)
    int4 pin = make_int4(0, 0, 0, 0);
    if (tile.p0 + tid < tile.p1) pin = a.pinfo[tile.p0 + tid];
    // With stored records the next chunk's first place is known one chunk ahead, so (in
    // FP32 arithmetic, whose registers allow it) the next chunk's observations (by place:
    // slot s holds place base + s) and its points' positions are loaded during the current
    // chunk's products, and its first phase waits on no memory.
    constexpr bool kPre = sizeof(Real) == 4;
    bool nxt = false;   // use: a next chunk exists (its header is in hdr)
    bool pre = false;   // this chunk's observations and positions are in the registers below
    // (each loaded value stays in its own register until the next chunk uses it: combining
    // them here would wait on the loads)
    int pf_kf = 0, pf_type = 0, pf_oct = 0, pf_flag = 0;
    ZT pf_z0 = 0, pf_z1 = 0, pf_z2 = 0;
    double pf_X0 = 0, pf_X1 = 0, pf_X2 = 0;   // thread t: position of the chunk's point t
    uint32_t cw[8];   // use: this thread's words of the chunk's record (loaded with the above)
    // the record words of the chunk whose header is in hdr and which starts at word recw
    auto load_words = [&](int tid_) {
        const int npr_ = (int)(hdr.z & 4095u);
        const int nwc_ = (int)((((hdr.z >> 12) & 1023u) + 2u) >> 1);
        int ntot_ = npr_ + nwc_ + ((nblk + 2) >> 1);
        if ((int64_t)recw + 4 + ntot_ > a.plan_cap) ntot_ = 0;
        const uint32_t *src = a.plan + recw + 4;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int i = tid_ + kNT * u;
            cw[u] = i < ntot_ ? src[i] : 0u;
        }
    };
    for (int p = tile.p0; p < tile.p1;) {
        // The thread index is re-derived per chunk behind an empty asm statement, so the
        // compiler recomputes the LDS addresses built from it inside the chunk instead of
        // keeping them all live across the loop (which overflows the FP64 register budget).
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        // ---- chunk of whole points: <= CO observations and <= PCAP pairs ------------
        int q, np;
        int kp = C::kPiece;   // pairs per piece in this chunk (the same in every thread)
        int npr = 0, nwc = 0, ntot = 0;
        if (use) {
            q = (int)hdr.y;
            npr = (int)(hdr.z & 4095u);
            nwc = (int)((((hdr.z >> 12) & 1023u) + 2u) >> 1);
            if (C::kAdaptive && ((hdr.z >> 22) & 3u)) kp = 3 + (int)((hdr.z >> 22) & 3u);
            ntot = npr + nwc + ((nblk + 2) >> 1);
            if ((int64_t)recw + 4 + ntot > a.plan_cap) ntot = 0;   // (the pool's bound; fails below)
            if (!(kPre && pre)) load_words(tid);
            if (q <= p || q > tile.p1 || ntot == 0) {   // records that do not fit the tile: not solvable
                fail = 1;
                break;
            }
            np = q - p;
            const int base = (int)hdr.w;
            // the previous chunk's owners read their products from the region that holds
            // the chunk's ranges (and its products read Z, which holds the positions until
            // phase 2)
            __syncthreads();
            if (kPre && pre && tid < np) {
                double *const xs = reinterpret_cast<double *>(sm.Z);
                xs[3 * tid] = pf_X0;
                xs[3 * tid + 1] = pf_X1;
                xs[3 * tid + 2] = pf_X2;
            }
            if (tid < np) {
                pst[tid + 1] = pin.w + pin.z - base;
                gst[tid] = pin.w;
                pid[tid] = pin.x;
                for (int i = pin.w - base; i < pin.w - base + pin.z; ++i) seg[i] = tid;
            }
            if (tid == 0) pst[0] = 0;
            pin = make_int4(0, 0, 0, 0);
            if (q + tid < tile.p1) pin = a.pinfo[q + tid];
            nxt = hdr.x != 0xffffffffu && (int64_t)hdr.x + 4 <= a.plan_cap;
            if (nxt) {
                recw = hdr.x;
                hdr = *reinterpret_cast<const uint4 *>(a.plan + recw);
            }
        } else {
            for (int i = tid; i < Kopt * 8; i += kNT) cm[i] = 0ull;
            const int cand = p + tid;
            int P = 0, ps = 0, m = 0, inrange = 0;
            if (cand < tile.p1) {
                P = pin.x;
                ps = pin.w;   // place of the point's first observation
                m = pin.z;
                inrange = 1;
            }
            // observations (high word) and pair slots (low word) up to and including this point
            const long long incl =
                block_inclusive_scan64(((long long)m << 32) | (long long)(m * (m + 1) / 2), sm.scan, tid);
            const int obs_incl = (int)(incl >> 32), pincl = (int)(incl & 0xffffffffll);
            const int ok = inrange && obs_incl <= C::CO && pincl <= C::PCAP;
            q = p + __syncthreads_count(ok);
            if (q == p) {   // one point exceeds a chunk: not solvable here
                fail = 1;
                break;
            }
            pin = make_int4(0, 0, 0, 0);
            if (q + tid < tile.p1) pin = a.pinfo[q + tid];
            // the chunk's point ranges and observation slots go to LDS
            np = q - p;
            if (tid < np) {
                pst[tid + 1] = obs_incl;
                gst[tid] = ps;
                pid[tid] = P;
                for (int i = obs_incl - m; i < obs_incl; ++i) seg[i] = tid;
            }
            if (tid == 0) pst[0] = 0;
        }
        int pl = 0, kl = 0, stereo = 0, oct = 0;
        bool act = false;
        double zu = 0, zv = 0, zr = 0;
        double X0 = 0, X1 = 0, X2 = 0;
        __syncthreads();
        const bool has = tid < pst[np];
        if (has) {   // observation slot tid: observation tid - pst[pl] of chunk point pl, and
                     // its point's position, loaded together
            pl = seg[tid];
            if (kPre && pre) {
                const double *const xs = reinterpret_cast<const double *>(sm.Z);
                X0 = xs[3 * pl];
                X1 = xs[3 * pl + 1];
                X2 = xs[3 * pl + 2];
                kl = pf_kf;
                stereo = pf_type;
                oct = pf_oct;
                act = (a.smask == nullptr) | (pf_flag == 0);
                zu = (double)pf_z0;
                zv = (double)pf_z1;
                zr = (double)pf_z2;
            } else {
                const int o = gst[pl] + tid - pst[pl];   // the chunk's places are contiguous
                const int64_t Pg = pid[pl];
                X0 = Xs[3 * Pg];
                X1 = Xs[3 * Pg + 1];
                X2 = Xs[3 * Pg + 2];
                kl = a.sobs.kf[o];
                // the flag is loaded without a branch (from a readable byte array when
                // there is none), so that it issues with the other loads
                const uint8_t flag = (a.smask ? a.smask : a.sobs.type)[o];
                act = (a.smask == nullptr) | (flag == 0);
                stereo = a.sobs.type[o];
                oct = a.sobs.oct[o];
                load_z<ZT>(a.sobs, o, zu, zv, zr);
            }
        }

        // ---- 1. per-observation terms -------------------------------------------------
        // (only the raw observation stays in registers across the point-sum barrier; the
        //  factored blocks are recomputed from it in phase 2)
        int s0 = 0, s1 = 0, ka = -1, dup = 0;
        double omd = 0.0;
        double rho = 0.0;
        if (has) {
            s0 = pst[pl];
            s1 = pst[pl + 1];
            ka = sm.opt[kl];
            const double *T = sm.T + kl * 12;
            double xc, yc, zc, eu, ev, er;
            const double e2 = residual(cam, T, X0, X1, X2, zu, zv, zr, stereo, xc, yc, zc, eu, ev, er);
            const double isg = wt[oct];
            double w;
            huber(e2 * isg, wt[kMaxLevels + stereo], a.robust, rho, w);
            if (!act) rho = 0.0;
            omd = act ? w * isg : 0.0;
            double Hll[6], bl[3];
            point_block_fp64(cam, T, xc, yc, zc, eu, ev, er, stereo, omd, Hll, bl);
#pragma unroll
            for (int i = 0; i < 6; ++i) sm.hs[tid * 9 + i] = Hll[i];
#pragma unroll
            for (int i = 0; i < 3; ++i) sm.hs[tid * 9 + 6 + i] = bl[i];
            if (!act) ka = -1;
            sm.oka[tid] = ka;
            if (ka >= 0 && !use) {   // the point in its camera's mask; a second hit is a duplicate
                const unsigned long long bit = 1ull << (pl & 63);
                dup = (__hip_atomic_fetch_or(&cm[ka * 8 + (pl >> 6)], bit, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_WORKGROUP) & bit) != 0;
            }
        }
        Facc += rho;
        // list counters of phase 3, cleared here so that phases 2 and 3 need no barrier
        // between them (the previous chunk's last reads of them precede a barrier); a
        // stored record goes to the lists instead
        if (!use) {
            for (int B = tid; B < nblk; B += kNT) {
                sm.cnt[B] = 0;
                sm.cur[B] = 0;
            }
        } else {
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int i = tid + kNT * u;
                if (i >= ntot) continue;
                const uint32_t v = cw[u];
                if (i < npr) {
                    sm.pairs[i] = v;
                } else if (i < npr + nwc) {
                    const int j = 2 * (i - npr);
                    pcs[j] = (unsigned short)(v & 0xffffu);
                    pcs[j + 1] = (unsigned short)(v >> 16);
                } else {
                    const int j = 2 * (i - npr - nwc);
                    pco[j] = (int)(v & 0xffffu);
                    if (j + 1 <= nblk) pco[j + 1] = (int)(v >> 16);
                }
            }
        }
        if (tid < 2 * kGroups) sm.touch[tid] = 0ull;
        int anydup = 0;   // a chunk with stored records was formed without duplicates
        if (use) __syncthreads();
        else anydup = __syncthreads_or(dup);

        // ---- 2. per-point sums, point factor, staged Z_a, D_a, r_a ---------------------
        double V[6] = {0, 0, 0, 0, 0, 0};
        double bs[3] = {0, 0, 0};
        if (has) {   // two observations per step: their 18 loads issue together
            for (int m = s0; m < s1; m += 2) {
                const bool two = m + 1 < s1;
                const double *h0 = sm.hs + m * 9, *h1 = sm.hs + (two ? m + 1 : m) * 9;
                double u0[9], u1[9];
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    u0[i] = h0[i];
                    u1[i] = h1[i];
                }
#pragma unroll
                for (int i = 0; i < 6; ++i) V[i] += u0[i];
#pragma unroll
                for (int i = 0; i < 3; ++i) bs[i] += u0[6 + i];
                if (two) {
#pragma unroll
                    for (int i = 0; i < 6; ++i) V[i] += u1[i];
#pragma unroll
                    for (int i = 0; i < 3; ++i) bs[i] += u1[6 + i];
                }
            }
        }
        double Li[6] = {0, 0, 0, 0, 0, 0};
        double t0 = 0, t1 = 0, t2 = 0;
        if (has) {
            V[0] += lambda;
            V[3] += lambda;
            V[5] += lambda;
            if (!chol3_inv<double>(V, Li)) fail = 1;
            lmul<double>(Li, bs[0], bs[1], bs[2], t0, t1, t2);
            if (tid == s0 && first_pass) {   // the point's factor, for this step's back-substitution
                double *f = a.pf + 12 * (int64_t)pid[pl];
#pragma unroll
                for (int i = 0; i < 6; ++i) f[i] = Li[i];
                f[6] = t0; f[7] = t1; f[8] = t2;
                f[9] = bs[0]; f[10] = bs[1]; f[11] = bs[2];
            }
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
            for (int i = 0; i < 18; ++i) sm.Z[tid * C::ZS + i] = Zr[i];
            // the observation's own term, D_a = Hpp_a - Z_a Z_a^T and r_a = bp_a - Z_a t, goes
            // into its camera's sums of this wavefront.  Lanes of the same camera belong to
            // different points; in FP32 chunks a lane adds the 27 entries starting from entry
            // 0, 9 or 18 (its point's index mod 3), so that fewer lanes of one atomic
            // instruction meet at the same address (three starts measured faster than two or
            // four; FP64 chunks have no registers left for the selects)
            Acc *dst = dacc + ((ncopy > 1 ? tid >> 6 : 0) * Kopt + ka) * 27;
            auto entry = [&](int e) -> Acc {
                if (e < 21) {
                    int i = 0;
                    while ((i + 1) * (i + 2) / 2 <= e) ++i;
                    const int j = e - i * (i + 1) / 2;
                    return (Acc)(H[i * 6 + j] - (Zr[i * 3] * Zr[j * 3] + Zr[i * 3 + 1] * Zr[j * 3 + 1] +
                                                 Zr[i * 3 + 2] * Zr[j * 3 + 2]));
                }
                const int i = e - 21;
                return (Acc)(bpd[i] - ((double)Zr[i * 3] * t0 + (double)Zr[i * 3 + 1] * t1 + (double)Zr[i * 3 + 2] * t2));
            };
            if constexpr (sizeof(Real) == 4) {
                const int cls = pl % 3;
#pragma unroll
                for (int e = 0; e < 27; ++e) {
                    const Acc v0 = entry(e), v1 = entry((e + 9) % 27), v2 = entry((e + 18) % 27);
                    const int o = cls == 0 ? e : cls == 1 ? (e + 9) % 27 : (e + 18) % 27;
                    lds_add(dst + o, cls == 0 ? v0 : cls == 1 ? v1 : v2);
                }
            } else {
#pragma unroll
                for (int e = 0; e < 27; ++e) lds_add(dst + e, entry(e));
            }
        }

        // ---- 3. pair lists sorted by camera block --------------------------------------
        // Without duplicate (point, camera) observations the pairs of block (kA, kB) are
        // the chunk's points seen by both cameras: their count is a popcount of the two
        // camera masks and a pair's place in its block is the number of such points
        // before its own, so the list is ordered by block, then point.  A chunk with a
        // duplicate counts and places its pairs with LDS atomics instead.
        if (!use) {
            const int nwrd = (q - p + 63) >> 6;
            if (!anydup) {
                for (int B = tid; B < nblk; B += kNT) {
                    const int Bg = bbase + B;
                    const int kA = block_row(Bg, Kopt), kB = kA + (Bg - block_id(kA, kA, Kopt));
                    int c = 0;
                    if (kA != kB)
                        for (int w = 0; w < nwrd; ++w) c += __popcll(cm[kA * 8 + w] & cm[kB * 8 + w]);
                    sm.cnt[B] = c;
                }
            } else if (ka >= 0) {
                for (int b0 = tid + 1; b0 < s1; b0 += 4) {   // partners four at a time: one wait per four
                    int kb[4];
    #pragma unroll
                    for (int u = 0; u < 4; ++u) kb[u] = b0 + u < s1 ? sm.oka[b0 + u] : -1;
    #pragma unroll
                    for (int u = 0; u < 4; ++u)
                        if (kb[u] >= 0) {
                            const int Bl = (ka <= kb[u] ? block_id(ka, kb[u], Kopt) : block_id(kb[u], ka, Kopt)) - bbase;
                            if (Bl >= 0 && Bl < nblk) atomicAdd(&sm.cnt[Bl], 1);
                        }
                }
            }
            __syncthreads();
            if constexpr (C::kAdaptive) {
                // pair offsets (bits 0-11, at most PCAP = 3072) and the piece offsets for
                // pieces of 4 (bits 12-22), 5 (23-33), 6 (34-43) and 8 pairs (44-53) in one
                // scan: a block of c pairs has at most c / kp + 1 pieces, so the fields stay
                // below PCAP / kp + kPassBlocks (1,244, 1,090, 988, 860)
                static_assert(C::PCAP < 4096 && C::PCAP / 4 + kPassBlocks < 2048 && C::PCAP / 6 + kPassBlocks < 1024,
                              "scan fields");
                const unsigned long long c = tid < nblk ? (unsigned long long)sm.cnt[tid] : 0ull;
                const unsigned long long v = c | (((c + 3) / 4) << 12) | (((c + 4) / 5) << 23) | (((c + 5) / 6) << 34) |
                                             (((c + 7) / 8) << 44);
                unsigned long long tot;
                const unsigned long long incl = block_inclusive_scan64_total(v, sm.scan, tid, tot);
                const unsigned long long ex = incl - v;
                int sh = 44, mask = 1023;
                kp = 8;
                if (((tot >> 34) & 1023ull) <= (unsigned long long)C::PB) { kp = 6; sh = 34; }
                if (((tot >> 23) & 2047ull) <= (unsigned long long)C::PB) { kp = 5; sh = 23; mask = 2047; }
                if (((tot >> 12) & 2047ull) <= (unsigned long long)C::PB) { kp = 4; sh = 12; mask = 2047; }
                if (tid < nblk) {
                    sm.cnt[tid] = (int)(ex & 4095ull);
                    pco[tid] = (int)((ex >> sh) & (unsigned long long)mask);
                }
                if (tid == nblk - 1) {
                    const int np_ = (int)((incl >> sh) & (unsigned long long)mask);
                    sm.cnt[nblk] = (int)(incl & 4095ull);
                    pco[nblk] = np_;
                    pcs[np_] = (unsigned short)(incl & 4095ull);
                }
            } else {   // pair offsets (low half) and piece offsets (high half) in one scan
                const int c = tid < nblk ? sm.cnt[tid] : 0;
                const int v = c | (((c + C::kPiece - 1) / C::kPiece) << 16);
                const int incl = block_inclusive_scan(v, sm.scan, tid);
                if (tid < nblk) {
                    sm.cnt[tid] = (incl - v) & 0xffff;
                    pco[tid] = (incl - v) >> 16;
                }
                if (tid == nblk - 1) {
                    sm.cnt[nblk] = incl & 0xffff;
                    pco[nblk] = incl >> 16;
                    if (C::kPiece > 1) pcs[incl >> 16] = (unsigned short)(incl & 0xffff);
                }
            }
            __syncthreads();
            if (store && tid == 0) {   // room for this chunk's record in the pool
                const int npr_c = nblk > 0 ? sm.cnt[nblk] : 0, npc_c = nblk > 0 ? pco[nblk] : 0;
                const unsigned long long words =
                    (unsigned long long)((4 + npr_c + ((npc_c + 2) >> 1) + ((nblk + 2) >> 1) + 3) & ~3);
                const unsigned long long off = atomicAdd(a.plan_ctr, words);
                rec[0] = off + words <= (unsigned long long)a.plan_cap ? (int)off : -1;
            }
            // Placement.  The pairs of one point are shared round-robin by all its observation
            // threads (pair g of a point of m observations goes to its thread g mod m), so no
            // thread places more than ceil((m - 1) / 2) of them; a chunk with a repeated
            // observation places each observation's pairs with its later partners (atomics).
            auto place = [&](int sa, int sb, int kA, int kB, int rk, int B) {
                // first = the observation on the lower camera; flag 2 = two observations of
                // one point on the same camera
                const int first = kA <= kB ? sa : sb, second = kA <= kB ? sb : sa;
                const unsigned fl = kA == kB ? 2u : 0u;
                const int pos = sm.cnt[B] + rk;
                sm.pairs[pos] = (unsigned)first | ((unsigned)second << 10) | (fl << 20);
                if (C::kPiece > 1) {
                    const int pq = piece_of(rk, kp);
                    if (rk == pq * kp) pcs[pco[B] + pq] = (unsigned short)pos;
                }
            };
            if (!anydup) {
                if (has) {
                    const int pw = pl >> 6;
                    const unsigned long long below = (1ull << (pl & 63)) - 1ull;
                    const int mp = s1 - s0, npp = mp * (mp - 1) / 2;
                    for (int g = tid - s0; g < npp; g += mp) {
                        // pair g = (a, b), a < b, in row order: row a starts at a m - a (a + 1) / 2
                        const float c = 2.0f * mp - 1.0f;
                        int ar = (int)((c - sqrtf(fmaxf(c * c - 8.0f * g, 0.0f))) * 0.5f);
                        ar = min(max(ar, 0), mp - 2);
                        if (ar > 0 && ar * mp - ar * (ar + 1) / 2 > g) --ar;
                        if (ar + 1 <= mp - 2 && (ar + 1) * mp - (ar + 1) * (ar + 2) / 2 <= g) ++ar;
                        const int br = ar + 1 + (g - (ar * mp - ar * (ar + 1) / 2));
                        const int sa = s0 + ar, sb = s0 + br;
                        const int kA = sm.oka[sa], kB = sm.oka[sb];
                        if (kA < 0 || kB < 0) continue;
                        const int lo = min(kA, kB), hi = max(kA, kB);
                        const int Bl = block_id(lo, hi, Kopt) - bbase;   // another pass's block
                        if (Bl < 0 || Bl >= nblk) continue;
                        int r = __popcll(cm[lo * 8 + pw] & cm[hi * 8 + pw] & below);
                        for (int w = 0; w < pw; ++w) r += __popcll(cm[lo * 8 + w] & cm[hi * 8 + w]);
                        place(sa, sb, kA, kB, r, Bl);
                    }
                }
            } else if (ka >= 0) {
                for (int b = tid + 1; b < s1; ++b) {
                    const int kb = sm.oka[b];
                    if (kb < 0) continue;
                    const int B = block_id(min(ka, kb), max(ka, kb), Kopt) - bbase;
                    if (B < 0 || B >= nblk) continue;
                    place(tid, b, ka, kb, atomicAdd(&sm.cur[B], 1), B);
                }
            }
            __syncthreads();
            if (store) {   // the chunk's record, for the later launches of this round
                const int off = rec[0];
                if (off < 0) {
                    store = false;
                } else {
                    const int npr_c = nblk > 0 ? sm.cnt[nblk] : 0, npc_c = nblk > 0 ? pco[nblk] : 0;
                    const int nwc_c = (npc_c + 2) >> 1, nwo_c = (nblk + 2) >> 1;
                    uint32_t *dst = a.plan + off;
                    for (int i = tid; i < npr_c; i += kNT) dst[4 + i] = sm.pairs[i];
                    for (int i = tid; i < nwc_c; i += kNT)
                        dst[4 + npr_c + i] = (uint32_t)pcs[2 * i] | ((uint32_t)pcs[2 * i + 1] << 16);
                    for (int i = tid; i < nwo_c; i += kNT)
                        dst[4 + npr_c + nwc_c + i] =
                            (uint32_t)pco[2 * i] | ((2 * i + 1 <= nblk ? (uint32_t)pco[2 * i + 1] : 0u) << 16);
                    if (tid == 0) {
                        const uint32_t sm_flag = (C::kAdaptive && kp < C::kPiece) ? (uint32_t)(kp - 3) : 0u;
                        *reinterpret_cast<uint4 *>(dst) =
                            make_uint4(0xffffffffu, (uint32_t)q, (uint32_t)npr_c | ((uint32_t)npc_c << 12) | (sm_flag << 22),
                                       (uint32_t)gst[0]);
                        if (prev_rec != 0xffffffffu) a.plan[prev_rec] = (uint32_t)off;
                        else first_rec = (uint32_t)off;
                        prev_rec = (uint32_t)off;
                    }
                }
            }
        } else {
            __syncthreads();   // Z staged
            if (kPre) {   // the next chunk's observations and positions
                pre = nxt;
                if (nxt) {
                    const int o = (int)hdr.w + tid;
                    if (o < a.sobs.n_obs) {
                        pf_kf = a.sobs.kf[o];
                        pf_flag = (a.smask ? a.smask : a.sobs.type)[o];
                        pf_type = a.sobs.type[o];
                        pf_oct = a.sobs.oct[o];
                        const ZT *z = static_cast<const ZT *>(a.sobs.z);
                        pf_z0 = z[o];
                        pf_z1 = z[(int64_t)a.sobs.n_obs + o];
                        pf_z2 = z[2 * (int64_t)a.sobs.n_obs + o];
                    }
                    if (q + tid < tile.p1) {
                        const int64_t P = pin.x;
                        pf_X0 = Xs[3 * P];
                        pf_X1 = Xs[3 * P + 1];
                        pf_X2 = Xs[3 * P + 2];
                    }
                    load_words(tid);   // (this chunk's words are in LDS since phase 1)
                }
            }
        }

        // ---- 4. piece products, PB at a time, then each owner sums its rows --------------
        const int npieces = nblk > 0 ? pco[nblk] : 0;
        for (int b0 = 0, bi = 0; b0 < npieces; b0 += C::PB, ++bi) {
            unsigned long long *touch = sm.touch + (bi & 1) * kGroups;
            {   // neighbouring threads 2k, 2k + 1 -> piece b0 + k, rows 0 .. 2 / 3 .. 5
                const int pi = b0 + (tid >> 1), h = tid & 1;
                if (pi < npieces) {
                    const int r0 = C::kPiece > 1 ? (int)pcs[pi] : pi;
                    const int r1 = C::kPiece > 1 ? (int)pcs[pi + 1] : pi + 1;
                    const unsigned e = sm.pairs[r0];
                    const int fl = e >> 20;
                    Real *out = sm.prod + (pi - b0) * C::PS;
                    if (h == 0) {   // the first piece of a block in this batch marks the block
                        const int ka = sm.oka[e & 1023], kb = sm.oka[(e >> 10) & 1023];
                        const int B = block_id(ka, kb, Kopt) - bbase;
                        if (pi == b0 || pi == pco[B])
                            __hip_atomic_fetch_or(&touch[B % kGroups], 1ull << (B / kGroups), __ATOMIC_RELAXED,
                                                  __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                    if constexpr (C::kAdaptive) {
                        if (kp == 4) piece_product<Real, 4>(sm, r0, r1, fl, h, out);
                        else if (kp == 5) piece_product<Real, 5>(sm, r0, r1, fl, h, out);
                        else if (kp == 6) piece_product<Real, 6>(sm, r0, r1, fl, h, out);
                        else piece_product<Real, C::kPiece>(sm, r0, r1, fl, h, out);
                    } else {
                        piece_product<Real, C::kPiece>(sm, r0, r1, fl, h, out);
                    }
                }
            }
            __syncthreads();
            const Real *col = sm.prod + qe;
            const unsigned long long live = grp < kGroups ? touch[grp] & ~m_skip & ~m_r : 0ull;
            // the other buffer was last read before this batch began: clear it for the next
            if (tid < kGroups) sm.touch[((bi + 1) & 1) * kGroups + tid] = 0ull;
#pragma unroll
            for (int k = 0; k < kSlots; ++k) {
                if (!((live >> k) & 1)) continue;
                const int B = grp + kGroups * k;
                const int p0 = max(pco[B], b0) - b0, p1 = min(pco[B + 1], b0 + C::PB) - b0;
                int pi = p0;   // four pieces per step: their loads are independent
                for (; pi + 4 <= p1; pi += 4)
                    acc[k] += ((Acc)col[pi * C::PS] + (Acc)col[(pi + 1) * C::PS]) +
                              ((Acc)col[(pi + 2) * C::PS] + (Acc)col[(pi + 3) * C::PS]);
                for (; pi < p1; ++pi) acc[k] += (Acc)col[pi * C::PS];
            }
            // the next batch overwrites the products; after the last one, the next chunk
            // writes this region only after its first barrier
            if (b0 + C::PB < npieces) __syncthreads();
        }
        p = q;
    }

    // ---- write-out: owned rows of S, r, and the tile's scalars ----------------------
    {
        double *part = a.part + W.part_off + (int64_t)(t - W.tile0) * W.part_stride;
        double *pr = a.partr + W.partr_off + (int64_t)(t - W.tile0) * n;
#pragma unroll
        for (int k = 0; k < kSlots; ++k) {
            if ((m_skip >> k) & 1) continue;
            const int B = bbase + grp + kGroups * k;
            const int kA = block_row(B, Kopt);
            const int ri = qe <= 5 ? qe - 1 : 5;
            if ((m_r >> k) & 1) {
                Acc v = (Acc)0;
                for (int w = 0; w < ncopy; ++w) v += dacc[(w * Kopt + kA) * 27 + 21 + ri];
                pr[6 * kA + ri] = (double)v;
                continue;
            }
            const int kB = kA + (B - block_id(kA, kA, Kopt));
            const int ie = qe / 6, je = qe - 6 * (qe / 6);
            Acc v = acc[k];
            if (kA == kB)
                for (int w = 0; w < ncopy; ++w) v += dacc[(w * Kopt + kA) * 27 + ie * (ie + 1) / 2 + je];
            const int ra = 6 * kA + ie, col = 6 * kB + je;
            part[ra >= col ? packed_lower(ra, col) : packed_lower(col, ra)] = (double)v;
        }
    }
    Facc = wave_sum(Facc);
    const int anyfail = __syncthreads_or(fail);
    if ((tid & 63) == 0) {
        sm.red[(tid >> 6) * 2] = Facc;
        sm.red[(tid >> 6) * 2 + 1] = 0.0;
    }
    __syncthreads();
    if (tid == 0 && first_pass) {
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
    // every chunk of the tile has its record: the later launches of the round use them
    if (tid == 0 && store && !anyfail && first_rec != 0xffffffffu) a.plan_head[slot] = (int32_t)first_rec;
    (void)E;
}

hipError_t launch_linearize(const LinArgs &a, int ntiles, int passes, size_t lds, bool mixed, hipStream_t s) {
    if (ntiles <= 0) return hipSuccess;
    dim3 grid(ntiles, passes > 0 ? passes : 1), block(kNT);
    const bool zf = a.obs.z_f32 != 0;
    if (mixed && a.acc32) {   // the literal precision form: S summed in FP32
        if (zf) hipLaunchKernelGGL((k_linearize<float, float, float>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_linearize<float, double, float>), grid, block, lds, s, a);
    } else if (mixed) {
        if (zf) hipLaunchKernelGGL((k_linearize<float, float, double>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_linearize<float, double, double>), grid, block, lds, s, a);
    } else {
        if (zf) hipLaunchKernelGGL((k_linearize<double, float, double>), grid, block, lds, s, a);
        else hipLaunchKernelGGL((k_linearize<double, double, double>), grid, block, lds, s, a);
    }
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_plan_reset(int32_t *head, int n, unsigned long long *ctr) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) head[i] = -1;
    if (i == 0) *ctr = 0ull;
}

hipError_t launch_plan_reset(const LinArgs &a, int slots, hipStream_t s) {
    if (!a.plan_head || slots <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_plan_reset, dim3((slots + 255) / 256), dim3(256), 0, s, a.plan_head, slots, a.plan_ctr);
    return hipGetLastError();
}

size_t lin_static_lds() {
    const void *f[6] = {(const void *)k_linearize<float, float, float>, (const void *)k_linearize<float, double, float>,
                        (const void *)k_linearize<float, float, double>, (const void *)k_linearize<float, double, double>,
                        (const void *)k_linearize<double, float, double>, (const void *)k_linearize<double, double, double>};
    size_t m = 0;
    for (const void *p : f) m = std::max(m, kernel_static_lds(p));
    return m;
}

}  // namespace lba
