// Dense dL/dalpha of the shared-decay large-M path (eq. 9): sum over events
// of beta w_i K(t_i^-) into row m_i, from the bucketed event streams.
//
// Two kernels per chunk.  Column blocks are the buckets of W = 64 CPL nodes,
// row blocks the buckets of DR = 2^DRB nodes (tiles of 16 x 256 nodes, or
// 16 x 128 and 16 x 64 for chunks whose event indices need more key bits).
//   dense_ck     one wave per (column block, run of CKR segments): walks the
//                block's records of the run once, in groups of 64, and stores
//                the block's state K at the start of every window (NGW
//                groups: 64 or 128 records) and after the last one (a checkpoint:
//                W float64 values and the anchor time tau of the state,
//                K_q(tau) = sum over the events j of node q before the
//                window of e^{-beta (tau - t_j)}).  A run
//                starts from the scan's carry at its first segment, so the
//                runs are independent.  The same pass sums, per column and
//                run, the weights w_j (dL/dmu) and the compensator terms
//                1 - e^{-beta (T - t_j)} (their alpha-derivative).
//   large_dense  one wave per (row block, column block, event range of whole
//                runs).  Window g of a run holds the wave's own events (the
//                events of its row block) with index after window g-1's last
//                record and up to window g's last record (after the last
//                window: up to the run's end).  Own event k adds
//                beta w_k K(t_k^-) to row m_k, where K(t_k^-) is checkpoint g
//                decayed to t_k plus the window's records that precede k.
//                With c_k = beta w_k e^{-beta (t_k - tau_g)} and
//                b_j = e^{beta (t_j - tau_g)} the window adds
//                  u K_g^T, u_p = sum of c_k over its own events of row p
//                (a rank-1 update: DR x W float64 FMAs into G held in
//                registers, lane = column), and c_k b_j at (m_k, m_j) for the
//                window's records j before k (one masked ds_add_f64 per own
//                event and 64 records before it, into an LDS tile of pair
//                terms).  The pair terms cost a wave instruction per own
//                event and column block, so the wide tiles (fewer column
//                blocks) are the fast ones.  Where a 64-record window holds
//                few own events (u mostly zero), 128-record windows (NGW = 2)
//                halve the per-window work and the rank-1 updates per event
//                at about 1.5 pair instructions per own event.
// The state is shared through the checkpoints instead of being rebuilt by
// every row block.  Every window issues the same loads at the same point
// (the next window's checkpoint, column group and header, the next batch of
// own records), one window ahead, so their latency hides behind a window of
// work.  dense_ck writes each window's bounds into its slot's header (the
// window's last record, the record count, the next slot of the walk), so the
// window loop reads them (vector loads, made wave-uniform when the window
// starts) instead of tracking runs.
#include "hk_device.h"
#include "hk_large.h"
#include "hk_stream.h"

namespace hk {

#ifndef HK_CKW
#define HK_CKW 4   // waves per checkpoint workgroup (dense_ck)
#endif

// Checkpoint slots: window w (groups NGW w to NGW w + NGW - 1) of (column
// block sb, run r) uses slot (P0 >> log2(64 NGW)) + 2 (sb nrun + r) + w,
// with P0 the position of the run's first record in the column block's
// share of the DR-node partition; the slots of different (sb, r) never
// overlap, and there are at most (events) / (64 NGW) + 2 NBC nrun + 1.
// Checkpoint slot record, in float64 words: the state (W); the window's
// header (8 words: the anchor time, the time of the window's last record,
// then int32 the event index of that record, the record count (<= 64 NGW),
// the next slot of the column block's walk (-1: none), the run, whether the
// window is wide, beta (last record - anchor) > HK_WIDE, and the event index
// of its 65th record (INT_MAX if none)); the window's 64 NGW record times;
// its 64 NGW record keys (u32, two per word; in a written group of 64 the
// lanes past the records hold 0xffffffff; a second group is written only
// when the window has more than 64 records); then the records' factors
// e^{beta (t_j - tau)} against the window's anchor (float32, two per word,
// 0 past the records), formed once here instead of once per row block.
// Within each group of 64 the records are permuted over the lanes by LDS
// bank (dense_ck), so validity is read from the key, not the lane.  The slot after a run's last window
// has state and header only (count 0; its window runs to the run's end).
template <int CPL, int NGW>
struct Slot {
    static constexpr int W = 64 * CPL;
    static constexpr int NR = 64 * NGW;          // records per window
    static constexpr int TAU = W;
    static constexpr int T = W + 8;              // NR record times
    static constexpr int KEY = T + NR;           // NR keys (u32)
    static constexpr int BJ = KEY + NR / 2;      // NR factors (float32)
    static constexpr int SIZE = BJ + NR / 2;
    static_assert(SIZE == HK_SLOT_WORDS(CPL, NGW), "slot layout");
};

// One workgroup of NWC waves per (column block, run), in three phases.
// (1) Wave v compacts the keys of the column block's events among its
// quarter of the run's marks, in index order, into its own LDS region
// (record e of the run, in index order, sits in the region of the wave
// whose prefix of counts brackets e).  (2) In rounds of NWC groups of 64
// records, wave v takes group NWC rho + v: it writes the group's records
// into its window's slot (and the window's header at the window's last
// group), and stages per record its column, weight, compensator term and
// decay to the group's last record.  (3) After each round the state walks
// the round's groups in order, waves 0 .. CPL - 1 holding 64 columns each:
// a window's checkpoint at its first group, then the state decays to the
// group's last record and adds the group's staged records of its columns,
// as do the per-column sums of weights and compensator terms (so every sum
// is formed in the order of a single walk, whatever the waves' timing).  Runs r with the same r / 8 share an XCD (their
// column blocks read the same events).  runinfo[sb][r] = (first slot,
// groups, P0, P1), P0..P1 the run's positions in the column block's share
// of the DR-node partition.
template <int CPL, int DRB, int NGW, int NWC>
__global__ __launch_bounds__(64 * NWC) void dense_ck(int64_t c0, int32_t nev, int32_t M, int32_t NBC, int32_t NBO,
                                                     int32_t nrun, int32_t ckr, int32_t nseg, double T,
                                                     const double* __restrict__ t, const int32_t* __restrict__ marks,
                                                     const float* __restrict__ wchunk, const float* __restrict__ beta,
                                                     const double* __restrict__ carry_seg,
                                                     const double* __restrict__ gcarry,
                                                     const double* __restrict__ seg_offdec,
                                                     const int32_t* __restrict__ bo_off,
                                                     const int32_t* __restrict__ bo_base, double* __restrict__ kck,
                                                     int4* __restrict__ runinfo, double* __restrict__ spart,
                                                     double* __restrict__ cpart) {
    using S = Slot<CPL, NGW>;
    constexpr int W = S::W;
    constexpr int DR = 1 << DRB;
    constexpr int SH = CPL == 4 ? 8 : CPL == 2 ? 7 : 6;   // bits of the local mark in a record key
    constexpr int UB = 16;                 // batches of marks in flight
    static_assert((HK_CKR * HK_SEG) % (64 * NWC) == 0, "whole batches per wave's region");
    static_assert(NWC >= CPL, "a wave per 64 columns of the state");
    __shared__ double SL[W], CL[W], DLw[CPL][64];
    __shared__ double Fr[NWC], st_c[NWC][64];
    __shared__ int32_t st_col[NWC][64];
    __shared__ float st_w[NWC][64], st_f[NWC][64];
    __shared__ uint32_t keys[HK_CKR * HK_SEG];
    __shared__ int32_t wcnt[NWC];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int32_t x = (int32_t)(blockIdx.x & 7u), grp = (int32_t)(blockIdx.x >> 3);
    const int32_t sb = grp % NBC;
    const int32_t r = (grp / NBC) * 8 + x;
    const int32_t sA = r * ckr;
    if (sA >= nseg) return;   // the whole workgroup
    const int32_t sB = sA + ckr < nseg ? sA + ckr : nseg;
    for (int i = threadIdx.x; i < W; i += 64 * NWC) {
        SL[i] = 0.0;
        CL[i] = 0.0;
        (&DLw[0][0])[i] = 0.0;
    }
    const int32_t a = sA * HK_SEG;
    const int32_t b = sB * HK_SEG < nev ? sB * HK_SEG : nev;
    const int32_t s0 = sb * W;
    // the column block's DR-node blocks are consecutive in the partition
    const int32_t k0 = sb * (W / DR);
    const int32_t k1 = k0 + W / DR < NBO ? k0 + W / DR : NBO;
    int32_t P0 = bo_base[k0], P1 = bo_base[k0];
    for (int32_t k = k0; k < k1; ++k) {
        P0 += bo_off[(int64_t)k * (nseg + 1) + sA];
        P1 += bo_off[(int64_t)k * (nseg + 1) + sB];
    }
    const int32_t ng = (P1 - P0 + 63) >> 6;
    const int32_t slot0 = (P0 >> (NGW == 2 ? 7 : 6)) + 2 * (sb * nrun + r);   // one slot per window
    if (threadIdx.x == 0) runinfo[(int64_t)sb * nrun + r] = make_int4(slot0, ng, P0, P1);

    // (1) compaction: wave v takes the run's events [a + v PS, a + (v + 1) PS)
    // (PS a multiple of 64; the regions fit the key array since the run has
    // at most HK_CKR * HK_SEG events)
    const int32_t PS = ((b - a + 64 * NWC - 1) / (64 * NWC)) * 64;
    const int32_t pa = a + wv * PS;
    const int32_t pb = pa + PS < b ? pa + PS : b;
    uint32_t* kw = keys + wv * PS;
    int cnt = 0;
    for (int32_t base = pa; base < pb; base += 64 * UB) {
        int mk[UB];
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int32_t i = base + 64 * u + lane;
            mk[u] = i < pb ? clamp_mark(marks[c0 + i], M) : -1;
        }
#pragma unroll
        for (int u = 0; u < UB; ++u) {
            const int32_t i = base + 64 * u + lane;
            const bool sel = mk[u] >= s0 && mk[u] < s0 + W;
            const uint64_t bal = __ballot(sel);
            const int pos = cnt + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32),
                                                                 __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
            if (sel) kw[pos] = ((uint32_t)i << SH) | (uint32_t)(mk[u] - s0);
            cnt += __builtin_popcountll(bal);
        }
    }
    if (lane == 0) wcnt[wv] = cnt;
    __syncthreads();
    int32_t pre[NWC + 1];   // wave-uniform
    pre[0] = 0;
#pragma unroll
    for (int v = 0; v < NWC; ++v) pre[v + 1] = pre[v] + wcnt[v];
    const int32_t cntT = pre[NWC];
    // LDS position of record e (0 <= e < cntT)
    auto kpos = [&](int32_t e) -> int32_t {
        int32_t pos = e;
#pragma unroll
        for (int v = 1; v < NWC; ++v)
            if (e >= pre[v]) pos = v * PS + (e - pre[v]);
        return pos;
    };
    const double bet = (double)beta[0];
    const double bl2 = bet * HK_LOG2E;   // decays as powers of 2
    const double tau0 = c0 + a > 0 ? t[c0 + a - 1] : t[c0];
    // the time of record e (wave-uniform e), or tau0 before the first
    auto rec_t = [&](int32_t e) -> double { return e < 0 ? tau0 : t[c0 + (int32_t)(keys[kpos(e)] >> SH)]; };
    // the state: wave v < CPL holds columns s0 + 64 v + lane
    double K = 0.0;
    {
        const int32_t col = s0 + wv * 64 + lane;
        if (wv < CPL && col < M) {
            K = carry_seg[(int64_t)sA * 2 * M + col];
            // carry_seg as in-group prefixes (gcarry given): add the scan
            // group's carry moved to the run's first segment
            if (gcarry) K = __builtin_fma(seg_offdec[sA], gcarry[(int64_t)(sA / HK_SG) * 2 * M + col], K);
        }
    }
    // group g's records, with the state's time at the group's start (the
    // time of the record before it) and the anchor of its window (the state's
    // time at the window's first group), loaded a round ahead
    struct Rec {
        uint32_t key;
        double t;
        float w;
        double tg, tw;
    };
    auto load = [&](Rec& q, int32_t g) {
        const int32_t e = 64 * g + lane;
        q.key = e < cntT ? keys[kpos(e)] : 0xffffffffu;
        const int32_t i = e < cntT ? (int32_t)(q.key >> SH) : a;
        q.t = t[c0 + i];
        q.w = wchunk[i];
        q.tg = rec_t(64 * g - 1);
        q.tw = g % NGW == 0 ? q.tg : rec_t(64 * NGW * (g / NGW) - 1);
    };
    const double tl = cntT > 0 ? rec_t(cntT - 1) : tau0;   // the state's time after the last group
    // a checkpoint's state (this wave's 64 columns): float64, or float32 in
    // the first half of the state words for the 32-row kernel
    auto put_state = [&](int32_t slot, double K) {
        if constexpr (DRB >= 5)
            reinterpret_cast<float*>(kck + (int64_t)slot * S::SIZE)[wv * 64 + lane] = (float)K;
        else
            kck[(int64_t)slot * S::SIZE + wv * 64 + lane] = K;
    };
    // a window's header: anchor time, time and event index of the window's
    // last record (after the last window: the anchor and the run's last
    // event), record count, next slot (-1: none), run, wide flag, index of
    // the 65th record
    auto put_hdr = [&](int32_t w, double tw, double tcl, int32_t hi, int32_t nv, int32_t nxt, int32_t first1) {
        double* out = kck + (int64_t)(slot0 + w) * S::SIZE;
        if (lane == 0) {
            out[S::TAU] = tw;
            out[S::TAU + 1] = tcl;
            int32_t* h = reinterpret_cast<int32_t*>(out + S::TAU + 2);
            h[0] = hi;
            h[1] = nv;
            h[2] = nxt;
            h[3] = r;
            // a window with column records spans at most to its last record
            // (own events of index <= hi are not later): wide or not is known
            h[4] = nv > 0 && !(bet * (tcl - tw) <= HK_WIDE);
            h[5] = first1;
        }
    };
    Rec q;
    if (wv < ng) load(q, wv);
    for (int32_t g0 = 0; g0 < ng; g0 += NWC) {
        const int32_t g = g0 + wv;
        Rec qn;
        if (g + NWC < ng) load(qn, g + NWC);   // the next round's group in flight
        if (g < ng) {
            const int rem = cntT - 64 * g;
            const int nv = rem < 64 ? rem : 64;
            const bool v = lane < nv;
            const double tn = rl_d(q.t, nv - 1);
            const double tg = q.tg, tw = q.tw;
            const int32_t w = g / NGW, half = (g % NGW) * 64;
            if (half == 64 * (NGW - 1) || g + 1 == ng)
                put_hdr(w, tw, tn, (int32_t)((uint32_t)rl_i((int)q.key, nv - 1) >> SH), half + nv, slot0 + w + 1,
                        half != 0 ? (int32_t)((uint32_t)rl_i((int)q.key, 0) >> SH) : 0x7fffffff);
            double* out = kck + (int64_t)(slot0 + w) * S::SIZE;
            // The record's lane in the slot.  The dense kernel adds each own
            // event's pair terms with one LDS atomic over a group's 64
            // records, at the records' columns of one tile row; the LDS
            // serves 16 lanes of 8-byte words a cycle from 16 banks (column
            // mod 16), so records sharing a bank in one quarter-wave
            // serialise.  Records sorted by bank (past the records: last)
            // and dealt round-robin over the four quarter-waves share a
            // bank in a quarter only when more than four have it.  Nothing
            // else depends on the order (each lane carries its record's
            // index, column, time and factor).
            int pos;
            {
                // rank of the record in (bank, lane) order from bit-sliced
                // ballots: from the top bit down, the lanes that agree with
                // this lane's bank so far and have a 0 where it has a 1 are
                // smaller; the lanes left at the end share its bank
                const int bank = v ? (int)(q.key & 15u) : 16;
                const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
                uint64_t eq = ~0ull;
                int before = 0;
#pragma unroll
                for (int i = 4; i >= 0; --i) {
                    const uint64_t bi = __ballot((bank >> i) & 1);
                    const bool one = (bank >> i) & 1;
                    if (one) before += __builtin_popcountll(eq & ~bi);
                    eq &= one ? bi : ~bi;
                }
                const int sidx = before + __builtin_popcountll(eq & below);   // a permutation of 0..63
                pos = (sidx & 3) * 16 + (sidx >> 2);
            }
            out[S::T + half + pos] = v ? q.t : 0.0;
            reinterpret_cast<uint32_t*>(out + S::KEY)[half + pos] = q.key;
            // the record's factor e^{beta (t_j - tau_w)} against the window's anchor
            reinterpret_cast<float*>(out + S::BJ)[half + pos] = v ? exp2_f64arg((q.t - tw) * bl2) : 0.0f;
            if (lane == 0) Fr[wv] = (double)exp2_f64arg((tg - tn) * bl2);
            st_col[wv][lane] = v ? (int)(q.key & (uint32_t)(W - 1)) : -1;
            st_w[wv][lane] = q.w;
            st_f[wv][lane] = exp2_f64arg((q.t - tn) * bl2);
            st_c[wv][lane] = -expm1(-bet * (T - q.t));
        }
        __syncthreads();
        // (3) the state through the round's groups, in order
        if (wv < CPL) {
            for (int u = 0; u < NWC && g0 + u < ng; ++u) {
                const int32_t gg = g0 + u;
                if (gg % NGW == 0) put_state(slot0 + gg / NGW, K);
                K *= Fr[u];
                const int col = st_col[u][lane];
                if (col >= wv * 64 && col < wv * 64 + 64) {
                    atomicAdd(&DLw[wv][col - wv * 64], (double)st_f[u][lane]);
                    atomicAdd(&SL[col], (double)st_w[u][lane]);
                    atomicAdd(&CL[col], st_c[u][lane]);
                }
                lds_wait();   // the adds land before the read below
                K += DLw[wv][lane];
                DLw[wv][lane] = 0.0;
                lds_wait();   // and the clear before the next group's adds
            }
        }
        __syncthreads();
        q = qn;
    }
    // after the last group: the window up to the run's end, then the next
    // run's first slot (its P0 is this run's P1)
    const int32_t np = (ng + NGW - 1) / NGW;
    if (wv < CPL) put_state(slot0 + np, K);
    if (wv == 0)
        put_hdr(np, tl, tl, sB * HK_SEG - 1, 0,
                sB < nseg ? (P1 >> (NGW == 2 ? 7 : 6)) + 2 * (sb * nrun + r + 1) : -1, 0x7fffffff);
    for (int i = threadIdx.x; i < W; i += 64 * NWC) {
        const int32_t col = s0 + i;
        if (col < M) {
            spart[(int64_t)r * M + col] += SL[i];
            cpart[(int64_t)r * M + col] += CL[i];
        }
    }
}

// Raw buffer access with 32-bit byte offsets: no 64-bit address arithmetic,
// and reads past the buffer's size return 0 instead of touching memory.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf(const void* p, uint32_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}
__device__ __forceinline__ uint32_t ld_u32(__amdgpu_buffer_rsrc_t r, uint32_t i) {
    return __builtin_amdgcn_raw_buffer_load_b32(r, i * 4u, 0, 0);
}
__device__ __forceinline__ float ld_f32(__amdgpu_buffer_rsrc_t r, uint32_t i) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, i * 4u, 0, 0));
}
__device__ __forceinline__ double ld_f64(__amdgpu_buffer_rsrc_t r, uint32_t i) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, i * 8u, 0, 0));
}

// One batch of 64 consecutive own records (lane l: record qL + l).
struct OwnBatch {
    uint32_t key;
    double t;
    float w;
};

// Data of one window: the checkpoint's state and the window's column
// records.
template <int CPL, int NGW>
struct Win {
    double K[CPL];
    uint32_t ckey[NGW];   // records lane and 64 + lane of the window
    float bj[NGW];        // their e^{beta (t_j - tau)} (0 past the window's records)
};
// The same for the 32-row kernel, whose checkpoints keep the state in float32
// (the matrix cores take it in float32; the first half of the slot's state
// words holds it, so a window reads half the state bytes)
template <int CPL, int NGW>
struct WinF {
    float K[CPL];
    uint32_t ckey[NGW];
    float bj[NGW];
};

// a window's header (wave-uniform)
struct Hdr {
    double tau;   // the window's anchor (the slot also keeps its last record's time)
    int32_t hi, nv, next, run, wide, first1;
};

// A window's header as read by vector loads (every lane the same address)
// and made wave-uniform only when its window starts: a scalar load shares
// the LDS operations' wait counter, so while one is in flight every LDS wait
// of the window before would also wait for the header to arrive from memory.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
struct HdrV {
    u32x2 tau;   // the anchor's bits
    u32x4 a;     // hi, nv, next, run
    u32x2 b;     // wide, first1
};
template <class S>
__device__ __forceinline__ HdrV load_hdr_v(__amdgpu_buffer_rsrc_t r, int32_t slot) {
    const uint32_t o = ((uint32_t)slot * S::SIZE + S::TAU) * 8u;
    HdrV h;
    h.tau = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(r, o, 0, 0));
    h.a = __builtin_bit_cast(u32x4, __builtin_amdgcn_raw_buffer_load_b128(r, o + 16u, 0, 0));
    h.b = __builtin_bit_cast(u32x2, __builtin_amdgcn_raw_buffer_load_b64(r, o + 32u, 0, 0));
    return h;
}
__device__ __forceinline__ Hdr hdr_uniform(const HdrV& v) {
    auto rf = [](uint32_t x) { return __builtin_amdgcn_readfirstlane((int)x); };
    Hdr h;
    h.tau = __hiloint2double(rf(v.tau.y), rf(v.tau.x));
    h.hi = rf(v.a.x);
    h.nv = rf(v.a.y);
    h.next = rf(v.a.z);
    h.run = rf(v.a.w);
    h.wide = rf(v.b.x);
    h.first1 = rf(v.b.y);
    return h;
}

template <int CPL, int DRB, int NGW>
__global__ __launch_bounds__(64 * HK_DW) __attribute__((amdgpu_waves_per_eu((1 << DRB) * CPL > 32 ? 2 : 3))) void large_dense(int32_t M, int32_t NBC, int32_t NBR, int32_t ER, int32_t rpr,
                                                  int32_t nrun, int32_t ckr, int32_t nseg, int32_t nrec,
                                                  int32_t nslot, const float* __restrict__ beta,
                                                  const int4* __restrict__ runinfo,
                                                  const int32_t* __restrict__ bo_off,
                                                  const int32_t* __restrict__ bo_base,
                                                  const uint32_t* __restrict__ bo_key,
                                                  const double* __restrict__ bo_t, const float* __restrict__ bo_w,
                                                  const double* __restrict__ kck, double* __restrict__ gpart) {
    using S = Slot<CPL, NGW>;
    constexpr int W = S::W;
    constexpr int DR = 1 << DRB;
    constexpr int SH = CPL == 4 ? 8 : CPL == 2 ? 7 : 6;   // bits of the local mark in a column record key
    __shared__ double GP[DR * W];             // pair terms, shared by the group's waves
    __shared__ double ULs[HK_DW][DR];         // per wave: the window's u
    __shared__ double2 ODs[HK_DW][68];        // per wave: own events of a pass (+3 read ahead)
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    double* UL = ULs[wv];
    double2* OD = ODs[wv];
    const int32_t blk = blockIdx.x;
    const int32_t nbb = NBR * NBC;
    int32_t er, local;
    if (ER >= 8) {
        // blocks of one event range on one XCD (blockIdx % 8)
        const int32_t slot = blk >> 3;
        er = (slot / nbb) * 8 + (blk & 7);
        local = slot % nbb;
    } else {
        // 8 / ER XCDs share one event range
        const int32_t per = 8 / ER, x = blk & 7;
        er = x / per;
        local = (blk >> 3) * per + x % per;
        if (local >= nbb) return;
    }
    if (er >= ER) return;
    const int32_t nrun_c = (nseg + ckr - 1) / ckr;
    const int32_t gA = er * rpr;
    if (gA >= nrun_c) return;
    const int32_t gB = gA + rpr < nrun_c ? gA + rpr : nrun_c;
    // this wave's share of the range's runs (possibly none)
    const int32_t rA = gA + (wv * (gB - gA)) / HK_DW;
    const int32_t rB = gA + ((wv + 1) * (gB - gA)) / HK_DW;
    const int32_t sb = local % NBC;
    const int32_t rb = local / NBC;
    const int32_t r0 = rb * DR, s0 = sb * W;
    double* gp = gpart + (int64_t)er * M * M;
    // main terms of the block in registers (row i, column s0 + 64 j + lane),
    // wave 0 from the partials so far, the others from zero; branch-free
    // load, out-of-range rows/columns read a clamped valid address and are
    // zeroed
    double Gm[DR][CPL];
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const int32_t col = s0 + j * 64 + lane;
        const int32_t cc = col < M ? col : M - 1;
#pragma unroll
        for (int i = 0; i < DR; ++i) {
            const int32_t row = r0 + i;
            const int32_t rr = row < M ? row : M - 1;
            Gm[i][j] = wv == 0 ? gp[(int64_t)rr * M + cc] : 0.0;
        }
#pragma unroll
        for (int i = 0; i < DR; ++i) {
            if (!(r0 + i < M && col < M)) Gm[i][j] = 0.0;
            if (i % HK_DW == wv) GP[i * W + j * 64 + lane] = 0.0;
        }
    }
    if (lane < DR) UL[lane] = 0.0;
    const double bet = (double)beta[0];
    const double bl2 = bet * HK_LOG2E;   // decays as powers of 2
    const __amdgpu_buffer_rsrc_t rK = buf(kck, (uint32_t)nslot * S::SIZE * 8u);
    const __amdgpu_buffer_rsrc_t rOk = buf(bo_key, (uint32_t)nrec * 4u);
    const __amdgpu_buffer_rsrc_t rOt = buf(bo_t, (uint32_t)nrec * 8u);
    const __amdgpu_buffer_rsrc_t rOw = buf(bo_w, (uint32_t)nrec * 4u);
    const int4* rinf = runinfo + (int64_t)sb * nrun;
    // own stream: records [Q0, Q1) of row block rb, q the next unconsumed
    // one.  o0 holds records [qL, qL + 64).  Every window refills o2 from q
    // and first moves the previous window's o2 to o1, so o1 (from q1s) is
    // always one window old: when o0 runs out, o1 usually covers q.
    const int32_t sA = rA * ckr, sB = rB * ckr < nseg ? rB * ckr : nseg;
    const int32_t Q0 = bo_base[rb] + bo_off[(int64_t)rb * (nseg + 1) + sA];
    const int32_t Q1 = bo_base[rb] + bo_off[(int64_t)rb * (nseg + 1) + sB];
    auto own_load = [&](OwnBatch& o, int32_t from) {
        const uint32_t e = (uint32_t)(from + lane);
        o.key = ld_u32(rOk, e);
        o.t = ld_f64(rOt, e);
        o.w = ld_f32(rOw, e);
    };
    int32_t q = Q0, qL = Q0, q1s = Q0, q2s = Q0;
    OwnBatch o0, o1, o2;
    own_load(o0, Q0);
    own_load(o2, Q0);
    auto load_win = [&](Win<CPL, NGW>& w, int32_t slot) {
        const uint32_t sl = (uint32_t)slot * S::SIZE;
#pragma unroll
        for (int j = 0; j < CPL; ++j) w.K[j] = ld_f64(rK, sl + j * 64 + lane);
#pragma unroll
        for (int h = 0; h < NGW; ++h) {
            w.bj[h] = ld_f32(rK, 2 * (sl + S::BJ) + 64 * h + lane);
            w.ckey[h] = ld_u32(rK, 2 * (sl + S::KEY) + 64 * h + lane);
        }
    };
    // window headers by vector loads, made wave-uniform when their window
    // starts (a scalar load would make the window's LDS waits wait for it)
    auto load_hdr = [&](int32_t slot) -> HdrV { return load_hdr_v<S>(rK, slot); };

    int32_t sc = 0;   // the current window's slot
    Hdr hc;           // and its header
    // own records of the window in o0 from lane p on (index <= hi): adds
    // their c_k to u and their pair terms to GP; returns how many there were
    auto pass = [&](const Win<CPL, NGW>& w, int p, double tw, int hi, bool cv0, bool cv1, int cidx0, int cidx1,
                    int colj0, int colj1, double bj0, double bj1) -> int {
        const OwnBatch& b = o0;
        const bool own = qL + lane < Q1 && lane >= p && (int)(b.key >> DRB) <= hi;
        const int nsel = __builtin_popcountll(__ballot(own));
        if (nsel == 0) return 0;
        const int kend = p + nsel;   // own lanes are [p, kend)
        // windows with column records: the header's flag; after a run's last
        // group: from the last selected own event
        bool narrow;
        if (hc.nv > 0) {
            narrow = hc.wide == 0;
        } else {
            const double tlo = rl_d(b.t, kend - 1);
            narrow = bet * (tlo - tw) <= HK_WIDE;
        }
        const int rowl = (int)(b.key & (DR - 1));
        if (narrow) {
            const float cf = own ? (float)(bet * (double)b.w) * exp2_f64arg((tw - b.t) * bl2) : 0.0f;
            if (own) {
                atomicAdd(&UL[rowl], (double)cf);
                // (row offset, index, c_k) of this own event for the pair
                // loop, read back by every lane (broadcast)
                OD[lane] = make_double2(__hiloint2double(rowl * W, (int)(b.key >> DRB)), (double)cf);
            }
            // pair terms: own event k adds c_k b_j at (row_k, m_j) for the
            // window's records j before it (zero elsewhere)
            // (the window's second 64 records only for an own event after the
            // first of them; the own events are in index order, so those
            // before it are the first kmid - p of the pass, and an own event
            // after it follows all 64 records of the full first group)
            auto pair1 = [&](const double2 od) {
                const int rofs = __double2hiint(od.x), ik = __double2loint(od.x);
                if (cidx0 < ik) atomicAdd(&GP[rofs + colj0], od.y * bj0);
            };
            auto pair2 = [&](const double2 od) {
                const int rofs = __double2hiint(od.x), ik = __double2loint(od.x);
                atomicAdd(&GP[rofs + colj0], od.y * bj0);
                if (cidx1 < ik) atomicAdd(&GP[rofs + colj1], od.y * bj1);
            };
            const int kmid = NGW == 2 ? p + __builtin_popcountll(__ballot(own && (int)(b.key >> DRB) <= hc.first1))
                                      : kend;
            // entries [ka, kb), two at a time, the next two read before this
            // pair's atomics (unrolled by two so that the entries read ahead
            // need no register moves; entries up to kb + 2 are read, those
            // past kb not used)
            auto run = [&](int ka, int kb, auto&& pf) __attribute__((always_inline)) {
                if (ka >= kb) return;
                double2 d1 = OD[ka], d2 = OD[ka + 1];
                for (int k = ka;; k += 4) {
                    const double2 n1 = OD[k + 2], n2 = OD[k + 3];
                    pf(d1);
                    if (k + 1 < kb) pf(d2);
                    if (k + 2 >= kb) break;
                    d1 = OD[k + 4];
                    d2 = OD[k + 5];
                    pf(n1);
                    if (k + 3 < kb) pf(n2);
                    if (k + 4 >= kb) break;
                }
            };
            run(p, kmid, pair1);
            if (NGW == 2) run(kmid, kend, pair2);
        } else {
            // wide window (anchored factors would leave float32 range):
            // c_k decayed from the window's anchor (below float32 range it
            // is zero, and so is its product with the state), exact
            // per-pair decays
            const double cw = bet * (double)b.w;
            if (own) atomicAdd(&UL[rowl], cw * (double)exp2_f64arg((tw - b.t) * bl2));
            // the records' times, waited for here so that no load of this
            // rare path stays in flight
            const double ct0 = ld_f64(rK, (uint32_t)sc * S::SIZE + S::T + lane);
            const double ct1 = NGW == 2 ? ld_f64(rK, (uint32_t)sc * S::SIZE + S::T + 64 + lane) : 0.0;
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
            for (int k = p; k < kend; ++k) {
                const uint32_t key = (uint32_t)rl_i((int)b.key, k);
                const int rofs = (int)(key & (DR - 1)) * W;
                const double tk = rl_d(b.t, k);
                const double ck = rl_d(cw, k);
                if (cv0 && cidx0 < (int)(key >> DRB))
                    atomicAdd(&GP[rofs + colj0], ck * (double)exp2_f64arg((ct0 - tk) * bl2));
                if (NGW == 2 && cv1 && cidx1 < (int)(key >> DRB))
                    atomicAdd(&GP[rofs + colj1], ck * (double)exp2_f64arg((ct1 - tk) * bl2));
            }
        }
        return nsel;
    };

    // the current window: slot sc with header hc; each window loads the next
    // one's data and header first (the same window again after the wave's
    // last one, so that every window issues the same loads)
    auto body = [&](Win<CPL, NGW>& cur, Win<CPL, NGW>& nxt) -> bool {
        const bool last = hc.nv == 0 && hc.run >= rB - 1;
        const int32_t sn = last ? sc : hc.next;
        load_win(nxt, sn);
        const HdrV hn = load_hdr(sn);
        o1 = o2;
        q1s = q2s;
        own_load(o2, q);
        q2s = q;

        const int nv = hc.nv;
        const int hi = hc.hi;
        const double tw = hc.tau;
        // records are permuted within their group: valid lanes by key
        const bool cv0 = nv > 0 && cur.ckey[0] != 0xffffffffu;
        const bool cv1 = NGW == 2 && nv > 64 && cur.ckey[NGW - 1] != 0xffffffffu;
        const int cidx0 = cv0 ? (int)(cur.ckey[0] >> SH) : 0x7fffffff;
        const int cidx1 = cv1 ? (int)(cur.ckey[NGW - 1] >> SH) : 0x7fffffff;
        const int colj0 = (int)(cur.ckey[0] & (uint32_t)(W - 1));
        const int colj1 = (int)(cur.ckey[NGW - 1] & (uint32_t)(W - 1));
        const double bj0 = (double)cur.bj[0], bj1 = (double)cur.bj[NGW - 1];
        int nown = 0;
        for (;;) {
            if (q - qL == 64) {
                // o0 used up: continue in o1, which covers q unless more than
                // 64 records went by in two windows (q >= q1s always); then
                // load o1 now and wait for it here, so that the other path
                // sees no load in flight
                if (q >= q1s + 64) {
                    own_load(o1, q);
                    q1s = q;
                    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
                }
                o0 = o1;
                qL = q1s;
            }
            const int n = pass(cur, q - qL, tw, hi, cv0, cv1, cidx0, cidx1, colj0, colj1, bj0, bj1);
            q += n;
            nown += n;
            if (n == 0 || q - qL < 64) break;
        }
        if (nown) {
            // rank-1 update G += u K_g^T, then clear u (u is this wave's;
            // its atomics on u land before the reads)
            lds_wait();
            double u[DR];
#pragma unroll
            for (int i = 0; i < DR; ++i) u[i] = UL[i];
#pragma unroll
            for (int i = 0; i < DR; ++i)
#pragma unroll
                for (int j = 0; j < CPL; ++j) Gm[i][j] = __builtin_fma(u[i], cur.K[j], Gm[i][j]);
            __builtin_amdgcn_wave_barrier();
            if (lane < DR) UL[lane] = 0.0;
            __builtin_amdgcn_wave_barrier();
        }
        sc = sn;
        hc = hdr_uniform(hn);
        return !last;
    };

    __syncthreads();
    if (rA < rB) {
        sc = rinf[rA].x;   // the first slot of the wave's first run
        hc = hdr_uniform(load_hdr(sc));
        Win<CPL, NGW> wa, wb;
        load_win(wa, sc);
        for (;;) {
            if (!body(wa, wb)) break;
            if (!body(wb, wa)) break;
        }
    }
    // the group's sum: the other waves add their main terms to the pair
    // tile, wave 0 writes its own plus the tile
    __syncthreads();
    if (wv != 0) {
#pragma unroll
        for (int i = 0; i < DR; ++i)
#pragma unroll
            for (int j = 0; j < CPL; ++j) atomicAdd(&GP[i * W + j * 64 + lane], Gm[i][j]);
    }
    __syncthreads();
    if (wv != 0) return;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const int32_t col = s0 + j * 64 + lane;
        if (col < M) {
#pragma unroll
            for (int rr = 0; rr < DR; ++rr) {
                const int32_t row = r0 + rr;
                if (row < M) gp[(int64_t)row * M + col] = Gm[rr][j] + GP[rr * W + j * 64 + lane];
            }
        }
    }
}

// The same dense dL/dalpha for tiles of 32 x 256 at large M: the rank-1
// part of each window (u K_g^T, a 32 x 256 outer product) runs on the matrix
// cores as four float32 MFMAs (one per 64 columns, two 32 x 32 blocks each)
// into float32 accumulators, added to the workgroup's float64 LDS tile every
// HK_FLUSH windows that had own events, and at the end; the tile also takes
// the pair terms and starts from the event range's float64 partials; the
// checkpoints keep this layout's state in float32, the form the matrix cores
// take.  Twice the rows per tile
// halve the window visits per event (the per-window loads, header and
// bookkeeping) at the same register count; NWV waves share the tile.
// float32 partial sums over at most HK_FLUSH windows, float64 beyond (the
// float32 state of the precision plan, float64 reductions).
// HK_FLUSH: 256 windows, more than a wave visits in one launch at c4's
// chunks of 2^20 events (about 150), so there the accumulators are flushed
// once, at the end; longer chunks flush every 256 windows (measured at c4,
// dense ms per step with 16 / 32 / 64: 3.89 / 3.77 / 3.69 in an earlier form
// of the kernel, and with 64 / 128 / 256 now: 3.33 / 3.31 / 3.28;
// dL/dalpha's error against the oracle at theta_pert on all 1e7 events
// 4.1e-8 at 16, 4.9e-8 at 64, 6.6e-8 at 256)
#ifndef HK_FLUSH
#define HK_FLUSH 256
#endif
template <int CPL, int DRB, int NGW, int NWV>
__global__ __launch_bounds__(64 * NWV) __attribute__((amdgpu_waves_per_eu(2))) void large_dense_f(int32_t M, int32_t NBC, int32_t NBR, int32_t ER, int32_t rpr,
                                                  int32_t nrun, int32_t ckr, int32_t nseg, int32_t nrec,
                                                  int32_t nslot, const float* __restrict__ beta,
                                                  const int4* __restrict__ runinfo,
                                                  const int32_t* __restrict__ bo_off,
                                                  const int32_t* __restrict__ bo_base,
                                                  const uint32_t* __restrict__ bo_key,
                                                  const double* __restrict__ bo_t, const float* __restrict__ bo_w,
                                                  const double* __restrict__ kck, double* __restrict__ gpart) {
    using S = Slot<CPL, NGW>;
    constexpr int W = S::W;
    constexpr int DR = 1 << DRB;
    constexpr int SH = CPL == 4 ? 8 : CPL == 2 ? 7 : 6;   // bits of the local mark in a column record key
    extern __shared__ double GP[];            // [DR * W] float64 tile, shared by the group's waves
    __shared__ double ULs[NWV][DR];           // per wave: the window's u (float64: LDS float32 atomics are slow)
    __shared__ double2 ODs[NWV][68];          // per wave: own events of a pass (+3 read ahead)
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    double* UL = ULs[wv];
    double2* OD = ODs[wv];
    const int32_t blk = blockIdx.x;
    const int32_t nbb = NBR * NBC;
    int32_t er, local;
    if (ER >= 8) {
        // blocks of one event range on one XCD (blockIdx % 8)
        const int32_t slot = blk >> 3;
        er = (slot / nbb) * 8 + (blk & 7);
        local = slot % nbb;
    } else {
        // 8 / ER XCDs share one event range
        const int32_t per = 8 / ER, x = blk & 7;
        er = x / per;
        local = (blk >> 3) * per + x % per;
        if (local >= nbb) return;
    }
    if (er >= ER) return;
    const int32_t nrun_c = (nseg + ckr - 1) / ckr;
    const int32_t gA = er * rpr;
    if (gA >= nrun_c) return;
    const int32_t gB = gA + rpr < nrun_c ? gA + rpr : nrun_c;
    // this wave's share of the range's runs (possibly none)
    const int32_t rA = gA + (wv * (gB - gA)) / NWV;
    const int32_t rB = gA + ((wv + 1) * (gB - gA)) / NWV;
    const int32_t sb = local % NBC;
    const int32_t rb = local / NBC;
    const int32_t r0 = rb * DR, s0 = sb * W;
    double* gp = gpart + (int64_t)er * M * M;
    // the tile starts from the event range's partials so far (coalesced:
    // a row of W columns per 64 NWV threads), zero outside the matrix
    for (int x = threadIdx.x; x < DR * W; x += 64 * NWV) {
        const int32_t row = r0 + x / W, col = s0 + x % W;
        GP[x] = row < M && col < M ? gp[(int64_t)row * M + col] : 0.0;
    }
    // the rank-1 part in float32 matrix-core accumulators: for column group
    // j (tile columns 64 j .. 64 j + 63), v_mfma_f32_32x32x1_2b_f32 adds the
    // outer products of u (rows 0..31, the A operand of both blocks: lane l
    // holds u[l mod 32]) with the state of columns 64 j + l (the B operand:
    // lanes 0..31 block 0, lanes 32..63 block 1).  Result register r of
    // lane l holds row 8 ((r mod 16) / 4) + 4 (l / 32) + r mod 4 of column
    // 64 j + 32 (r / 16) + l mod 32 (layout measured on the device).
    static_assert(DR == 32 && CPL == 4, "32 x 256 tiles");
    typedef float f32x32 __attribute__((ext_vector_type(32)));
    f32x32 acc0 = {}, acc1 = {}, acc2 = {}, acc3 = {};
    int nacc = 0;   // windows added to the accumulators since their last flush
    auto flush1 = [&](f32x32& a, int j) __attribute__((always_inline)) {
#pragma unroll
        for (int r = 0; r < 32; ++r) {
            const int row = 8 * ((r & 15) >> 2) + 4 * (lane >> 5) + (r & 3);
            const int col = 64 * j + 32 * (r >> 4) + (lane & 31);
            atomicAdd(&GP[row * W + col], (double)a[r]);
        }
        a = f32x32{};
    };
    auto flush = [&]() __attribute__((always_inline)) {
        flush1(acc0, 0);
        flush1(acc1, 1);
        flush1(acc2, 2);
        flush1(acc3, 3);
    };
    if (lane < DR) UL[lane] = 0.0;
    const double bet = (double)beta[0];
    const double bl2 = bet * HK_LOG2E;   // decays as powers of 2
    const __amdgpu_buffer_rsrc_t rK = buf(kck, (uint32_t)nslot * S::SIZE * 8u);
    const __amdgpu_buffer_rsrc_t rOk = buf(bo_key, (uint32_t)nrec * 4u);
    const __amdgpu_buffer_rsrc_t rOt = buf(bo_t, (uint32_t)nrec * 8u);
    const __amdgpu_buffer_rsrc_t rOw = buf(bo_w, (uint32_t)nrec * 4u);
    const int4* rinf = runinfo + (int64_t)sb * nrun;
    // own stream: records [Q0, Q1) of row block rb, q the next unconsumed
    // one.  o0 holds records [qL, qL + 64).  Every window refills o2 from q
    // and first moves the previous window's o2 to o1, so o1 (from q1s) is
    // always one window old: when o0 runs out, o1 usually covers q.
    const int32_t sA = rA * ckr, sB = rB * ckr < nseg ? rB * ckr : nseg;
    const int32_t Q0 = bo_base[rb] + bo_off[(int64_t)rb * (nseg + 1) + sA];
    const int32_t Q1 = bo_base[rb] + bo_off[(int64_t)rb * (nseg + 1) + sB];
    auto own_load = [&](OwnBatch& o, int32_t from) {
        const uint32_t e = (uint32_t)(from + lane);
        o.key = ld_u32(rOk, e);
        o.t = ld_f64(rOt, e);
        o.w = ld_f32(rOw, e);
    };
    int32_t q = Q0, qL = Q0, q1s = Q0, q2s = Q0;
    OwnBatch o0, o1, o2;
    own_load(o0, Q0);
    own_load(o2, Q0);
    auto load_win = [&](WinF<CPL, NGW>& w, int32_t slot) {
        const uint32_t sl = (uint32_t)slot * S::SIZE;
#pragma unroll
        for (int j = 0; j < CPL; ++j) w.K[j] = ld_f32(rK, 2 * sl + j * 64 + lane);
#pragma unroll
        for (int h = 0; h < NGW; ++h) {
            w.bj[h] = ld_f32(rK, 2 * (sl + S::BJ) + 64 * h + lane);
            w.ckey[h] = ld_u32(rK, 2 * (sl + S::KEY) + 64 * h + lane);
        }
    };
    // window headers by vector loads, made wave-uniform when their window
    // starts (a scalar load would make the window's LDS waits wait for it)
    auto load_hdr = [&](int32_t slot) -> HdrV { return load_hdr_v<S>(rK, slot); };

    int32_t sc = 0;   // the current window's slot
    Hdr hc;           // and its header
    // own records of the window in o0 from lane p on (index <= hi): adds
    // their c_k to u and their pair terms to GP; returns how many there were
    auto pass = [&](const WinF<CPL, NGW>& w, int p, double tw, int hi, bool cv0, bool cv1, int cidx0, int cidx1,
                    int colj0, int colj1, double bj0, double bj1) -> int {
        const OwnBatch& b = o0;
        const bool own = qL + lane < Q1 && lane >= p && (int)(b.key >> DRB) <= hi;
        const int nsel = __builtin_popcountll(__ballot(own));
        if (nsel == 0) return 0;
        const int kend = p + nsel;   // own lanes are [p, kend)
        // windows with column records: the header's flag; after a run's last
        // group: from the last selected own event
        bool narrow;
        if (hc.nv > 0) {
            narrow = hc.wide == 0;
        } else {
            const double tlo = rl_d(b.t, kend - 1);
            narrow = bet * (tlo - tw) <= HK_WIDE;
        }
        const int rowl = (int)(b.key & (DR - 1));
        if (narrow) {
            const float cf = own ? (float)(bet * (double)b.w) * exp2_f64arg((tw - b.t) * bl2) : 0.0f;
            if (own) {
                atomicAdd(&UL[rowl], (double)cf);
                // (row offset, index, c_k) of this own event for the pair
                // loop, read back by every lane (broadcast)
                OD[lane] = make_double2(__hiloint2double(rowl * W, (int)(b.key >> DRB)), (double)cf);
            }
            // pair terms: own event k adds c_k b_j at (row_k, m_j) for the
            // window's records j before it (zero elsewhere); the window's
            // second 64 records only for an own event after the first of
            // them.  The own events are in index order, so those before it
            // are the first kmid - p of the pass: two loops, no test per event
            auto pair1 = [&](const double2 od) {
                const int rofs = __double2hiint(od.x), ik = __double2loint(od.x);
                if (cidx0 < ik) atomicAdd(&GP[rofs + colj0], od.y * bj0);
            };
            // (an own event after the second group's first record follows
            // all 64 records of the first group, which is full whenever a
            // second one exists: its first atomic needs no mask)
            auto pair2 = [&](const double2 od) {
                const int rofs = __double2hiint(od.x), ik = __double2loint(od.x);
                atomicAdd(&GP[rofs + colj0], od.y * bj0);
                if (cidx1 < ik) atomicAdd(&GP[rofs + colj1], od.y * bj1);
            };
            const int kmid = NGW == 2 ? p + __builtin_popcountll(__ballot(own && (int)(b.key >> DRB) <= hc.first1))
                                      : kend;
            // entries [ka, kb), two at a time, the next two read before this
            // pair's atomics (unrolled by two so that the entries read ahead
            // need no register moves; entries up to kb + 2 are read, those
            // past kb not used)
            auto run = [&](int ka, int kb, auto&& pf) __attribute__((always_inline)) {
                if (ka >= kb) return;
                double2 d1 = OD[ka], d2 = OD[ka + 1];
                for (int k = ka;; k += 4) {
                    const double2 n1 = OD[k + 2], n2 = OD[k + 3];
                    pf(d1);
                    if (k + 1 < kb) pf(d2);
                    if (k + 2 >= kb) break;
                    d1 = OD[k + 4];
                    d2 = OD[k + 5];
                    pf(n1);
                    if (k + 3 < kb) pf(n2);
                    if (k + 4 >= kb) break;
                }
            };
            run(p, kmid, pair1);
            if (NGW == 2) run(kmid, kend, pair2);
        } else {
            // wide window (anchored factors would leave float32 range):
            // c_k decayed from the window's anchor (below float32 range it
            // is zero, and so is its product with the state), exact
            // per-pair decays
            const double cw = bet * (double)b.w;
            if (own) atomicAdd(&UL[rowl], cw * (double)exp2_f64arg((tw - b.t) * bl2));
            // the records' times, waited for here so that no load of this
            // rare path stays in flight
            const double ct0 = ld_f64(rK, (uint32_t)sc * S::SIZE + S::T + lane);
            const double ct1 = NGW == 2 ? ld_f64(rK, (uint32_t)sc * S::SIZE + S::T + 64 + lane) : 0.0;
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
            for (int k = p; k < kend; ++k) {
                const uint32_t key = (uint32_t)rl_i((int)b.key, k);
                const int rofs = (int)(key & (DR - 1)) * W;
                const double tk = rl_d(b.t, k);
                const double ck = rl_d(cw, k);
                if (cv0 && cidx0 < (int)(key >> DRB))
                    atomicAdd(&GP[rofs + colj0], ck * (double)exp2_f64arg((ct0 - tk) * bl2));
                if (NGW == 2 && cv1 && cidx1 < (int)(key >> DRB))
                    atomicAdd(&GP[rofs + colj1], ck * (double)exp2_f64arg((ct1 - tk) * bl2));
            }
        }
        return nsel;
    };

    // the current window: slot sc with header hc; each window loads the next
    // one's data and header first (the same window again after the wave's
    // last one, so that every window issues the same loads)
    auto body = [&](WinF<CPL, NGW>& cur, WinF<CPL, NGW>& nxt) -> bool {
        const bool last = hc.nv == 0 && hc.run >= rB - 1;
        const int32_t sn = last ? sc : hc.next;
        load_win(nxt, sn);
        const HdrV hn = load_hdr(sn);
        o1 = o2;
        q1s = q2s;
        own_load(o2, q);
        q2s = q;

        const int nv = hc.nv;
        const int hi = hc.hi;
        const double tw = hc.tau;
        // records are permuted within their group: valid lanes by key
        const bool cv0 = nv > 0 && cur.ckey[0] != 0xffffffffu;
        const bool cv1 = NGW == 2 && nv > 64 && cur.ckey[NGW - 1] != 0xffffffffu;
        const int cidx0 = cv0 ? (int)(cur.ckey[0] >> SH) : 0x7fffffff;
        const int cidx1 = cv1 ? (int)(cur.ckey[NGW - 1] >> SH) : 0x7fffffff;
        const int colj0 = (int)(cur.ckey[0] & (uint32_t)(W - 1));
        const int colj1 = (int)(cur.ckey[NGW - 1] & (uint32_t)(W - 1));
        const double bj0 = (double)cur.bj[0], bj1 = (double)cur.bj[NGW - 1];
        int nown = 0;
        for (;;) {
            if (q - qL == 64) {
                // o0 used up: continue in o1, which covers q unless more than
                // 64 records went by in two windows (q >= q1s always); then
                // load o1 now and wait for it here, so that the other path
                // sees no load in flight
                if (q >= q1s + 64) {
                    own_load(o1, q);
                    q1s = q;
                    __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0)
                }
                o0 = o1;
                qL = q1s;
            }
            const int n = pass(cur, q - qL, tw, hi, cv0, cv1, cidx0, cidx1, colj0, colj1, bj0, bj1);
            q += n;
            nown += n;
            if (n == 0 || q - qL < 64) break;
        }
        if (nown) {
            // rank-1 update G += u K_g^T on the matrix cores (float32), then
            // clear u (u is this wave's; its atomics on u land before the reads)
            lds_wait();
            const float uv = (float)UL[lane & 31];
            acc0 = __builtin_amdgcn_mfma_f32_32x32x1f32(uv, cur.K[0], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f32_32x32x1f32(uv, cur.K[1], acc1, 0, 0, 0);
            acc2 = __builtin_amdgcn_mfma_f32_32x32x1f32(uv, cur.K[2], acc2, 0, 0, 0);
            acc3 = __builtin_amdgcn_mfma_f32_32x32x1f32(uv, cur.K[3], acc3, 0, 0, 0);
            __builtin_amdgcn_wave_barrier();
            if (lane < DR) UL[lane] = 0.0;
            __builtin_amdgcn_wave_barrier();
            if (++nacc == HK_FLUSH) {
                flush();
                nacc = 0;
            }
        }
        sc = sn;
        hc = hdr_uniform(hn);
        return !last;
    };

    __syncthreads();
    if (rA < rB) {
        sc = rinf[rA].x;   // the first slot of the wave's first run
        hc = hdr_uniform(load_hdr(sc));
        WinF<CPL, NGW> wa, wb;
        load_win(wa, sc);
        for (;;) {
            if (!body(wa, wb)) break;
            if (!body(wb, wa)) break;
        }
    }
    // every wave adds what its registers hold to the tile, which then goes
    // back to the event range's partials
    if (nacc) flush();
    __syncthreads();
    for (int x = threadIdx.x; x < DR * W; x += 64 * NWV) {
        const int32_t row = r0 + x / W, col = s0 + x % W;
        if (row < M && col < M) gp[(int64_t)row * M + col] = GP[x];
    }
}

template <int CPL, int DRB, int NGW>
static void dense_launch_t(LargeArgs& A, int64_t c0, int32_t nev, int32_t nseg, int32_t nrun_c, hipStream_t st,
                           bool ck_only) {
    {
        TimedScope tk(7, st);
        const unsigned nck = (unsigned)(((nrun_c + 7) / 8) * 8 * A.NBC);
        hipLaunchKernelGGL((dense_ck<CPL, DRB, NGW, HK_CKW>), dim3(nck), dim3(64 * HK_CKW), 0, st, c0, nev, A.M, A.NBC,
                           A.NBO, A.NRUN,
                           A.CKR, nseg, A.T, A.t, A.marks, A.wchunk, A.beta, A.carry_seg,
                           A.carry_prefix ? A.gcarry : (const double*)nullptr, A.seg_offdec, A.bo_off, A.bo_base,
                           A.kck, A.runinfo, A.spart, A.cpart_);
    }
    if (ck_only) return;
    TimedScope ts(0, st);
    const int32_t rpr = A.NRUN / A.ER;   // runs per event range (both powers of two)
    const int32_t nbb = A.NBR * A.NBC;
    const unsigned nblk = A.ER >= 8 ? (unsigned)(nbb * ((A.ER + 7) / 8) * 8)
                                    : (unsigned)(((nbb + 8 / A.ER - 1) / (8 / A.ER)) * 8);
    if constexpr (DRB >= 5) {
        hipLaunchKernelGGL((large_dense_f<CPL, DRB, NGW, HK_DWF>), dim3(nblk), dim3(64 * HK_DWF),
                           (size_t)(1 << DRB) * 64 * CPL * sizeof(double), st, A.M, A.NBC, A.NBR, A.ER, rpr, A.NRUN,
                           A.CKR, nseg, nev, (int32_t)A.nslot, A.beta, A.runinfo, A.bo_off, A.bo_base, A.bo_key,
                           A.bo_t, A.bo_w, A.kck, A.gpart);
    } else {
        hipLaunchKernelGGL((large_dense<CPL, DRB, NGW>), dim3(nblk), dim3(64 * HK_DW), 0, st, A.M, A.NBC, A.NBR, A.ER,
                           rpr, A.NRUN, A.CKR, nseg, nev, (int32_t)A.nslot, A.beta, A.runinfo, A.bo_off, A.bo_base,
                           A.bo_key, A.bo_t, A.bo_w, A.kck, A.gpart);
    }
}

// dynamic LDS of the float32-accumulator dense kernel (its float64 tile):
// granted once per kernel and device above 64 KiB
hawkes_status dense_allow_lds(const LargeArgs& A) {
    if (A.DRB < 5) return HAWKES_OK;
    const size_t bytes = (size_t)(1 << A.DRB) * 64 * A.CPL * sizeof(double);
    return allow_lds((const void*)large_dense_f<4, 5, 2, HK_DWF>, bytes, true);
}

void large_dense_launch(LargeArgs& A, int64_t c0, int64_t c1, int32_t nseg, hipStream_t st, bool ck_only) {
    const int32_t nrun_c = (nseg + A.CKR - 1) / A.CKR;
    const int32_t nev = (int32_t)(c1 - c0);
    // the tiles the layout selects: 16 x 256, 16 x 128, 16 x 64
    // and the window length the layout selects (A.NGW groups of 64 records)
    if (A.DRB == 5) {
        // the layout selects 32-row tiles only with 256 columns and 128-record windows
        dense_launch_t<4, 5, 2>(A, c0, nev, nseg, nrun_c, st, ck_only);
    } else if (A.NGW == 2) {
        if (A.CPL == 4)
            dense_launch_t<4, 4, 2>(A, c0, nev, nseg, nrun_c, st, ck_only);
        else if (A.CPL == 2)
            dense_launch_t<2, 4, 2>(A, c0, nev, nseg, nrun_c, st, ck_only);
        else
            dense_launch_t<1, 4, 2>(A, c0, nev, nseg, nrun_c, st, ck_only);
    } else {
        if (A.CPL == 4)
            dense_launch_t<4, 4, 1>(A, c0, nev, nseg, nrun_c, st, ck_only);
        else if (A.CPL == 2)
            dense_launch_t<2, 4, 1>(A, c0, nev, nseg, nrun_c, st, ck_only);
        else
            dense_launch_t<1, 4, 1>(A, c0, nev, nseg, nrun_c, st, ck_only);
    }
}

}  // namespace hk
