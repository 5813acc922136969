// Small-M engine (M <= 8): exact Hawkes log-likelihood and gradient for one
// or many independent sequences, shared decay per sequence.
//
// Each lane owns one "item": a run of at most L consecutive events of one
// sequence.  The full node state lives in the lane's registers in float64:
//   K_q(t) = sum_{j<i, m_j=q} e^{-beta (t - t_j)}          (eq. 11 state)
//   J_q(t) = sum_{j<i, m_j=q} (t - t_j) e^{-beta (t - t_j)} (time-weighted;
//            equal to t K - L with the paper's L of eq. 12)
// and R = alpha_{p,:} . K is the state of eq. 3 for target p.
//
// Three phases make the per-lane recurrence a parallel scan (the prefix scan
// of affine maps of "Methods"; a run of events acts on (K, J) as
//   K -> e^{-beta D} K + K_run,  J -> e^{-beta D} (J + D K) + J_run,
// a map of the paper's (s I, v) form extended by the shear D K):
//   A  each lane folds its item into such a map (span D, K_run, J_run); the
//      wave then runs a segmented inclusive scan of the 64 maps (a new
//      sequence resets the state);
//   B  one thread per (sequence, node) chains the per-wave aggregates of its
//      sequence in order;
//   C  each lane rebuilds its carry-in from (B) and its in-wave prefix and
//      replays its events, forming lambda_i, log lambda_i, 1/lambda_i and the
//      gradient sums of eqs. 8-10, written as per-item float64 partials;
//   R  per-sequence reduction of the partials in a fixed order.
#include "hk_device.h"
#include "hk_internal.h"

namespace hk {

// ---------------------------------------------------------------- setup
// One workgroup of 1024 threads: exclusive scans over the sequences of
//   item counts ceil(len/L), reduction-chunk counts ceil(items/RCH),
//   node counts m_s and m_s^2 (parameter packing offsets).
// event range of sequence s clamped to [0, n_total) so that malformed offsets
// can never address outside t / marks
__device__ __forceinline__ void seq_range(const int64_t* __restrict__ ev_off, int32_t s, int64_t n_total,
                                          int64_t* e0, int64_t* e1) {
    int64_t a = ev_off[s], b = ev_off[s + 1];
    a = a < 0 ? 0 : (a > n_total ? n_total : a);
    b = b < a ? a : (b > n_total ? n_total : b);
    *e0 = a;
    *e1 = b;
}

__global__ __launch_bounds__(1024) void small_setup(int32_t S, int64_t n_total, const int64_t* __restrict__ ev_off,
                                                    const int32_t* __restrict__ m_s, int32_t L,
                                                    int64_t* __restrict__ item_off,
                                                    int64_t* __restrict__ chunk_off,
                                                    int64_t* __restrict__ mu_off,
                                                    int64_t* __restrict__ a_off) {
    __shared__ int64_t sh[4][1024];
    __shared__ int64_t carry[4];
    if (threadIdx.x < 4) carry[threadIdx.x] = 0;
    __syncthreads();
    for (int32_t base = 0; base < S; base += 1024) {
        const int32_t s = base + (int32_t)threadIdx.x;
        int64_t v[4] = {0, 0, 0, 0};
        if (s < S) {
            int64_t e0, e1;
            seq_range(ev_off, s, n_total, &e0, &e1);
            const int64_t len = e1 - e0;
            const int64_t items = len > 0 ? (len + L - 1) / L : 0;
            const int64_t mm = m_s[s] < 1 ? 1 : m_s[s];
            v[0] = items;
            v[1] = (items + HK_RCH - 1) / HK_RCH;
            v[2] = mm;
            v[3] = mm * mm;
        }
        for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = v[k];
        __syncthreads();
        // inclusive Hillis-Steele scan in shared memory
        for (int d = 1; d < 1024; d <<= 1) {
            int64_t add[4] = {0, 0, 0, 0};
            if ((int)threadIdx.x >= d)
                for (int k = 0; k < 4; ++k) add[k] = sh[k][threadIdx.x - d];
            __syncthreads();
            for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += add[k];
            __syncthreads();
        }
        if (s < S) {
            item_off[s] = carry[0] + sh[0][threadIdx.x] - v[0];
            chunk_off[s] = carry[1] + sh[1][threadIdx.x] - v[1];
            mu_off[s] = carry[2] + sh[2][threadIdx.x] - v[2];
            a_off[s] = carry[3] + sh[3][threadIdx.x] - v[3];
        }
        __syncthreads();
        if (threadIdx.x == 1023)
            for (int k = 0; k < 4; ++k) carry[k] += sh[k][1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        item_off[S] = carry[0];
        chunk_off[S] = carry[1];
        mu_off[S] = carry[2];
        a_off[S] = carry[3];
    }
}

// largest s in [0, S) with off[s] <= x (off nondecreasing, off[0] = 0 <= x)
__device__ __forceinline__ int32_t find_seq(const int64_t* __restrict__ off, int32_t S, int64_t x) {
    int32_t lo = 0, hi = S - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

struct ItemInfo {
    int32_t s;      // sequence
    int64_t k;      // item index within the sequence
    int64_t a, b;   // event range [a, b)
    bool valid;
};

__device__ __forceinline__ ItemInfo item_info(int64_t it, int32_t S, const int64_t* __restrict__ item_off,
                                              const int64_t* __restrict__ ev_off, int32_t L, int64_t n_total,
                                              int64_t n_items_cap) {
    ItemInfo r;
    const int64_t total = item_off[S];
    r.valid = it < total && it < n_items_cap;
    if (!r.valid) { r.s = 0; r.k = 0; r.a = 0; r.b = 0; return r; }
    r.s = find_seq(item_off, S, it);
    // sequences with zero items share item_off values; find_seq returns the last
    // of them, which is the one that owns item `it`.
    r.k = it - item_off[r.s];
    int64_t e0, e1;
    seq_range(ev_off, r.s, n_total, &e0, &e1);
    r.a = e0 + r.k * L;
    r.b = r.a + L < e1 ? r.a + L : e1;
    if (r.a >= r.b) r.valid = false;
    return r;
}

// (K, J) at t0^+ propagated by D = t1 - t0 >= 0 and added to (Kb, Jb)
template <int MP>
__device__ __forceinline__ void compose(double* K, double* J, double D, double beta,
                                        const double* Kb, const double* Jb) {
    const double s = exp(-beta * D);
#pragma unroll
    for (int q = 0; q < MP; ++q) {
        const double k0 = K[q];
        K[q] = __builtin_fma(s, k0, Kb[q]);
        J[q] = __builtin_fma(s, __builtin_fma(D, k0, J[q]), Jb[q]);
    }
}

// Coalesced staging of the items' events.  A wave's items are consecutive,
// so their events are one contiguous range, but each lane walks its own
// item: lane-strided loads would touch a cache line per lane per load.
// Instead, in round r the wave loads event 8 r + j of each of its NI items
// with eight lanes per item (slot v of lane l: item 8 v + l / 8, event
// l mod 8, i.e. 64 contiguous bytes of times per item), writes them to LDS
// as [item][8] and every lane reads its item's 8 events back.  Indices past
// an item's last event repeat the last one, and slots of invalid items load
// nothing, so all loads stay in range.
template <int NI>
struct Stage {
    static constexpr int NV = NI / 8;   // load slots per lane
    int64_t base;                       // the wave's first event (items are consecutive)
    int32_t a[NV], last[NV];            // relative to base; last < 0: invalid item
    double tv[NV];
    int mv[NV];
    // lane `owner(i)` holds item i's range [ia, ib)
    template <typename F>
    __device__ __forceinline__ void init(int lane, int64_t ia, int64_t ib, bool valid, F owner) {
        base = (int64_t)__shfl((long long)(valid ? ia : 0), owner(0), 64);
        base = ((int64_t)__builtin_amdgcn_readfirstlane((int)(base >> 32)) << 32) |
               (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)base);
        const int32_t a0 = valid ? (int32_t)(ia - base) : 0, l0 = valid ? (int32_t)(ib - 1 - base) : -1;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int src = owner(8 * v + (lane >> 3));
            a[v] = __shfl(a0, src, 64);
            last[v] = __shfl(l0, src, 64);
        }
    }
    __device__ __forceinline__ void load(const double* __restrict__ t, const int32_t* __restrict__ marks, int lane,
                                         int r) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            int32_t e = a[v] + 8 * r + (lane & 7);
            e = e < last[v] ? e : last[v];
            tv[v] = 0.0;
            mv[v] = 0;
            if (last[v] >= 0) {
                tv[v] = t[base + e];
                mv[v] = marks[base + e];
            }
        }
    }
    __device__ __forceinline__ void put(double* Ts, int* Ms, int lane) const {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            Ts[64 * v + lane] = tv[v];
            Ms[64 * v + lane] = mv[v];
        }
    }
};

// ---------------------------------------------------------------- phase A
template <int MP>
__global__ __launch_bounds__(256) void small_agg(int32_t S, int64_t n_total, const int64_t* __restrict__ ev_off,
                                                 const int64_t* __restrict__ item_off, int32_t L,
                                                 const double* __restrict__ t, const int32_t* __restrict__ marks,
                                                 const int32_t* __restrict__ m_s, const float* __restrict__ beta,
                                                 double* __restrict__ item_pref,   // [items][2 + 2MP]
                                                 double* __restrict__ tile_agg,    // [tiles][2 + 2MP]
                                                 int64_t n_items_cap) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                         __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int64_t it = wave * 64 + lane;
    if (wave * 64 >= n_items_cap) return;   // whole wave beyond the buffers (wave-uniform)
    ItemInfo inf = item_info(it, S, item_off, ev_off, L, n_total, n_items_cap);
    double K[MP], J[MP];
    double D = 0.0;
    int reset = 1;
    double bet = 0.0;
    const bool work = inf.valid && inf.b > inf.a;
    int32_t M = 1;
    double tref = 0.0, tl = 0.0;
    if (work) {
        M = m_s[inf.s] < 1 ? 1 : (m_s[inf.s] > MP ? MP : m_s[inf.s]);
        bet = (double)beta[inf.s];
        reset = inf.k == 0;
        tref = reset ? t[inf.a] : t[inf.a - 1];
        tl = t[inf.b - 1];
    }
    // the item's map, summed per node in LDS: each event adds its terms at
    // the item's last event, e^{-beta (tl - t)} to K and (tl - t) e^{..} to J
    // (rows of 2 MP + 1 doubles: an odd stride spreads the lanes over the banks)
    constexpr int AR = 2 * MP + 1;
    __shared__ double AG[4][64][AR];
    double* ag = AG[threadIdx.x >> 6][lane];
#pragma unroll
    for (int q = 0; q < 2 * MP; ++q) ag[q] = 0.0;
    lds_wait();
    // the wave's events in rounds of 8 per item, staged through LDS, the next
    // round's loads in flight while the current one is processed
    __shared__ double Tst[4][512];
    __shared__ int Mst[4][512];
    double* Ts = Tst[threadIdx.x >> 6];
    int* Ms = Mst[threadIdx.x >> 6];
    Stage<64> stg;
    stg.init(lane, inf.a, inf.b, work, [](int i) { return i; });
    stg.load(t, marks, lane, 0);
    const int rounds = (L + 7) / 8;
    for (int r = 0; r < rounds; ++r) {
        stg.put(Ts, Ms, lane);
        if (r + 1 < rounds) stg.load(t, marks, lane, r + 1);
        __builtin_amdgcn_wave_barrier();
        double tv[8];
        int mv[8];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            tv[j] = Ts[8 * lane + j];
            mv[j] = Ms[8 * lane + j];
        }
        __builtin_amdgcn_wave_barrier();
        const int64_t e0 = inf.a + 8 * r;
        if (work && e0 < inf.b) {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                if (e0 + j < inf.b) {
                    const double d = tl - tv[j];
                    const double e = exp_f64(-bet * d);
                    const int q = clamp_mark(mv[j], M);
                    atomicAdd(&ag[q], e);
                    atomicAdd(&ag[MP + q], d * e);
                }
            }
        }
    }
    lds_wait();   // the adds land before the reads
#pragma unroll
    for (int q = 0; q < MP; ++q) {
        K[q] = ag[q];
        J[q] = ag[MP + q];
    }
    if (work) D = tl - tref;
    // segmented inclusive scan over the wave's 64 items
    for (int d = 1; d < 64; d <<= 1) {
        const double oD = shfl_up_d(D, d);
        const int oreset = __shfl_up(reset, d, 64);
        double oK[MP], oJ[MP];
#pragma unroll
        for (int q = 0; q < MP; ++q) { oK[q] = shfl_up_d(K[q], d); oJ[q] = shfl_up_d(J[q], d); }
        if (lane >= d && !reset) {
            // other (earlier) then me: me has no reset, so both lie in my sequence
            double nK[MP], nJ[MP];
#pragma unroll
            for (int q = 0; q < MP; ++q) { nK[q] = oK[q]; nJ[q] = oJ[q]; }
            compose<MP>(nK, nJ, D, bet, K, J);
#pragma unroll
            for (int q = 0; q < MP; ++q) { K[q] = nK[q]; J[q] = nJ[q]; }
            D = oD + D;
            reset = oreset;
        }
    }
    // exclusive prefix = inclusive value of the previous lane (identity for lane 0)
    const double pD = shfl_up_d(D, 1);
    const int preset = __shfl_up(reset, 1, 64);
    double pK[MP], pJ[MP];
#pragma unroll
    for (int q = 0; q < MP; ++q) { pK[q] = shfl_up_d(K[q], 1); pJ[q] = shfl_up_d(J[q], 1); }
    if (it < n_items_cap) {
        double* o = item_pref + it * (2 + 2 * MP);
        o[0] = lane == 0 ? 0.0 : pD;
        o[1] = lane == 0 ? 0.0 : (double)preset;
#pragma unroll
        for (int q = 0; q < MP; ++q) {
            o[2 + q] = lane == 0 ? 0.0 : pK[q];
            o[2 + MP + q] = lane == 0 ? 0.0 : pJ[q];
        }
    }
    if (lane == 63) {
        double* o = tile_agg + wave * (2 + 2 * MP);
        o[0] = D;
        o[1] = (double)reset;
#pragma unroll
        for (int q = 0; q < MP; ++q) { o[2 + q] = K[q]; o[2 + MP + q] = J[q]; }
    }
}

// ---------------------------------------------------------------- phase B
// thread per (sequence, node): chain the aggregates of the waves its sequence spans
template <int MP>
__global__ __launch_bounds__(256) void small_tile_scan(int32_t S, int64_t n_items_cap,
                                                       const int64_t* __restrict__ item_off,
                                                       const float* __restrict__ beta,
                                                       const double* __restrict__ tile_agg,
                                                       double* __restrict__ tile_carry) {   // [tiles][2MP]
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= (int64_t)S * MP) return;
    const int32_t s = (int32_t)(gid / MP);
    const int q = (int)(gid % MP);
    const int64_t f = item_off[s];
    int64_t l = item_off[s + 1];
    l = l > n_items_cap ? n_items_cap : l;
    if (l <= f) return;
    const int64_t t0 = f / 64, t1 = (l - 1) / 64;
    if (t1 == t0) return;
    const double bet = (double)beta[s];
    const int W = 2 + 2 * MP;
    double K = tile_agg[t0 * W + 2 + q], J = tile_agg[t0 * W + 2 + MP + q];
    for (int64_t tt = t0 + 1; tt <= t1; ++tt) {
        tile_carry[tt * 2 * MP + q] = K;
        tile_carry[tt * 2 * MP + MP + q] = J;
        if (tt == t1) break;
        const double D = tile_agg[tt * W + 0];
        const double ex = exp(-bet * D);
        const double Kb = tile_agg[tt * W + 2 + q], Jb = tile_agg[tt * W + 2 + MP + q];
        const double k0 = K;
        K = __builtin_fma(ex, k0, Kb);
        J = __builtin_fma(ex, __builtin_fma(D, k0, J), Jb);
    }
}

// ---------------------------------------------------------------- phase C
// Partial layout per item (float64, item-major, stride PW):
//   0 log-sum, 1 compensator sum_j colsum[m_j] (1 - e^{-beta (T - t_j)}),
//   GRAD: 2 E = sum_j colsum[m_j] (T - t_j) e^{-beta (T - t_j)},
//         3 sum_i w_i (R_i - beta D_i), 4.. S_q, 4+MP.. C_q, 4+2MP.. G[p][q]
template <int MP, bool GRAD, bool INTENS>
__global__ __launch_bounds__(256) void small_compute(int32_t S, int64_t n_total, const int64_t* __restrict__ ev_off,
                                                     const int64_t* __restrict__ item_off, int32_t L,
                                                     const double* __restrict__ t, const int32_t* __restrict__ marks,
                                                     const int32_t* __restrict__ m_s, const double* __restrict__ T_s,
                                                     const float* __restrict__ mu, const float* __restrict__ alpha,
                                                     const float* __restrict__ beta,
                                                     const int64_t* __restrict__ mu_off, const int64_t* __restrict__ a_off,
                                                     const double* __restrict__ item_pref,
                                                     const double* __restrict__ tile_carry,
                                                     double* __restrict__ part, int32_t PW,
                                                     float* __restrict__ lambda_out, int64_t n_items_cap) {
    const int lane = threadIdx.x & 63;
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                         __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int64_t it = wave * 64 + lane;
    if (it >= n_items_cap) return;
    ItemInfo inf = item_info(it, S, item_off, ev_off, L, n_total, n_items_cap);
    if (!inf.valid) return;
    const int32_t M = m_s[inf.s] < 1 ? 1 : (m_s[inf.s] > MP ? MP : m_s[inf.s]);
    const double bet = (double)beta[inf.s];
    const double T = T_s[inf.s];
    const float* al = alpha + a_off[inf.s];
    const float* mus = mu + mu_off[inf.s];
    double colsum[MP];
#pragma unroll
    for (int q = 0; q < MP; ++q) {
        double c = 0.0;
        if (q < M)
            for (int p = 0; p < M; ++p) c += (double)al[p * M + q];
        colsum[q] = c;
    }
    double K[MP], J[MP];
#pragma unroll
    for (int q = 0; q < MP; ++q) { K[q] = 0.0; J[q] = 0.0; }
    double tp;
    if (inf.k == 0) {
        tp = t[inf.a];
    } else {
        tp = t[inf.a - 1];
        const double* pr = item_pref + it * (2 + 2 * MP);
        const double pD = pr[0];
        const bool preset = pr[1] != 0.0;
#pragma unroll
        for (int q = 0; q < MP; ++q) { K[q] = pr[2 + q]; J[q] = pr[2 + MP + q]; }
        if (!preset) {
            const int64_t tile = it / 64;
            double cK[MP], cJ[MP];
#pragma unroll
            for (int q = 0; q < MP; ++q) {
                cK[q] = tile_carry[tile * 2 * MP + q];
                cJ[q] = tile_carry[tile * 2 * MP + MP + q];
            }
            // the tile carry exists whenever this item's sequence started in an
            // earlier tile, which is exactly the case preset == 0 and k > 0
            compose<MP>(cK, cJ, pD, bet, K, J);
#pragma unroll
            for (int q = 0; q < MP; ++q) { K[q] = cK[q]; J[q] = cJ[q]; }
        }
    }
    double logsum = 0.0, comp = 0.0, Esum = 0.0, gb = 0.0;
    double Sq[MP], Cq[MP], G[GRAD ? MP : 1][GRAD ? MP : 1];
#pragma unroll
    for (int q = 0; q < MP; ++q) { Sq[q] = 0.0; Cq[q] = 0.0; }
    if (GRAD) {
#pragma unroll
        for (int p = 0; p < (GRAD ? MP : 1); ++p)
#pragma unroll
            for (int q = 0; q < (GRAD ? MP : 1); ++q) G[p][q] = 0.0;
    }
    int mp = -1;
    // events in blocks of 8 per lane, the next block's loads in flight while
    // the current one is processed (clamped indices stay valid)
    const int64_t last = inf.b - 1;
    double tn[8];
    int mn[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int64_t e = inf.a + j < last ? inf.a + j : last;
        tn[j] = t[e];
        mn[j] = marks[e];
    }
    for (int64_t e0 = inf.a; e0 < inf.b; e0 += 8) {
    double tv[8];
    int mv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        tv[j] = tn[j];
        mv[j] = mn[j];
        const int64_t e = e0 + 8 + j < last ? e0 + 8 + j : last;
        tn[j] = t[e];
        mn[j] = marks[e];
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (e0 + j >= inf.b) continue;
        const int64_t e = e0 + j;
        const double te = tv[j];
        const double d = te - tp;
        const double s = exp_f64(-bet * d);
#pragma unroll
        for (int q = 0; q < MP; ++q) {
            const double k1 = s * (K[q] + (q == mp ? 1.0 : 0.0));
            J[q] = __builtin_fma(s, J[q], d * k1);
            K[q] = k1;
        }
        const int p = clamp_mark(mv[j], M);
        double R = 0.0, Dd = 0.0;
#pragma unroll
        for (int q = 0; q < MP; ++q) {
            const double a = q < M ? (double)al[p * M + q] : 0.0;
            R = __builtin_fma(a, K[q], R);
            Dd = __builtin_fma(a, J[q], Dd);
        }
        const double lam = (double)mus[p] + bet * R;
        if (INTENS) lambda_out[e] = (float)lam;
        logsum += log(lam);
        const double x = bet * (T - te);
        const double ex = exp_f64(-x);
        double csp = 0.0;
#pragma unroll
        for (int q = 0; q < MP; ++q) csp = (q == p) ? colsum[q] : csp;
        comp += csp * (1.0 - ex);
        if (GRAD) {
            const double w = 1.0 / lam;
            gb += w * (R - bet * Dd);
            Esum += csp * (T - te) * ex;
#pragma unroll
            for (int q = 0; q < MP; ++q) {
                Sq[q] += (q == p) ? w : 0.0;
                Cq[q] += (q == p) ? (1.0 - ex) : 0.0;
            }
#pragma unroll
            for (int r = 0; r < (GRAD ? MP : 1); ++r) {
                const double cr = (r == p) ? w : 0.0;
#pragma unroll
                for (int q = 0; q < (GRAD ? MP : 1); ++q) G[r][q] = __builtin_fma(cr, K[q], G[r][q]);
            }
        }
        tp = te;
        mp = p;
    }
    }
    double* o = part + it * (int64_t)PW;
    o[0] = logsum;
    o[1] = comp;
    if (GRAD) {
        o[2] = Esum;
        o[3] = gb;
#pragma unroll
        for (int q = 0; q < MP; ++q) { o[4 + q] = Sq[q]; o[4 + MP + q] = Cq[q]; }
#pragma unroll
        for (int r = 0; r < (GRAD ? MP : 1); ++r)
#pragma unroll
            for (int q = 0; q < (GRAD ? MP : 1); ++q) o[4 + 2 * MP + r * MP + q] = G[r][q];
    }
}

// Column-split phase C for the gradient (MP >= 4): LPI lanes per item; lane
// c of the item's group holds the state K_q, J_q of its CL = MP / LPI nodes
// q = c CL .. c CL + CL - 1 and those columns of the item's dL/dalpha block,
// so the block needs MP CL instead of MP^2 float64 per lane and more waves
// share a SIMD.  Events go in blocks of 8: the block's decays
// e^{-beta (t_j - t_{j-1})} and e^{-beta (T - t_j)} are computed once, by
// lane j mod LPI, before the in-order pass over the block and fetched from it
// by the other lanes; R = alpha_{p,:} . K and D = alpha_{p,:} . J are summed
// over the group (a butterfly, identical in every lane); the block's
// logarithms are taken afterwards, again one event per lane.  The per-node
// sums of the event's node (w, 1 - e^{-beta (T - t)} and (T - t)
// e^{-beta (T - t)}) go to the item's LDS row by the event's lane (LDS
// atomics: no selects over the nodes), and the compensator and its
// beta-derivative come from them at the item's end, weighted by the column
// sums of alpha.  The lanes' scalar partials are summed in lane order.
// Lane l's double from lane (l & ~1) + S of its pair (CTL 0xA0: S = 0, 0xF5:
// S = 1) or from lane l ^ 1 (0xB1): DPP quad permutations on the vector ALU,
// where __shfl would take an LDS round trip.  Both lanes of a pair are active
// together (they walk the same item).
template <int CTL>
__device__ __forceinline__ double pair_dpp(double x) {
    const int lo = __builtin_amdgcn_mov_dpp(__double2loint(x), CTL, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(x), CTL, 0xF, 0xF, false);
    return __hiloint2double(hi, lo);
}

template <int MP, int LPI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void small_compute_c(int32_t S, int64_t n_total, const int64_t* __restrict__ ev_off,
                                                       const int64_t* __restrict__ item_off, int32_t L,
                                                       const double* __restrict__ t,
                                                       const int32_t* __restrict__ marks,
                                                       const int32_t* __restrict__ m_s,
                                                       const double* __restrict__ T_s, const float* __restrict__ mu,
                                                       const float* __restrict__ alpha,
                                                       const float* __restrict__ beta,
                                                       const int64_t* __restrict__ mu_off,
                                                       const int64_t* __restrict__ a_off,
                                                       const double* __restrict__ item_pref,
                                                       const double* __restrict__ tile_carry,
                                                       double* __restrict__ part, int32_t PW, int64_t n_items_cap) {
    constexpr int IPW = 64 / LPI;  // items per wave
    constexpr int CL = MP / LPI;   // nodes (columns) per lane
    constexpr int NB = 8;          // events per block
    constexpr int NO = NB / LPI;   // block events whose decays and logarithm a lane takes
    const int lane = threadIdx.x & 63;
    const int c = lane % LPI;
    const int g0 = lane - c;       // the group's first lane
    const int qa = c * CL;         // this lane's first node
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) +
                         __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    const int64_t it = wave * IPW + lane / LPI;
    if (wave * IPW >= n_items_cap) return;   // the whole wave (wave-uniform)
    // every lane stays to the end (the event loads are cooperative); lanes
    // of invalid items (sequence 0's parameters, no events) write nothing
    const ItemInfo inf = item_info(it, S, item_off, ev_off, L, n_total, n_items_cap);
    const bool work = inf.valid;
    const int32_t M = m_s[inf.s] < 1 ? 1 : (m_s[inf.s] > MP ? MP : m_s[inf.s]);
    const double bet = (double)beta[inf.s];
    const double T = T_s[inf.s];
    const float* al = alpha + a_off[inf.s];
    const float* mus = mu + mu_off[inf.s];
    // the item's alpha (MP x MP, zero past M) and mu in LDS, written by its
    // LPI lanes and read by them only (the events' rows are then LDS reads
    // instead of dependent global loads)
    constexpr int AW = MP * MP + (MP < 4 ? 4 : MP);   // floats per item, a multiple of 4
    __shared__ __align__(16) float ALs[4 * IPW][AW];
    float* A_ = ALs[(threadIdx.x >> 6) * IPW + lane / LPI];
    // per node of the item: sum of w, of 1 - e^{-beta (T - t)}, of (T - t) e^{-beta (T - t)}
    __shared__ double SCE[4 * IPW][3 * MP];
    double* sce = SCE[(threadIdx.x >> 6) * IPW + lane / LPI];
    for (int e = c; e < 3 * MP; e += LPI) sce[e] = 0.0;
    for (int e = c; e < AW; e += LPI) {
        const int pr = e / MP, qc = e % MP;
        float v = 0.0f;
        if (e < MP * MP) {
            if (pr < M && qc < M) v = al[pr * M + qc];
        } else if (e - MP * MP < M) {
            v = mus[e - MP * MP];
        }
        A_[e] = v;
    }
    lds_wait();   // the item's rows and cleared sums before any read or atomic
    double K[CL], J[CL];
#pragma unroll
    for (int u = 0; u < CL; ++u) { K[u] = 0.0; J[u] = 0.0; }
    double tp = 0.0;
    if (!work) {
    } else if (inf.k == 0) {
        tp = t[inf.a];
    } else {
        tp = t[inf.a - 1];
        const double* pr = item_pref + it * (2 + 2 * MP);
        const double pD = pr[0];
        const bool preset = pr[1] != 0.0;
#pragma unroll
        for (int u = 0; u < CL; ++u) { K[u] = pr[2 + qa + u]; J[u] = pr[2 + MP + qa + u]; }
        if (!preset) {
            // the tile carry exists whenever this item's sequence started in
            // an earlier tile, which is exactly the case preset == 0, k > 0
            const int64_t tile = it / 64;
            const double sd = exp(-bet * pD);
#pragma unroll
            for (int u = 0; u < CL; ++u) {
                const double cK = tile_carry[tile * 2 * MP + qa + u];
                const double cJ = tile_carry[tile * 2 * MP + MP + qa + u];
                const double nK = __builtin_fma(sd, cK, K[u]);
                J[u] = __builtin_fma(sd, __builtin_fma(pD, cK, cJ), J[u]);
                K[u] = nK;
            }
        }
    }
    double lsum = 0.0, gbs = 0.0;
    double Gc[MP][CL];
#pragma unroll
    for (int u = 0; u < CL; ++u)
#pragma unroll
        for (int r = 0; r < MP; ++r) Gc[r][u] = 0.0;
    int mp = -1;
    // the items' events in rounds of NB, staged through LDS (coalesced
    // loads), the next round's loads in flight while one is processed
    static_assert(NB == 8, "rounds of the staging are 8 events");
    __shared__ double Tst[4][IPW * 8];
    __shared__ int Mst[4][IPW * 8];
    double* Ts = Tst[threadIdx.x >> 6];
    int* Ms = Mst[threadIdx.x >> 6];
    Stage<IPW> stg;
    stg.init(lane, inf.a, inf.b, work, [](int i) { return i * LPI; });
    stg.load(t, marks, lane, 0);
    const int rounds = (L + NB - 1) / NB;
    for (int rd = 0; rd < rounds; ++rd) {
        stg.put(Ts, Ms, lane);
        if (rd + 1 < rounds) stg.load(t, marks, lane, rd + 1);
        __builtin_amdgcn_wave_barrier();
        double tv[NB];
        int mv[NB];
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            tv[j] = Ts[8 * (lane / LPI) + j];
            mv[j] = Ms[8 * (lane / LPI) + j];
        }
        __builtin_amdgcn_wave_barrier();
        const int64_t e0 = inf.a + (int64_t)NB * rd;
        if (!work || e0 >= inf.b) continue;
        // this lane's events of the block: j = c + LPI o (past the item's
        // end the staged values repeat its last event and are not used)
        double so[NO], xo[NO];
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            const int j = c + LPI * o;
            const double tj = tv[j];
            const double tjm = j == 0 ? tp : tv[j - 1];
            so[o] = exp_f64(-bet * (tj - tjm));
            xo[o] = exp_f64(-bet * (T - tj));
        }
        double lo[NO], ro[NO];
#pragma unroll
        for (int o = 0; o < NO; ++o) { lo[o] = 1.0; ro[o] = 0.0; }
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (e0 + j >= inf.b) break;
            double sj, ex;
            if (LPI == 2) {
                sj = j % 2 == 0 ? pair_dpp<0xA0>(so[j / 2]) : pair_dpp<0xF5>(so[j / 2]);
                ex = j % 2 == 0 ? pair_dpp<0xA0>(xo[j / 2]) : pair_dpp<0xF5>(xo[j / 2]);
            } else {
                const int src = g0 + j % LPI;
                sj = __shfl(so[j / LPI], src, 64);
                ex = __shfl(xo[j / LPI], src, 64);
            }
            const double te = tv[j];
            const double d = te - tp;
            const int p = clamp_mark(mv[j], M);
            double R = 0.0, Dd = 0.0;
#pragma unroll
            for (int u = 0; u < CL; ++u) {
                const double k1 = sj * (K[u] + (qa + u == mp ? 1.0 : 0.0));
                J[u] = __builtin_fma(sj, J[u], d * k1);
                K[u] = k1;
                const double a = (double)A_[p * MP + qa + u];
                R = __builtin_fma(a, K[u], R);
                Dd = __builtin_fma(a, J[u], Dd);
            }
            if (LPI == 2) {
                R += pair_dpp<0xB1>(R);
                Dd += pair_dpp<0xB1>(Dd);
            } else {
#pragma unroll
                for (int off = 1; off < LPI; off <<= 1) {
                    R += __shfl_xor(R, off, 64);
                    Dd += __shfl_xor(Dd, off, 64);
                }
            }
            const double lam = (double)A_[MP * MP + p] + bet * R;
            // 1 / lambda: hardware reciprocal and two Newton steps
            double w = __builtin_amdgcn_rcp(lam);
            w = __builtin_fma(w, __builtin_fma(-lam, w, 1.0), w);
            w = __builtin_fma(w, __builtin_fma(-lam, w, 1.0), w);
            if (c == j % LPI) {
                lo[j / LPI] = lam;
                ro[j / LPI] = w * (R - bet * Dd);
                atomicAdd(&sce[p], w);
                atomicAdd(&sce[MP + p], 1.0 - ex);
                atomicAdd(&sce[2 * MP + p], (T - te) * ex);
            }
#pragma unroll
            for (int u = 0; u < CL; ++u)
#pragma unroll
                for (int r = 0; r < MP; ++r) Gc[r][u] = __builtin_fma(r == p ? w : 0.0, K[u], Gc[r][u]);
            tp = te;
            mp = p;
        }
#pragma unroll
        for (int o = 0; o < NO; ++o) {
            lsum += log(lo[o]);
            gbs += ro[o];
        }
    }
    // the group's scalar partials, summed in lane order
    double tl = 0.0, tg = 0.0;
#pragma unroll
    for (int i = 0; i < LPI; ++i) {
        tl += __shfl(lsum, g0 + i, 64);
        tg += __shfl(gbs, g0 + i, 64);
    }
    lds_wait();   // the per-node sums' atomics land before they are read
    if (!work) return;
    double* o = part + it * (int64_t)PW;
    if (c == 0) {
        // compensator and its beta-derivative part from the per-node sums,
        // weighted by the column sums of alpha
        double tc = 0.0, te2 = 0.0;
#pragma unroll
        for (int q = 0; q < MP; ++q) {
            double cs = 0.0;
#pragma unroll
            for (int p = 0; p < MP; ++p) cs += (double)A_[p * MP + q];
            tc = __builtin_fma(cs, sce[MP + q], tc);
            te2 = __builtin_fma(cs, sce[2 * MP + q], te2);
        }
        o[0] = tl;
        o[1] = tc;
        o[2] = te2;
        o[3] = tg;
    }
#pragma unroll
    for (int u = 0; u < CL; ++u) {
        o[4 + qa + u] = sce[qa + u];
        o[4 + MP + qa + u] = sce[MP + qa + u];
#pragma unroll
        for (int r = 0; r < MP; ++r) o[4 + 2 * MP + r * MP + qa + u] = Gc[r][u];
    }
}

// ---------------------------------------------------------------- reduction
// level 1: per (sequence, chunk of HK_RCH items): thread per partial entry
__global__ __launch_bounds__(128) void small_reduce1(int32_t S, int64_t n_items_cap,
                                                    const int64_t* __restrict__ item_off,
                                                    const int64_t* __restrict__ chunk_off,
                                                    const double* __restrict__ part, int32_t PW,
                                                    double* __restrict__ cpart, int64_t n_chunks_cap) {
    const int64_t c = blockIdx.x;
    if (c >= n_chunks_cap) return;
    if (c >= chunk_off[S]) return;
    const int32_t s = find_seq(chunk_off, S, c);
    const int64_t kc = c - chunk_off[s];
    const int64_t i0 = item_off[s] + kc * HK_RCH;
    int64_t i1e = item_off[s + 1];
    i1e = i1e > n_items_cap ? n_items_cap : i1e;
    const int64_t i1 = i0 + HK_RCH < i1e ? i0 + HK_RCH : i1e;
    for (int e = threadIdx.x; e < PW; e += blockDim.x) {
        double acc = 0.0;
        for (int64_t i = i0; i < i1; ++i) acc += part[i * PW + e];
        cpart[c * PW + e] = acc;
    }
}

// level 2: per sequence; assemble eqs. 2, 8, 9, 10
template <int MP, bool GRAD>
__global__ __launch_bounds__(128) void small_reduce2(int32_t S, int64_t n_chunks_cap,
                                                    const int64_t* __restrict__ chunk_off,
                                                    const int32_t* __restrict__ m_s, const double* __restrict__ T_s,
                                                    const float* __restrict__ mu, const float* __restrict__ beta,
                                                    const int64_t* __restrict__ mu_off, const int64_t* __restrict__ a_off,
                                                    const double* __restrict__ cpart, int32_t PW,
                                                    double* __restrict__ loglik, double* __restrict__ g_mu,
                                                    double* __restrict__ g_alpha, double* __restrict__ g_beta) {
    const int32_t s = blockIdx.x;
    if (s >= S) return;
    __shared__ double tot[4 + 2 * MP + MP * MP];
    const int64_t c0 = chunk_off[s];
    int64_t c1 = chunk_off[s + 1];
    c1 = c1 > n_chunks_cap ? n_chunks_cap : c1;
    for (int e = threadIdx.x; e < PW; e += blockDim.x) {
        double acc = 0.0;
        for (int64_t c = c0; c < c1; ++c) acc += cpart[c * PW + e];
        tot[e] = acc;
    }
    __syncthreads();
    const int32_t M = m_s[s] < 1 ? 1 : (m_s[s] > MP ? MP : m_s[s]);
    const double T = T_s[s];
    const float* mus = mu + mu_off[s];
    if (threadIdx.x == 0) {
        double musum = 0.0;
        for (int p = 0; p < M; ++p) musum += (double)mus[p];
        loglik[s] = tot[0] - T * musum - tot[1];
        if (GRAD && g_beta) g_beta[s] = tot[3] - tot[2];
    }
    if (GRAD) {
        const double bet = (double)beta[s];
        for (int x = threadIdx.x; x < M * M; x += blockDim.x) {
            const int p = x / M, q = x % M;
            if (g_alpha) g_alpha[a_off[s] + x] = bet * tot[4 + 2 * MP + p * MP + q] - tot[4 + MP + q];
        }
        for (int q = threadIdx.x; q < M; q += blockDim.x)
            if (g_mu) g_mu[mu_off[s] + q] = tot[4 + q] - T;
    }
}

// ---------------------------------------------------------------- host launch
template <int MP>
static hawkes_status run_small_mp(const SmallArgs& A, hipStream_t st) {
    const int32_t PW = A.grad ? 4 + 2 * MP + MP * MP : 2;
    const int64_t waves = (A.n_items_cap + 63) / 64;
    const int64_t blocks = (waves + 3) / 4;
    TimedScope* t5 = new TimedScope(5, st);
    hipLaunchKernelGGL(small_setup, dim3(1), dim3(1024), 0, st, A.S, A.n_total, A.ev_off, A.m_s, A.L,
                       A.item_off, A.chunk_off, A.mu_off, A.a_off);
    hipLaunchKernelGGL(small_agg<MP>, dim3((unsigned)blocks), dim3(256), 0, st, A.S, A.n_total, A.ev_off,
                       A.item_off, A.L,
                       A.t, A.marks, A.m_s, A.beta, A.item_pref, A.tile_agg, A.n_items_cap);
    const int64_t nthr = (int64_t)A.S * MP;
    hipLaunchKernelGGL(small_tile_scan<MP>, dim3((unsigned)((nthr + 255) / 256)), dim3(256), 0, st, A.S,
                       A.n_items_cap, A.item_off, A.beta, A.tile_agg, A.tile_carry);
    delete t5;
    TimedScope* t4 = new TimedScope(4, st);
    bool done = false;
    if constexpr (MP >= 4) {
        if (A.grad) {
            constexpr int LPI = 2;   // lanes per item (4 measured slower for MP = 8)
            const int64_t wc = (A.n_items_cap * LPI + 63) / 64;
            hipLaunchKernelGGL((small_compute_c<MP, LPI>), dim3((unsigned)((wc + 3) / 4)), dim3(256), 0, st, A.S,
                               A.n_total, A.ev_off, A.item_off, A.L, A.t, A.marks, A.m_s, A.T_s, A.mu, A.alpha,
                               A.beta, A.mu_off, A.a_off, A.item_pref, A.tile_carry, A.part, PW, A.n_items_cap);
            done = true;
        }
    }
    if (done) {
    } else if (A.grad) {
        hipLaunchKernelGGL((small_compute<MP, true, false>), dim3((unsigned)blocks), dim3(256), 0, st, A.S,
                           A.n_total, A.ev_off, A.item_off, A.L, A.t, A.marks, A.m_s, A.T_s, A.mu, A.alpha, A.beta,
                           A.mu_off, A.a_off, A.item_pref, A.tile_carry, A.part, PW, (float*)nullptr,
                           A.n_items_cap);
    } else if (A.lambda_out) {
        hipLaunchKernelGGL((small_compute<MP, false, true>), dim3((unsigned)blocks), dim3(256), 0, st, A.S,
                           A.n_total, A.ev_off, A.item_off, A.L, A.t, A.marks, A.m_s, A.T_s, A.mu, A.alpha, A.beta,
                           A.mu_off, A.a_off, A.item_pref, A.tile_carry, A.part, PW, A.lambda_out,
                           A.n_items_cap);
    } else {
        hipLaunchKernelGGL((small_compute<MP, false, false>), dim3((unsigned)blocks), dim3(256), 0, st, A.S,
                           A.n_total, A.ev_off, A.item_off, A.L, A.t, A.marks, A.m_s, A.T_s, A.mu, A.alpha, A.beta,
                           A.mu_off, A.a_off, A.item_pref, A.tile_carry, A.part, PW, (float*)nullptr,
                           A.n_items_cap);
    }
    delete t4;
    hipLaunchKernelGGL(small_reduce1, dim3((unsigned)A.n_chunks_cap), dim3(128), 0, st, A.S, A.n_items_cap,
                       A.item_off,
                       A.chunk_off, A.part, PW, A.cpart, A.n_chunks_cap);
    if (A.grad)
        hipLaunchKernelGGL((small_reduce2<MP, true>), dim3((unsigned)A.S), dim3(128), 0, st, A.S, A.n_chunks_cap,
                           A.chunk_off,
                           A.m_s, A.T_s, A.mu, A.beta, A.mu_off, A.a_off, A.cpart, PW, A.loglik, A.g_mu,
                           A.g_alpha, A.g_beta);
    else
        hipLaunchKernelGGL((small_reduce2<MP, false>), dim3((unsigned)A.S), dim3(128), 0, st, A.S, A.n_chunks_cap,
                           A.chunk_off,
                           A.m_s, A.T_s, A.mu, A.beta, A.mu_off, A.a_off, A.cpart, PW, A.loglik, A.g_mu,
                           A.g_alpha, A.g_beta);
    return hipGetLastError() == hipSuccess ? HAWKES_OK : HAWKES_EDEVICE;
}

hawkes_status run_small(const SmallArgs& A, hipStream_t st) {
    switch (A.MP) {
        case 1: return run_small_mp<1>(A, st);
        case 2: return run_small_mp<2>(A, st);
        case 4: return run_small_mp<4>(A, st);
        case 8: return run_small_mp<8>(A, st);
        default: return HAWKES_EUNSUPPORTED;
    }
}

}  // namespace hk
