// Large-M engine: one sequence, M > 8 nodes, decay shared by all targets.
//
// The sequence is evaluated in chunks of CH events (constant memory: only
// M-vector carries cross a chunk boundary, as in the batched procedure of
// Algorithm 2).  Within a chunk, segments of HK_SEG events are the scan
// elements.  The state is the source-indexed pair of the paper's gradient
// recurrence (eq. 11) and its time-weighted companion:
//   K_q(t) = sum_{j: t_j<t, m_j=q} e^{-beta (t - t_j)}
//   J_q(t) = sum_{j: t_j<t, m_j=q} (t - t_j) e^{-beta (t - t_j)}
// A run of events maps the state at its start to the state at its end by
//   K -> e^{-beta D} K + K_run,   J -> e^{-beta D} (J + D K) + J_run
// (the (s I, v) maps of "Methods", with a shear for J); composing these is
// the associative operator of the scan.
//
// Per chunk:
//   agg      one wave per segment folds its events into (K_run, J_run)
//   scan     one thread per node chains the segment maps -> carry-in per segment
//   forward  a workgroup of two waves per segment replays its events 64 at a
//            time (one per lane; each wave takes every other nonzero of the
//            event's row of alpha, the first wave adds the partial sums and
//            does the rest).  Each node keeps a lazily decayed record (tau_q, K_q, J_q)
//            in LDS; lambda_i needs only the nonzeros of alpha's row m_i
//            (R = alpha_{m_i,:} . K, eq. 3), read from a CSR copy of alpha,
//            plus the same-batch events found through a per-node lane mask.
//            It writes lambda_i / per-segment float64 partials and, for the
//            gradient, per-event coefficients for the dense kernel.
//   bucket   the chunk's events partitioned by blocks of 16 nodes (hk_bucket.hip)
//   dense    dense dL/dalpha (first term of eq. 9, hk_dense.hip): state
//            checkpoints per column block, then tiles of 16 rows x up to 256
//            columns per event range, the rank-1 part of each window in
//            registers and its pair terms in float64 LDS.
#include "hk_device.h"
#include "hk_large.h"
#include <stdlib.h>
#include <mutex>

namespace hk {

// ------------------------------------------------------------------ setup
__global__ void fill_d(double* p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// colsum[q] = sum_p alpha[p][q]: a workgroup of 16 waves per 64 columns,
// wave r sums rows r, r+16, ... (coalesced over q), then a fixed-order sum
__global__ __launch_bounds__(1024) void large_colsum(int32_t M, const float* __restrict__ alpha,
                                                     float* __restrict__ colsum) {
    __shared__ double part[16][64];
    const int lane = threadIdx.x & 63, r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int32_t q = blockIdx.x * 64 + lane;
    double c = 0.0;
    if (q < M) {
#pragma unroll 8
        for (int32_t p = r; p < M; p += 16) c += (double)alpha[(int64_t)p * M + q];
    }
    part[r][lane] = c;
    __syncthreads();
    if (r == 0 && q < M) {
        double v = 0.0;
        for (int k = 0; k < 16; ++k) v += part[k][lane];
        colsum[q] = (float)v;
    }
}

// csr_ptr[p+1] = nnz of row p (one wave per row, coalesced).  With trans != 0
// the rows are the columns of alpha (compressed-column form, strided reads).
__device__ __forceinline__ float alpha_at(const float* __restrict__ alpha, int32_t M, int32_t r, int32_t c,
                                          int trans) {
    return trans ? alpha[(int64_t)c * M + r] : alpha[(int64_t)r * M + c];
}

__global__ __launch_bounds__(64) void large_rowcount(int32_t M, const float* __restrict__ alpha,
                                                     int32_t* __restrict__ csr_ptr, int trans) {
    const int32_t p = blockIdx.x;
    const int lane = threadIdx.x;
    int32_t cnt = 0;
    for (int32_t q = lane; q < M; q += 64) cnt += alpha_at(alpha, M, p, q, trans) != 0.0f;
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_down(cnt, off, 64);
    if (lane == 0) {
        csr_ptr[p + 1] = cnt;
        if (p == 0) csr_ptr[0] = 0;
    }
}

// inclusive scan of csr_ptr[1..M] in one workgroup
__global__ __launch_bounds__(1024) void large_csr_scan(int32_t M, int32_t* __restrict__ csr_ptr) {
    __shared__ int32_t sh[1024];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int32_t base = 0; base < M; base += 1024) {
        const int32_t i = base + threadIdx.x;
        const int32_t v = i < M ? csr_ptr[i + 1] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const int32_t a = (int)threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
            __syncthreads();
            sh[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < M) csr_ptr[i + 1] = carry + sh[threadIdx.x];
        __syncthreads();
        if (threadIdx.x == 1023) carry += sh[1023];
        __syncthreads();
    }
}

// one wave per row: compact the nonzeros of row p in column order
__global__ __launch_bounds__(64) void large_csr_fill(int32_t M, const float* __restrict__ alpha,
                                                     const int32_t* __restrict__ csr_ptr,
                                                     int2* __restrict__ csr_cv,
                                                     int trans) {
    const int32_t p = blockIdx.x;
    const int lane = threadIdx.x;
    int32_t o = csr_ptr[p];
    for (int32_t q0 = 0; q0 < M; q0 += 64) {
        const int32_t q = q0 + lane;
        const float a = q < M ? alpha_at(alpha, M, p, q, trans) : 0.0f;
        const uint64_t nz = __ballot(a != 0.0f);
        if (a != 0.0f) {
            const int32_t r = __builtin_popcountll(nz & (lane ? (~0ull >> (64 - lane)) : 0ull));
            csr_cv[o + r] = make_int2(q, __float_as_int(a));
        }
        o += __builtin_popcountll(nz);
    }
}

// node_info[p] = (csr begin, csr end, mu_p, colsum_p): one 16-byte load per event
__global__ void large_node_info(int32_t M, const int32_t* __restrict__ csr_ptr, const float* __restrict__ mu,
                                const float* __restrict__ colsum, int4* __restrict__ node_info) {
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    node_info[p] = make_int4(csr_ptr[p], csr_ptr[p + 1], __float_as_int(mu[p]), __float_as_int(colsum[p]));
}

// ------------------------------------------------------------------ agg
// one wave per segment; LDS: aggK[M], aggJ[M] (float64)
__global__ __launch_bounds__(64) void large_seg_agg(int64_t c0, int64_t c1, int32_t M, const double* __restrict__ t,
                                                    const int32_t* __restrict__ marks, const float* __restrict__ beta,
                                                    double* __restrict__ agg, double* __restrict__ seg_span,
                                                    double* __restrict__ seg_dec) {
    extern __shared__ double lds[];
    double* aK = lds;
    double* aJ = lds + M;
    const int32_t s = blockIdx.x;
    const int64_t a = c0 + (int64_t)s * HK_SEG;
    const int64_t b = a + HK_SEG < c1 ? a + HK_SEG : c1;
    const int lane = threadIdx.x;
    for (int32_t q = lane; q < M; q += 64) { aK[q] = 0.0; aJ[q] = 0.0; }
    __syncthreads();
    const double bet = (double)beta[0];
    const double te = t[b - 1];
    // the segment's times and marks, all loads issued up front (past the
    // end: a valid index, not added)
    constexpr int NBT = HK_SEG / 64;
    double ts[NBT];
    int mks[NBT];
#pragma unroll
    for (int u = 0; u < NBT; ++u) {
        const int64_t i = a + 64 * u + lane;
        const int64_t ic = i < b ? i : b - 1;
        ts[u] = t[ic];
        mks[u] = marks[ic];
    }
#pragma unroll
    for (int u = 0; u < NBT; ++u) {
        if (a + 64 * u + lane < b) {
            const double d = te - ts[u];
            const double e = exp_f64(-bet * d);
            const int mi = clamp_mark(mks[u], M);
            atomicAdd(&aK[mi], e);
            atomicAdd(&aJ[mi], d * e);
        }
    }
    __syncthreads();
    double* o = agg + (int64_t)s * 2 * M;
    for (int32_t q = lane; q < M; q += 64) { o[q] = aK[q]; o[M + q] = aJ[q]; }
    if (lane == 0) {
        // span and decay from the event before the segment to its last event
        const double tr = a > 0 ? t[a - 1] : t[a];
        seg_span[s] = te - tr;
        seg_dec[s] = exp(-bet * (te - tr));
    }
}

// ------------------------------------------------------------------ scan
// Segment maps are chained in three parallel steps (groups of HK_SG segments):
//   1 thread per (group, node): exclusive prefix inside the group, group map
//   2 thread per node: chain the group maps from the chunk carry
//   3 thread per (segment, node): carry_seg[s] = group carry moved to the
//     segment start, plus the in-group prefix
// carry_seg[s] is the state just after the event preceding segment s.

// beta_pt: per-target decays (R-form state) or nullptr (one shared decay,
// seg_dec / gdec precomputed)
// The threads also write the group's gspan/gdec and every segment's
// seg_off/seg_offdec: the time from the event before the group to the event
// before the segment, and its decay (shared decay beta[0]).
__global__ __launch_bounds__(256) void large_scan_local(int32_t nseg, int32_t M, const double* __restrict__ agg,
                                 const double* __restrict__ seg_dec, const double* __restrict__ seg_span,
                                 double* __restrict__ carry_seg, double* __restrict__ gagg,
                                 const float* __restrict__ beta_pt, const float* __restrict__ beta,
                                 double* __restrict__ gspan, double* __restrict__ gdec,
                                 double* __restrict__ seg_off, double* __restrict__ seg_offdec) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int32_t ngr = (nseg + HK_SG - 1) / HK_SG;
    if (gid >= (int64_t)ngr * M) return;
    const int32_t g = (int32_t)(gid / M), q = (int32_t)(gid % M);
    const int32_t s0 = g * HK_SG, s1 = s0 + HK_SG < nseg ? s0 + HK_SG : nseg;
    // offset u of the group (u = 0 .. s1 - s0, the last one the group's
    // span) is summed by the threads q = u, u + M, ..: each sums the spans in
    // the same order as one serial pass would, so the values do not depend on
    // M, and the group's exps run side by side instead of one after another
    if (q <= s1 - s0) {
        // the group's spans, loaded together (not one dependent load per
        // term of the sum)
        double sp[HK_SG];
#pragma unroll
        for (int v = 0; v < HK_SG; ++v) sp[v] = seg_span[s0 + v < s1 ? s0 + v : s1 - 1];
    for (int32_t u = q; u <= s1 - s0; u += M) {
        const double b0 = (double)beta[0];
        double D = 0.0;
#pragma unroll
        for (int v = 0; v < HK_SG; ++v)
            if (v < u) D += sp[v];
        const double e = exp(-b0 * D);
        if (u < s1 - s0) {
            seg_off[s0 + u] = D;
            seg_offdec[s0 + u] = e;
        } else {
            gspan[g] = D;
            gdec[g] = e;
        }
    }
    }
    double K = 0.0, J = 0.0;
    const double bq = beta_pt ? (double)beta_pt[q] : 0.0;
    // the group's segment maps of node q, all loads issued up front
    double rk[HK_SG], rj[HK_SG];
#pragma unroll
    for (int u = 0; u < HK_SG; ++u) {
        const int32_t s = s0 + u < s1 ? s0 + u : s1 - 1;
        rk[u] = agg[(int64_t)s * 2 * M + q];
        rj[u] = agg[(int64_t)s * 2 * M + M + q];
    }
#pragma unroll
    for (int u = 0; u < HK_SG; ++u) {
        const int32_t s = s0 + u;
        if (s < s1) {
            double* o = carry_seg + (int64_t)s * 2 * M;
            o[q] = K;
            o[M + q] = J;
            const double D = seg_span[s];
            const double ex = beta_pt ? exp(-bq * D) : seg_dec[s];
            const double k0 = K;
            K = __builtin_fma(ex, k0, rk[u]);
            J = __builtin_fma(ex, __builtin_fma(D, k0, J), rj[u]);
        }
    }
    gagg[(int64_t)g * 2 * M + q] = K;
    gagg[(int64_t)g * 2 * M + M + q] = J;
}

__global__ __launch_bounds__(256) void large_scan_groups(int32_t nseg, int32_t M, const double* __restrict__ gagg,
                                  const double* __restrict__ gspan, const double* __restrict__ gdec,
                                  double* __restrict__ gcarry, double* __restrict__ carry,
                                  const float* __restrict__ beta_pt) {
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M) return;
    const int32_t ngr = (nseg + HK_SG - 1) / HK_SG;
    double K = carry[q], J = carry[M + q];
    const double bq = beta_pt ? (double)beta_pt[q] : 0.0;
    // 16 group maps of node q at a time, their loads issued up front
    constexpr int PF = 16;
    for (int32_t g0 = 0; g0 < ngr; g0 += PF) {
        double gk[PF], gj[PF];
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int32_t g = g0 + u < ngr ? g0 + u : ngr - 1;
            gk[u] = gagg[(int64_t)g * 2 * M + q];
            gj[u] = gagg[(int64_t)g * 2 * M + M + q];
        }
#pragma unroll
        for (int u = 0; u < PF; ++u) {
            const int32_t g = g0 + u;
            if (g < ngr) {
                gcarry[(int64_t)g * 2 * M + q] = K;
                gcarry[(int64_t)g * 2 * M + M + q] = J;
                const double D = gspan[g];
                const double ex = beta_pt ? exp(-bq * D) : gdec[g];
                const double k0 = K;
                K = __builtin_fma(ex, k0, gk[u]);
                J = __builtin_fma(ex, __builtin_fma(D, k0, J), gj[u]);
            }
        }
    }
    carry[q] = K;
    carry[M + q] = J;
}

__global__ void large_scan_apply(int32_t nseg, int32_t M, const double* __restrict__ seg_off,
                                 const double* __restrict__ seg_offdec, const double* __restrict__ gcarry,
                                 double* __restrict__ carry_seg, const float* __restrict__ beta_pt) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid >= (int64_t)nseg * M) return;
    const int32_t s = (int32_t)(gid / M), q = (int32_t)(gid % M);
    const int32_t g = s / HK_SG;
    const double D = seg_off[s];
    const double ex = beta_pt ? exp(-(double)beta_pt[q] * D) : seg_offdec[s];
    const double Kc = gcarry[(int64_t)g * 2 * M + q], Jc = gcarry[(int64_t)g * 2 * M + M + q];
    double* o = carry_seg + (int64_t)s * 2 * M;
    const double Kl = o[q], Jl = o[M + q];
    o[q] = __builtin_fma(ex, Kc, Kl);
    o[M + q] = __builtin_fma(ex, __builtin_fma(D, Kc, Jc), Jl);
}

// ------------------------------------------------------------------ forward
#ifndef HK_FWW
#define HK_FWW 2   // waves per forward-pass segment
#endif
#ifndef HK_FW
#define HK_FW 16   // nonzeros of an event's row of alpha loaded one batch ahead
#endif
// RM (several decay kernels): the pass runs once per kernel and writes, per
// event, R = alpha_{m_i,:} . K(t_i) to rk and (GRAD) D = alpha_{m_i,:} . J(t_i)
// to dk instead of forming lambda; large_combine then sums the kernels.
// SUPP (with GRAD): also adds beta w_i K_q(t_i) to gsup[k] for every nonzero
// k = (m_i, q) of alpha's CSR (hardware float64 atomics): the first term of
// eq. 9 on alpha's support only.  Segment s adds into copy s & cmask (copies
// MM apart): consecutive workgroups go to different XCDs, so each copy sees
// mostly one XCD's atomics and a copy's addresses see a fraction of the
// contention.
// X (optional parts, each off when its pointer is null):
//   gcarry    carry_seg holds only the in-group prefixes of the scan
//             (large_scan without its apply pass): the state entering segment
//             s is formed here from its group's carry, seg_off and seg_offdec
//   bcnt      the chunk partition's counts, events per (node block of 2^bs
//             nodes, segment), written as bucket_count would
// 1 / x for a positive normal float64 x: the hardware reciprocal and two
// Newton steps (within about 1 ulp; an IEEE division takes twice the
// instructions)
__device__ __forceinline__ double recip(double x) {
    double r = __builtin_amdgcn_rcp(x);
    r = __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

template <bool GRAD, bool INTENS, bool SUPP, int NW, bool RM = false>
__global__ __launch_bounds__(64 * NW) void large_forward(int64_t c0, int64_t c1, int32_t M, double T,
                                                    const double* __restrict__ t, const int32_t* __restrict__ marks,
                                                    const float* __restrict__ mu, const float* __restrict__ beta,
                                                    const int4* __restrict__ node_info,
                                                    const int2* __restrict__ csr_cv,
                                                    const double* __restrict__ carry_seg,
                                                    double* __restrict__ seg_part,
                                                    float* __restrict__ wchunk,
                                                    float* __restrict__ lambda_out,
                                                    double* __restrict__ gsup, int32_t cmask,
                                                    double* __restrict__ rk, double* __restrict__ dk,
                                                    FwdExtra X) {
    extern __shared__ double lds[];
    double2* rKJ = reinterpret_cast<double2*>(lds);       // [M] (K_q, J_q) at rtau (event included)
    uint64_t* rmask = (uint64_t*)(lds + 2 * M);           // [M] lanes of this batch with mark q
    __shared__ double tb[64], eb[64];
    __shared__ double Rs[(NW > 1 ? NW - 1 : 1) * 64], Ds[(NW > 1 ? NW - 1 : 1) * 64];   // other waves' partial sums
    const int32_t s = blockIdx.x;
    const int lane = threadIdx.x & 63;
    // NW waves share a segment's events; wave wv takes the aligned pairs of
    // nonzeros wv, wv + NW, ... of each event's row of alpha
    const int wv = NW == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    static_assert(!SUPP || NW == 1, "the support-restricted sums are formed by one wave");
    static_assert(!(RM && (SUPP || INTENS)), "per-kernel sums only");
    const int64_t a = c0 + (int64_t)s * HK_SEG;
    const int64_t b = a + HK_SEG < c1 ? a + HK_SEG : c1;
    const double bet = (double)beta[0];
    const double tref = a > 0 ? t[a - 1] : t[a];
    // anchored records when the segment's span allows: with u = t - tref,
    // rKJ[q] = (S0_q, S1_q) with S0_q = sum_j e^{beta u_j}, S1_q = sum_j u_j e^{beta u_j}
    // over the node's events so far (the carry enters as S0 = K(tref),
    // S1 = -J(tref)); then K_q(t) = e^{-beta u} S0_q and
    // J_q(t) = e^{-beta u} (u S0_q - S1_q): one exponential per event instead
    // of one per nonzero of alpha's row, and records grow by plain additions.
    // Otherwise (beta u could overflow float64) each record keeps its own
    // time rtau[q] and is decayed on use.
    const bool anch = bet * (t[b - 1] - tref) <= 600.0;
    // [M] the lazy records' times, in the segment's slot of a global scratch
    // buffer (24 bytes of LDS per node instead of 32: M up to 6741).  Three
    // waves per SIMD (168 registers, six workgroups per CU at M = 1000) made
    // the pass slower at c4's shape: 0.674 against 0.591 ms per step
    double* rtau = X.rtau + (int64_t)s * 2 * M;
    const double* cs = carry_seg + (int64_t)s * 2 * M;
    const double* gc = X.gcarry ? X.gcarry + (int64_t)(s / HK_SG) * 2 * M : nullptr;
    const double Dg = gc ? X.seg_off[s] : 0.0, exg = gc ? X.seg_offdec[s] : 0.0;
    for (int32_t q = threadIdx.x; q < M; q += 64 * NW) {
        double Kq = cs[q], Jq = cs[M + q];
        if (gc) {
            // the group's carry moved to the segment start, plus the prefix
            const double Kc = gc[q];
            Jq = __builtin_fma(exg, __builtin_fma(Dg, Kc, gc[M + q]), Jq);
            Kq = __builtin_fma(exg, Kc, Kq);
        }
        if (!anch) rtau[q] = tref;
        rKJ[q] = make_double2(Kq, anch ? -Jq : Jq);
        rmask[q] = 0ull;
    }
    // events per node block (partition counts): dynamic LDS after the
    // records, present when bcnt is given
    int32_t* lcnt = reinterpret_cast<int32_t*>(lds + 3 * M);
    if (X.bcnt)
        for (int32_t k = threadIdx.x; k < X.nbo; k += 64 * NW) lcnt[k] = 0;
    __syncthreads();
    double logsum = 0.0, comp = 0.0, Esum = 0.0, gb = 0.0;
    // software pipeline over batches of 64 events: times and marks are loaded
    // three batches ahead, node records two ahead and the first FW nonzeros
    // of each event's row of alpha one ahead (clamped indices keep every load
    // valid), so the gathers' latency hides behind a batch of work.  The row
    // is read in aligned pairs of entries (pair P holds entries 2P and 2P + 1,
    // one 16-byte load; the first and last pair may hold a neighbour row's
    // entry, which is skipped): these gathers hit a different cache line per
    // lane, so the number of load instructions, not bytes, sets their cost.
    constexpr int FW = HK_FW;          // nonzeros loaded ahead per event
    constexpr int FP = FW / (2 * NW);  // pairs of them loaded by this wave
    static_assert(FP >= 1 && FP * 2 * NW == FW, "look-ahead must be whole pairs per wave");
    const int4* __restrict__ cv4 = reinterpret_cast<const int4*>(csr_cv);
    auto ld_tm = [&](int64_t base, double& tt, int& mm) {
        const int64_t j = base + lane;
        const int64_t jc = j < b ? j : b - 1;
        tt = t[jc];
        mm = clamp_mark(marks[jc], M);
    };
    // pairs past the row's last entry are replaced by its first pair (an
    // empty row reads pair nv.x / 2, inside the array's one spare pair)
    auto ld_row = [&](const int4& nv, int4 (&pr)[FP]) {
        const int32_t p0 = nv.x >> 1, pl = (nv.y - 1) >> 1;
#pragma unroll
        for (int j = 0; j < FP; ++j) {
            const int32_t P = p0 + NW * j + wv;
            pr[j] = cv4[P <= pl ? P : p0];
        }
    };
    double t0, t1, t2;
    int m0, m1, m2;
    ld_tm(a, t0, m0);
    ld_tm(a + 64, t1, m1);
    ld_tm(a + 128, t2, m2);
    int4 n0 = node_info[m0], n1 = node_info[m1];
    int4 pr0[FP];
    ld_row(n0, pr0);
    for (int64_t base = a; base < b; base += 64) {
        const int64_t i = base + lane;
        const bool valid = i < b;
        const double ti = valid ? t0 : 0.0;
        const int mi = valid ? m0 : 0;
        const int4 ni = n0;
        // loads for the batches ahead
        double t3;
        int m3;
        ld_tm(base + 192, t3, m3);
        const int4 n2 = node_info[m2];
        int4 pr1[FP];
        ld_row(n1, pr1);
        const double ui = ti - tref;
        // the last wave takes the batch's compensator terms (they do not need
        // the sums), beside the first wave's logarithm and reciprocal (one
        // wave: the first does all)
        constexpr int WC = NW - 1;
        double eti = 0.0;   // e^{beta u_i} (anchored records; the first wave)
        if (wv == 0) {
            eti = anch && valid ? exp_f64(bet * ui) : 0.0;
            tb[lane] = ti;
            eb[lane] = eti;
            if (valid) atomicOr((unsigned long long*)&rmask[mi], 1ull << lane);
            if (X.bcnt && valid) atomicAdd(&lcnt[mi >> X.bs], 1);
        }
        __syncthreads();
        double R = 0.0, Dd = 0.0, lam = 1.0, w = 0.0, em1 = 0.0;
        const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        const int32_t k0 = ni.x, k1 = ni.y, p0 = k0 >> 1;
        double ks[SUPP ? 2 * FP : 1];   // the loaded pairs' sums, for gsup (NW = 1)
            // anchored sums of source q (records plus the batch's earlier
            // events of q): K_q(t_i) = e^{-beta u_i} s0
            auto sums_a = [&](int32_t q, double& s0, double& s1) {
                const double2 kj = rKJ[q];   // one LDS read for both
                s0 = kj.x;
                s1 = GRAD ? kj.y : 0.0;
                uint64_t bits = rmask[q] & below;
                while (bits) {
                    const int jj = __builtin_ctzll(bits);
                    bits &= bits - 1;
                    const double ej = eb[jj];
                    s0 += ej;
                    if (GRAD) s1 = __builtin_fma(tb[jj] - tref, ej, s1);
                }
            };
            // source q's record decayed to ti plus the batch's earlier events
            // of q: Kv = K_q(t_i), Jv = J_q(t_i)
            auto sums_w = [&](int32_t q, double& Kv, double& Jv) {
                const double d = ti - rtau[q];
                const double e = exp_f64(-bet * d);
                const double2 kj = rKJ[q];
                const double kq = kj.x;
                Kv = e * kq;
                Jv = GRAD ? e * __builtin_fma(d, kq, kj.y) : 0.0;
                uint64_t bits = rmask[q] & below;
                while (bits) {
                    const int jj = __builtin_ctzll(bits);
                    bits &= bits - 1;
                    const double dj = ti - tb[jj];
                    const double ej = exp_f64(-bet * dj);
                    Kv += ej;
                    if (GRAD) Jv = __builtin_fma(dj, ej, Jv);
                }
            };
            if (!valid) {
            } else if (anch) {
                // source q with weight av
                auto terma = [&](int32_t q, float av) -> double {
                    double s0, s1;
                    sums_a(q, s0, s1);
                    R = __builtin_fma((double)av, s0, R);
                    if (GRAD) Dd = __builtin_fma((double)av, __builtin_fma(ui, s0, -s1), Dd);
                    return s0;
                };
#pragma unroll
                for (int j = 0; j < FP; ++j) {
                    const int32_t kb = 2 * (p0 + NW * j + wv);
                    if (kb < k1) {
                        if (kb >= k0) {
                            const double v = terma(pr0[j].x, __int_as_float(pr0[j].y));
                            if (SUPP) ks[2 * j] = v;
                        }
                        if (kb + 1 < k1) {
                            const double v = terma(pr0[j].z, __int_as_float(pr0[j].w));
                            if (SUPP) ks[2 * j + 1] = v;
                        }
                    }
                }
                for (int32_t kb = 2 * (p0 + NW * FP + wv); kb < k1; kb += 2 * NW) {
                    const int4 e = cv4[kb >> 1];
                    terma(e.x, __int_as_float(e.y));
                    if (kb + 1 < k1) terma(e.z, __int_as_float(e.w));
                }
            } else {
            auto term = [&](int32_t q, float av) -> double {
                double Kv, Jv;
                sums_w(q, Kv, Jv);
                R = __builtin_fma((double)av, Kv, R);
                if (GRAD) Dd = __builtin_fma((double)av, Jv, Dd);
                return Kv;
            };
#pragma unroll
            for (int j = 0; j < FP; ++j) {
                const int32_t kb = 2 * (p0 + NW * j + wv);
                if (kb < k1) {
                    if (kb >= k0) {
                        const double v = term(pr0[j].x, __int_as_float(pr0[j].y));
                        if (SUPP) ks[2 * j] = v;
                    }
                    if (kb + 1 < k1) {
                        const double v = term(pr0[j].z, __int_as_float(pr0[j].w));
                        if (SUPP) ks[2 * j + 1] = v;
                    }
                }
            }
            for (int32_t kb = 2 * (p0 + NW * FP + wv); kb < k1; kb += 2 * NW) {
                const int4 e = cv4[kb >> 1];
                term(e.x, __int_as_float(e.y));
                if (kb + 1 < k1) term(e.z, __int_as_float(e.w));
            }
            }
        if (NW > 1) {
            // the other waves' partial sums to the first, added in wave order
            if (wv > 0) {
                Rs[(wv - 1) * 64 + lane] = R;
                Ds[(wv - 1) * 64 + lane] = Dd;
            }
            __syncthreads();
            if (wv == 0) {
#pragma unroll
                for (int v = 0; v < NW - 1; ++v) {
                    R += Rs[v * 64 + lane];
                    Dd += Ds[v * 64 + lane];
                }
            }
        }
        // e^{-beta u_i} (anchored records) as the reciprocal of e^{beta u_i}
        // (1 <= e^{beta u_i} <= e^600): a division instead of a second
        // exponential on the first wave, whose share of the batch is the longer
        double ei = 1.0;
        if (anch && valid && wv == 0) ei = recip(eti);
        if (!RM && valid && wv == WC) {
            // compensator terms of the event's node (eq. 2) and their
            // beta-derivative part (eq. 10)
            const double x = bet * (T - ti);
            const double ex = exp_f64(-x);
            // 1 - e^{-x}: by subtraction when every event of the batch has
            // x >= 0.5 (then 1 - e^{-x} >= 0.39 and the subtraction loses
            // nothing), else by expm1 (a wave-uniform choice)
            if (__ballot(x < 0.5) == 0)
                em1 = 1.0 - ex;
            else
                em1 = -expm1(-x);
            const double cs_m = (double)__int_as_float(ni.w);
            comp += cs_m * em1;
            if (GRAD) Esum += cs_m * (T - ti) * ex;
        }
        if (RM && valid && wv == 0) {
            if (anch) {
                R *= ei;
                Dd *= ei;
            }
            rk[i - c0] = R;
            if (GRAD) dk[i - c0] = Dd;
        } else if (valid && wv == 0) {
            if (anch) {
                R *= ei;
                Dd *= ei;
            }
            lam = __builtin_fma(bet, R, (double)__int_as_float(ni.z));
        if (INTENS) lambda_out[i] = (float)lam;
            logsum += log(lam);
            if (GRAD) {
                w = recip(lam);
                gb += w * (R - bet * Dd);
            }
            if (SUPP) {
                // beta w_i K_q(t_i) for each nonzero (m_i, q); the sums past
                // the loaded pairs are formed again
                const double bw = bet * w * ei;
                double* gs = gsup + (int64_t)(s & cmask) * M * M;
#pragma unroll
                for (int j = 0; j < 2 * FP; ++j) {
                    const int32_t k = 2 * p0 + j;
                    if (k >= k0 && k < k1) unsafeAtomicAdd(&gs[k], bw * ks[j]);
                }
                for (int32_t k = 2 * (p0 + FP); k < k1; ++k) {
                    double v, unused;
                    if (anch)
                        sums_a(csr_cv[k].x, v, unused);
                    else
                        sums_w(csr_cv[k].x, v, unused);
                    unsafeAtomicAdd(&gs[k], bw * v);
                }
            }
        }
        if (!RM && GRAD && valid && wv == 0) wchunk[i - c0] = (float)w;
        // the records take the batch's events (the last wave, beside the
        // first wave's work above: nothing there reads the records), then the
        // batch's masks are cleared
        if (anch) {
            // anchored records: the batch's events of a node add their terms,
            // in index order, through one leader lane per node
            if (valid && wv == WC) {
                uint64_t grp = rmask[mi];
                if (__builtin_ctzll(grp) == lane) {
                    const double2 kj = rKJ[mi];
                    double s0 = kj.x, s1 = kj.y;
                    while (grp) {
                        const int j = __builtin_ctzll(grp);
                        grp &= grp - 1;
                        s0 += eb[j];
                        if (GRAD) s1 = __builtin_fma(tb[j] - tref, eb[j], s1);
                    }
                    rKJ[mi] = make_double2(s0, s1);
                }
            }
        } else if (valid && wv == WC) {
            // lazy record update, one leader lane per node, events in index order
            uint64_t grp = rmask[mi];
            if (__builtin_ctzll(grp) == lane) {
                double tq = rtau[mi];
                const double2 kj = rKJ[mi];
                double kq = kj.x, jq = kj.y;
                while (grp) {
                    const int j = __builtin_ctzll(grp);
                    grp &= grp - 1;
                    const double d = tb[j] - tq;
                    const double e = exp_f64(-bet * d);
                    jq = e * __builtin_fma(d, kq, jq);
                    kq = __builtin_fma(e, kq, 1.0);
                    tq = tb[j];
                }
                rtau[mi] = tq;
                rKJ[mi] = make_double2(kq, jq);
            }
        }
        if (wv == WC) {
            lds_wait();   // every lane's read of its mask before the clear
            if (valid) rmask[mi] = 0ull;
        }
        __syncthreads();
        t0 = t1;
        m0 = m1;
        t1 = t2;
        m1 = m2;
        t2 = t3;
        m2 = m3;
        n0 = n1;
        n1 = n2;
#pragma unroll
        for (int j = 0; j < FP; ++j) pr0[j] = pr1[j];
    }
    if (X.bcnt) {
        __syncthreads();
        for (int32_t k = threadIdx.x; k < X.nbo; k += 64 * NW) X.bcnt[(int64_t)k * gridDim.x + s] = lcnt[k];
    }
    // deterministic wave reductions of the float64 partials: the log-sum and
    // dL/dbeta part in the first wave, the compensator sums in the last
    if (RM || (wv != 0 && wv != NW - 1)) return;
    for (int off = 32; off > 0; off >>= 1) {
        logsum += __shfl_down(logsum, off, 64);
        comp += __shfl_down(comp, off, 64);
        Esum += __shfl_down(Esum, off, 64);
        gb += __shfl_down(gb, off, 64);
    }
    // the segment slot's sums over the chunks so far (slot s of every chunk,
    // in chunk order; one reduction over the slots ends the call)
    if (lane == 0) {
        double* o = seg_part + (int64_t)s * 4;
        if (wv == 0) {
            o[0] += logsum;
            o[3] += gb;
        }
        if (wv == NW - 1) {
            o[1] += comp;
            o[2] += Esum;
        }
    }
}

// acc[k] += sum over segments of seg_part[s][k] (width values per segment);
// per value a fixed-order tree (deterministic), four values per pass
__global__ __launch_bounds__(256) void large_chunk_acc(int32_t nseg, int32_t width,
                                                       const double* __restrict__ seg_part,
                                                       double* __restrict__ acc) {
    __shared__ double sh[4][256];
    const int tid = threadIdx.x;
    for (int k0 = 0; k0 < width; k0 += 4) {
        double v[4] = {0.0, 0.0, 0.0, 0.0};
        for (int32_t s = tid; s < nseg; s += 256)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (k0 + j < width) v[j] += seg_part[(int64_t)s * width + k0 + j];
#pragma unroll
        for (int j = 0; j < 4; ++j) sh[j][tid] = v[j];
        __syncthreads();
        for (int st = 128; st > 0; st >>= 1) {
            if (tid < st)
#pragma unroll
                for (int j = 0; j < 4; ++j) sh[j][tid] += sh[j][tid + st];
            __syncthreads();
        }
        if (tid < 4 && k0 + tid < width) acc[k0 + tid] += sh[tid][0];
        __syncthreads();
    }
}

// Several decay kernels (Background, eq. 1 with K > 1): the per-kernel
// forward passes left R_k(i) = alpha^k_{m_i,:} . K^k(t_i) and D_k(i) =
// alpha^k_{m_i,:} . J^k(t_i) for each event of the chunk; here
//   lambda_i = mu_{m_i} + sum_k beta_k R_k(i),   w_i = 1 / lambda_i,
// and the segment's float64 partials: log-sum, compensator
// sum_k colsum_k[m_i] (1 - e^{-beta_k (T - t_i)}), and per kernel E_k (its
// beta-derivative) and sum_i w_i (R_k(i) - beta_k D_k(i)) (eq. 10 per kernel).
// One workgroup of 256 per segment, fixed-order block sums.
template <bool GRAD, bool INTENS>
__global__ __launch_bounds__(256) void large_combine(int64_t c0, int64_t c1, int32_t M, int32_t K, double T,
                                                     const double* __restrict__ t,
                                                     const int32_t* __restrict__ marks,
                                                     const float* __restrict__ mu, const float* __restrict__ beta,
                                                     const float* __restrict__ colsum,
                                                     const double* __restrict__ rk, const double* __restrict__ dk,
                                                     int64_t CH, double* __restrict__ seg_part,
                                                     float* __restrict__ wchunk, float* __restrict__ lambda_out) {
    __shared__ double sh[256];
    const int32_t s = blockIdx.x;
    const int64_t a = c0 + (int64_t)s * HK_SEG;
    const int64_t b = a + HK_SEG < c1 ? a + HK_SEG : c1;
    double logsum = 0.0, comp = 0.0, E[HK_KMAX], gb[HK_KMAX];
#pragma unroll
    for (int k = 0; k < HK_KMAX; ++k) E[k] = gb[k] = 0.0;
    for (int64_t i = a + threadIdx.x; i < b; i += 256) {
        const int mi = clamp_mark(marks[i], M);
        const double ti = t[i];
        const int64_t r = i - c0;
        double lam = (double)mu[mi];
        for (int k = 0; k < K; ++k) lam = __builtin_fma((double)beta[k], rk[k * CH + r], lam);
        if (INTENS) lambda_out[i] = (float)lam;
        logsum += log(lam);
        const double w = 1.0 / lam;
        if (GRAD) wchunk[r] = (float)w;
#pragma unroll
        for (int k = 0; k < HK_KMAX; ++k) {
            if (k < K) {
                const double bk = (double)beta[k];
                const double x = bk * (T - ti);
                const double cs = (double)colsum[(int64_t)k * M + mi];
                comp += cs * -expm1(-x);
                if (GRAD) {
                    E[k] += cs * (T - ti) * exp_f64(-x);
                    gb[k] += w * (rk[k * CH + r] - bk * dk[k * CH + r]);
                }
            }
        }
    }
    const int W = 2 + 2 * K;
    double* o = seg_part + (int64_t)s * W;
    double v = block_sum_d<256>(logsum, sh);
    if (threadIdx.x == 0) o[0] = v;
    v = block_sum_d<256>(comp, sh);
    if (threadIdx.x == 0) o[1] = v;
#pragma unroll
    for (int k = 0; k < HK_KMAX; ++k) {
        if (k < K) {
            v = block_sum_d<256>(E[k], sh);
            if (threadIdx.x == 0) o[2 + k] = v;
            v = block_sum_d<256>(gb[k], sh);
            if (threadIdx.x == 0) o[2 + K + k] = v;
        }
    }
}

// ------------------------------------------------------------------ finalize
// column sums of the per-run partials (dL/dmu sums, compensator terms),
// folded into row 0, each in a fixed order
__global__ void large_colfold(int32_t M, int32_t NSC, double* __restrict__ spart, double* __restrict__ cpart) {
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M) return;
    double s = 0.0, c = 0.0;
#pragma unroll 16
    for (int32_t e = 0; e < NSC; ++e) {
        s += spart[(int64_t)e * M + q];
        c += cpart[(int64_t)e * M + q];
    }
    spart[q] = s;
    cpart[q] = c;
}

// Kernel k of K (decay kernels): the log-likelihood and dL/dmu with k = 0,
// dL/dbeta_k from the call-level sums acc = (logsum, comp, E[K], gbeta[K]),
// dL/dalpha of kernel k from its partials (g_alpha, gpart and cpart point at
// kernel k's).
__global__ __launch_bounds__(256) void large_final(int32_t M, int32_t ER, int32_t NSC, double T, const float* __restrict__ mu,
                            const double* __restrict__ acc, const double* __restrict__ gpart,
                            const double* __restrict__ spart, const double* __restrict__ cpart,
                            double* __restrict__ loglik, double* __restrict__ g_mu, double* __restrict__ g_alpha,
                            double* __restrict__ g_beta, int grad, int sup, int32_t K, int32_t k) {
    const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t MM = (int64_t)M * M;
    if (blockIdx.x == 0) {
        // sum of mu in a fixed order: strided partial sums, then a tree
        __shared__ double ps[256];
        double v = 0.0;
        for (int32_t p = threadIdx.x; p < M; p += 256) v += (double)mu[p];
        ps[threadIdx.x] = v;
        __syncthreads();
        for (int h = 128; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) ps[threadIdx.x] += ps[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            if (k == 0) loglik[0] = acc[0] - T * ps[0] - acc[1];
            if (grad && g_beta) g_beta[k] = acc[2 + K + k] - acc[2 + k];
        }
    }
    if (!grad) return;
    if (x < MM && g_alpha && sup) {
        g_alpha[x] = 0.0;   // large_sup_scatter then writes the support
    } else if (x < MM && g_alpha) {
        const int32_t q = (int32_t)(x % M);
        double g = 0.0, c = 0.0;
        for (int32_t e = 0; e < ER; ++e) g += gpart[(int64_t)e * MM + x];
        for (int32_t e = 0; e < NSC; ++e) c += cpart[(int64_t)e * M + q];
        g_alpha[x] = g - c;
    }
    if (x < M && g_mu && k == 0) {
        double s = 0.0;
        for (int32_t e = 0; e < NSC; ++e) s += spart[(int64_t)e * M + x];
        g_mu[x] = s - T;
    }
}

// support-restricted dL/dalpha: one wave per row p writes, for each nonzero
// (p, q) of alpha, the first term summed over the ncopy copies (in order)
// minus the column's compensator sum (cpart row 0 after large_colfold); runs
// after large_final zeroed g_alpha
__global__ __launch_bounds__(64) void large_sup_scatter(int32_t M, int32_t ncopy,
                                                        const int32_t* __restrict__ csr_ptr,
                                                        const int2* __restrict__ csr_cv,
                                                        const double* __restrict__ gsup,
                                                        const double* __restrict__ cpart,
                                                        double* __restrict__ g_alpha) {
    const int32_t p = blockIdx.x;
    const int64_t MM = (int64_t)M * M;
    const int32_t k1 = csr_ptr[p + 1];
    for (int32_t k = csr_ptr[p] + (int32_t)threadIdx.x; k < k1; k += 64) {
        const int32_t q = csr_cv[k].x;
        double g = 0.0;
        for (int32_t c = 0; c < ncopy; ++c) g += gsup[c * MM + k];
        g_alpha[(int64_t)p * M + q] = g - cpart[q];
    }
}

// ------------------------------------------------------------------ host
size_t large_layout(LargeArgs& A, const hawkes_problem* p, bool grad, void* ws, size_t ws_bytes) {
    A.n = p->n;
    A.M = p->m;
    A.K = p->k;
    A.per_target = p->beta_mode == HAWKES_BETA_PER_TARGET;
    A.T = p->T;
    // chunks no longer than the sequence needs (at least 2^12 events): the
    // per-chunk buffers then scale with n for short sequences
    int lg = p->chunk_log2 ? p->chunk_log2 : 20;
    while (lg > 12 && ((int64_t)1 << (lg - 1)) >= p->n) --lg;
    A.CH = (int64_t)1 << lg;
    A.nchunks = (A.n + A.CH - 1) / A.CH;
    A.nseg = (int32_t)((A.CH + HK_SEG - 1) / HK_SEG);
    A.NB = (A.M + 63) / 64;
    // shared decay: tiles of DR = 16 rows x W = 64 CPL columns.  Every own
    // event is visited once per column block (a pair-term instruction each),
    // every window once per row block (state loads and the rank-1 update),
    // and G takes 16 CPL float64 registers per lane: 16 x 256 is the fastest
    // that fits (two waves per SIMD), with 16 x 128 and 16 x 64 for the
    // longer chunks, since a column record key holds the event index above
    // log2(W) bits, and no wider than the nodes need.  A tuned width
    // (hawkes_set_tuning) replaces the rule where the chunk allows it.
    const hawkes_tuning tu = tuning_snapshot();
    A.CPL = A.per_target ? 1 : lg <= 24 ? 4 : lg <= 25 ? 2 : 1;
    while (A.CPL > 1 && 32 * A.CPL >= A.M) A.CPL >>= 1;
    if (!A.per_target && tu.dense_cols > 0) {
        const int v = tu.dense_cols / 64;
        const int vlg = v == 4 ? 24 : v == 2 ? 25 : 26;
        if (lg <= vlg) A.CPL = v;
    }
    A.DRB = 4;
    // window length of the dense kernel: a 64-record window holds about
    // 1024 / max(W, M) own events of a 16-row block; with fewer than 8 the
    // rank-1 update's u is mostly zero, and 128-record windows halve the
    // per-window work at about 1.5 pair instructions per own event
    {
        const int Wc = 64 * A.CPL;
        A.NGW = !A.per_target && 1024 / (Wc > A.M ? Wc : A.M) < 8 ? 2 : 1;
    }
    // 32-row tiles with float32 register accumulators (large_dense_f) for the
    // widest tiles at large M: half the window visits per event; the tuning
    // (dense_rows) can select either where the tiles are 256 x 128-record
    if (!A.per_target && A.CPL == 4 && A.NGW == 2) {
        if (tu.dense_rows == 32 || (tu.dense_rows == 0 && A.M >= HK_F32_MIN_M)) A.DRB = 5;
    }
    const int nwv = A.DRB == 5 ? HK_DWF : HK_DW;   // waves per dense workgroup
    A.NBR = A.per_target ? A.NB : (A.M + (1 << A.DRB) - 1) >> A.DRB;
    A.NBC = A.per_target ? A.NB : (A.M + 64 * A.CPL - 1) / (64 * A.CPL);
    // event ranges per chunk for the dense kernel: a power of two so that the
    // ranges map onto the 8 XCDs evenly; about 4096 workgroups in total
    // (shared decay: two waves each, 18 KiB of LDS per group, so that several
    // rounds balance the waves' uneven work) or 2048 (per target, 34 KiB;
    // 16 x 256 tiles, 34 KiB and two waves per SIMD: measured best at c4's
    // size) unless the tuning (hawkes_set_tuning) sets it
    // (32-row float32-accumulator tiles: 512 workgroups of four waves, two
    // resident per CU, i.e. one round; measured at c4, dense ms per launch
    // with 4 / 8 / 16 / 32 ranges: 0.416 / 0.420 / 0.434 / 0.534, and a
    // quarter of the partials' traffic at 4)
    const int64_t nbb = (int64_t)A.NBR * A.NBC;
    const int64_t target = A.DRB == 5 ? 2048 / HK_DWF : A.per_target || A.CPL == 4 ? 2048 : 4096;
    const int64_t want = (target + nbb - 1) / nbb;
    int32_t er = 1;
    while (er < want) er <<= 1;
    if (!A.per_target && tu.dense_ranges > 0) er = tu.dense_ranges;   // a knob of the shared-decay kernel only
    while (er > A.nseg && er > 1) er >>= 1;
    // shared decay: every wave of a dense workgroup gets at least one run
    while (!A.per_target && er > 1 && A.nseg / er < nwv) er >>= 1;
    A.ER = er;
    // checkpoint runs: whole runs per event range, nwv or more per range
    // (nseg and ER are powers of two)
    A.CKR = A.nseg / (er * nwv);
    if (A.CKR > HK_CKR) A.CKR = HK_CKR;
    if (A.CKR < 1) A.CKR = 1;
    A.NRUN = A.nseg / A.CKR;
    A.grad = grad;
    const int64_t M = A.M, MM = M * M, K = A.K;
    Carve c(ws, ws_bytes);
    A.csr_ptr = c.take<int32_t>(K * (M + 1));
    A.csr_cv = c.take<int2>(K * cv_stride(MM));
    A.colsum = c.take<float>(K * M);
    if (K > 1) {
        A.rk = c.take<double>((size_t)K * A.CH);
        if (grad) A.dk = c.take<double>((size_t)K * A.CH);
    }
    A.agg = c.take<double>((size_t)A.nseg * 2 * M);
    A.seg_span = c.take<double>(A.nseg);
    A.seg_dec = c.take<double>(A.nseg);
    A.seg_off = c.take<double>(A.nseg);
    A.seg_offdec = c.take<double>(A.nseg);
    A.ngr = (A.nseg + HK_SG - 1) / HK_SG;
    A.gagg = c.take<double>((size_t)A.ngr * 2 * M);
    A.gcarry = c.take<double>((size_t)A.ngr * 2 * M);
    A.gspan = c.take<double>(A.ngr);
    A.gdec = c.take<double>(A.ngr);
    A.node_info = c.take<int4>(K * M);
    A.carry_seg = c.take<double>((size_t)K * A.nseg * 2 * M);
    A.carry = c.take<double>(K * 2 * M);
    A.pt_flags = c.take<float>(2);
    A.seg_part = c.take<double>((size_t)A.nseg * (2 + 2 * K));
    A.acc = c.take<double>(2 + 2 * K);
    A.ll_scratch = c.take<double>(1);
    if (A.per_target) {
        A.csc_ptr = c.take<int32_t>(M + 1);
        A.csc_cv = c.take<int2>(MM);
        A.ebseg = c.take<double>((size_t)A.nseg * M);
        A.ebacc = c.take<double>(M);
        if (grad) {
            // constant memory: w of one chunk, and two levels of chunk-start
            // states (the chunks of each level-1 slot are chained again into
            // the level-2 slots during the reverse sweep)
            A.wv = c.take<float>((size_t)A.CH);
            A.pt_ckr = (A.nchunks + HK_PTCK - 1) / HK_PTCK;
            if (A.pt_ckr < 1) A.pt_ckr = 1;
            A.pt_ck = c.take<double>((size_t)2 * HK_PTCK * 2 * M);
            A.aggA = c.take<double>((size_t)A.nseg * M);
            A.rcarry_seg = c.take<double>((size_t)A.nseg * M);
            A.rgagg = c.take<double>((size_t)A.ngr * M);
            A.rgcarry = c.take<double>((size_t)A.ngr * M);
            A.achunk = c.take<double>(M);
        }
    }
    if (grad) {
        if (!A.per_target) A.wchunk = c.take<float>(A.CH);
        if (A.per_target) {
            A.bk_cnt = c.take<int32_t>((size_t)A.NB * A.nseg);
            A.bk_off = c.take<int32_t>((size_t)A.NB * (A.nseg + 1));
            A.bk_base = c.take<int32_t>(A.NB);
            A.bk_key = c.take<uint32_t>(A.CH);
            A.bk_t = c.take<double>(A.CH);
            A.bk_w = c.take<float>(A.CH);
        }
        A.gpart = c.take<double>((size_t)K * A.ER * MM);
        const int64_t nsp = A.per_target ? A.ER : A.NRUN;
        A.spart = c.take<double>((size_t)K * nsp * M);
        A.cpart_ = c.take<double>((size_t)K * nsp * M);
        if (!A.per_target) {
            A.nslot = A.CH / (64 * A.NGW) + 2 * (int64_t)A.NBC * A.NRUN + 2;
            A.kck = c.take<double>((size_t)A.nslot * HK_SLOT_WORDS(A.CPL, A.NGW));
            A.runinfo = c.take<int4>((size_t)A.NBC * A.NRUN);
            A.NBO = (A.M + (1 << A.DRB) - 1) >> A.DRB;
            A.bo_cnt = c.take<int32_t>((size_t)A.NBO * A.nseg);
            A.bo_off = c.take<int32_t>((size_t)A.NBO * (A.nseg + 1));
            A.bo_base = c.take<int32_t>(A.NBO);
            A.bo_key = c.take<uint32_t>(A.CH);
            A.bo_t = c.take<double>(A.CH);
            A.bo_w = c.take<float>(A.CH);
        }
    }
    return c.off + 256;
}

void large_chunk_acc_launch(int32_t nseg, int32_t width, const double* seg_part, double* acc, hipStream_t st) {
    hipLaunchKernelGGL(large_chunk_acc, dim3(1), dim3(256), 0, st, nseg, width, seg_part, acc);
}

size_t lds_limit() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        return 64 * 1024;
    return (size_t)v;
}

// Kernels whose dynamic LDS exceeds 64 KiB are allowed, once per (kernel,
// device), as much as the device's per-workgroup LDS leaves beside the
// kernel's own static LDS (asking for more than that is refused); later calls
// (including ones under stream capture) only look the pair up.  A refusal
// clears the runtime's last-error state, so that it does not surface at an
// unrelated later call.
hawkes_status allow_lds(const void* kernel, size_t bytes, bool with_static) {
    const size_t lim = lds_limit();
    if (bytes > lim) return HAWKES_EUNSUPPORTED;
    // with_static: the kernel's static LDS comes on top of `bytes`, so the
    // grant is needed even at 64 KiB of dynamic LDS
    if (!with_static && bytes <= 64 * 1024) return HAWKES_OK;
    static std::mutex mu;
    static const void* done_k[128];
    static int done_d[128];
    static size_t done_cap[128];
    static int n_done = 0;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return HAWKES_EDEVICE;
    std::lock_guard<std::mutex> g(mu);
    for (int i = 0; i < n_done; ++i)
        if (done_k[i] == kernel && done_d[i] == dev) return bytes <= done_cap[i] ? HAWKES_OK : HAWKES_EUNSUPPORTED;
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, kernel) != hipSuccess) {
        (void)hipGetLastError();
        return HAWKES_EDEVICE;
    }
    if (fa.sharedSizeBytes >= lim) return HAWKES_EUNSUPPORTED;
    const size_t cap = lim - fa.sharedSizeBytes;
    if (bytes > cap) return HAWKES_EUNSUPPORTED;
    if (hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)cap) != hipSuccess) {
        (void)hipGetLastError();
        return HAWKES_EUNSUPPORTED;
    }
    if (n_done < 128) {
        done_k[n_done] = kernel;
        done_d[n_done] = dev;
        done_cap[n_done] = cap;
        ++n_done;
    }
    return HAWKES_OK;
}

void large_build_index(int32_t M, const float* alpha, int trans, int32_t* ptr, int2* cv, hipStream_t st) {
    hipLaunchKernelGGL(large_rowcount, dim3(M), dim3(64), 0, st, M, alpha, ptr, trans);
    hipLaunchKernelGGL(large_csr_scan, dim3(1), dim3(1024), 0, st, M, ptr);
    hipLaunchKernelGGL(large_csr_fill, dim3(M), dim3(64), 0, st, M, alpha, ptr, cv, trans);
}

void large_scan(LargeArgs& A, int32_t nseg, const float* beta_pt, hipStream_t st, bool apply) {
    const int32_t M = A.M;
    // the first two passes are serial chains per thread, ngr * M and M
    // threads in all: workgroups of one wave spread them over every CU
    const unsigned gM = (unsigned)((M + 63) / 64);
    const int32_t ngr = (nseg + HK_SG - 1) / HK_SG;
    const int64_t nloc = (int64_t)ngr * M, napp = (int64_t)nseg * M;
    hipLaunchKernelGGL(large_scan_local, dim3((unsigned)((nloc + 63) / 64)), dim3(64), 0, st, nseg, M, A.agg,
                       A.seg_dec, A.seg_span, A.carry_seg, A.gagg, beta_pt, A.beta, A.gspan, A.gdec, A.seg_off,
                       A.seg_offdec);
    hipLaunchKernelGGL(large_scan_groups, dim3(gM), dim3(64), 0, st, nseg, M, A.gagg, A.gspan, A.gdec, A.gcarry,
                       A.carry, beta_pt);
    if (apply)
        hipLaunchKernelGGL(large_scan_apply, dim3((unsigned)((napp + 255) / 256)), dim3(256), 0, st, nseg, M,
                           A.seg_off, A.seg_offdec, A.gcarry, A.carry_seg, beta_pt);
}

// Several decay kernels (K > 1, shared decay per kernel; Background eq. 1,
// gradients per kernel as in eqs. 8-10).  Per chunk: for each kernel k its
// segment maps, carries and forward pass (R mode), then large_combine forms
// lambda and the shared w_i = 1/lambda_i; with the gradient the chunk's events
// are partitioned once and the dense dL/dalpha kernels run once per kernel
// (decay beta_k, kernel k's state checkpoints and partial sums).
static hawkes_status run_large_multi(LargeArgs& A, hipStream_t st) {
    const int32_t M = A.M, K = A.K;
    const int64_t MM = (int64_t)M * M;
    const unsigned gM = (unsigned)((M + 255) / 256);
    const size_t lds_agg = (size_t)2 * M * sizeof(double);
    const size_t lds_fwd = (size_t)M * (sizeof(uint64_t) + 2 * sizeof(double));
    if (allow_lds((const void*)large_seg_agg, lds_agg) != HAWKES_OK ||
        allow_lds((const void*)large_forward<true, false, false, HK_FWW, true>, lds_fwd) != HAWKES_OK ||
        allow_lds((const void*)large_forward<false, false, false, HK_FWW, true>, lds_fwd) != HAWKES_OK)
        return HAWKES_EUNSUPPORTED;
    if (A.grad && (uint64_t)A.nslot * (uint64_t)HK_SLOT_WORDS(A.CPL, A.NGW) * 8u >= (1ull << 32))
        return HAWKES_EUNSUPPORTED;
    if (A.grad && dense_allow_lds(A) != HAWKES_OK) return HAWKES_EUNSUPPORTED;
    const int32_t W = 2 + 2 * K;
    hipLaunchKernelGGL(fill_d, dim3(16), dim3(256), 0, st, A.carry, (int64_t)K * 2 * M, 0.0);
    hipLaunchKernelGGL(fill_d, dim3(1), dim3(64), 0, st, A.acc, (int64_t)W, 0.0);
    if (A.grad) {
        const int64_t ng = (int64_t)K * A.ER * MM;
        hipLaunchKernelGGL(fill_d, dim3((unsigned)((ng + 255) / 256 < 65535 ? (ng + 255) / 256 : 65535)),
                           dim3(256), 0, st, A.gpart, ng, 0.0);
        hipLaunchKernelGGL(fill_d, dim3(64), dim3(256), 0, st, A.spart, (int64_t)K * A.NRUN * M, 0.0);
        hipLaunchKernelGGL(fill_d, dim3(64), dim3(256), 0, st, A.cpart_, (int64_t)K * A.NRUN * M, 0.0);
    }
    // per kernel: column sums, CSR copy and node records of alpha^k
    for (int32_t k = 0; k < K; ++k) {
        const float* ak = A.alpha + (int64_t)k * MM;
        int32_t* pk = A.csr_ptr + (int64_t)k * (M + 1);
        hipLaunchKernelGGL(large_colsum, dim3((unsigned)((M + 63) / 64)), dim3(1024), 0, st, M, ak,
                           A.colsum + (int64_t)k * M);
        large_build_index(M, ak, 0, pk, A.csr_cv + k * cv_stride(MM), st);
        hipLaunchKernelGGL(large_node_info, dim3(gM), dim3(256), 0, st, M, pk, A.mu, A.colsum + (int64_t)k * M,
                           A.node_info + (int64_t)k * M);
    }
    // kernel k's view of the per-kernel arrays
    auto view = [&](int32_t k) {
        LargeArgs B = A;
        B.K = 1;
        B.beta = A.beta + k;
        B.carry = A.carry + (int64_t)k * 2 * M;
        B.carry_seg = A.carry_seg + (int64_t)k * A.nseg * 2 * M;
        B.gpart = A.gpart ? A.gpart + (int64_t)k * A.ER * MM : nullptr;
        B.spart = A.spart ? A.spart + (int64_t)k * A.NRUN * M : nullptr;
        B.cpart_ = A.cpart_ ? A.cpart_ + (int64_t)k * A.NRUN * M : nullptr;
        return B;
    };
    for (int64_t ch = 0; ch < A.nchunks; ++ch) {
        const int64_t c0 = ch * A.CH;
        const int64_t c1 = c0 + A.CH < A.n ? c0 + A.CH : A.n;
        const int32_t nseg = (int32_t)((c1 - c0 + HK_SEG - 1) / HK_SEG);
        for (int32_t k = 0; k < K; ++k) {
            LargeArgs B = view(k);
            // the lazy records' times go to the segment maps' buffer, which
            // the scan has consumed by then
            FwdExtra Xm{};
            Xm.rtau = B.agg;
            {
                TimedScope ts(2, st);
                hipLaunchKernelGGL(large_seg_agg, dim3(nseg), dim3(64), lds_agg, st, c0, c1, M, A.t, A.marks,
                                   B.beta, B.agg, B.seg_span, B.seg_dec);
            }
            {
                TimedScope ts(3, st);
                large_scan(B, nseg, nullptr, st);
            }
            TimedScope ts(1, st);
            if (A.grad)
                hipLaunchKernelGGL((large_forward<true, false, false, HK_FWW, true>), dim3(nseg), dim3(64 * HK_FWW),
                                   lds_fwd, st, c0, c1, M, A.T, A.t, A.marks, A.mu, B.beta,
                                   A.node_info + (int64_t)k * M, A.csr_cv + k * cv_stride(MM), B.carry_seg,
                                   A.seg_part, A.wchunk, (float*)nullptr, (double*)nullptr, 0,
                                   A.rk + (int64_t)k * A.CH, A.dk + (int64_t)k * A.CH, Xm);
            else
                hipLaunchKernelGGL((large_forward<false, false, false, HK_FWW, true>), dim3(nseg), dim3(64 * HK_FWW),
                                   lds_fwd, st, c0, c1, M, A.T, A.t, A.marks, A.mu, B.beta,
                                   A.node_info + (int64_t)k * M, A.csr_cv + k * cv_stride(MM), B.carry_seg,
                                   A.seg_part, A.wchunk, (float*)nullptr, (double*)nullptr, 0,
                                   A.rk + (int64_t)k * A.CH, (double*)nullptr, Xm);
        }
        {
            TimedScope ts(1, st);
            if (A.grad)
                hipLaunchKernelGGL((large_combine<true, false>), dim3(nseg), dim3(256), 0, st, c0, c1, M, K, A.T, A.t,
                                   A.marks, A.mu, A.beta, A.colsum, A.rk, A.dk, A.CH, A.seg_part, A.wchunk,
                                   (float*)nullptr);
            else if (A.lambda_out)
                hipLaunchKernelGGL((large_combine<false, true>), dim3(nseg), dim3(256), 0, st, c0, c1, M, K, A.T, A.t,
                                   A.marks, A.mu, A.beta, A.colsum, A.rk, A.dk, A.CH, A.seg_part, A.wchunk,
                                   A.lambda_out);
            else
                hipLaunchKernelGGL((large_combine<false, false>), dim3(nseg), dim3(256), 0, st, c0, c1, M, K, A.T,
                                   A.t, A.marks, A.mu, A.beta, A.colsum, A.rk, A.dk, A.CH, A.seg_part, A.wchunk,
                                   (float*)nullptr);
        }
        hipLaunchKernelGGL(large_chunk_acc, dim3(1), dim3(256), 0, st, nseg, W, A.seg_part, A.acc);
        if (A.grad) {
            {
                TimedScope tb(6, st);
                bucket_chunk_into(A, c0, c1, nseg, A.wchunk, A.DRB, A.bo_cnt, A.bo_off, A.bo_base, A.bo_key, A.bo_t,
                                  A.bo_w, st, false);
            }
            for (int32_t k = 0; k < K; ++k) {
                LargeArgs B = view(k);
                large_dense_launch(B, c0, c1, nseg, st, false);
            }
        }
    }
    const int64_t nfin = A.grad ? (MM > M ? MM : M) : 1;
    for (int32_t k = 0; k < K; ++k) {
        LargeArgs B = view(k);
        if (A.grad) hipLaunchKernelGGL(large_colfold, dim3(gM), dim3(256), 0, st, M, A.NRUN, B.spart, B.cpart_);
        hipLaunchKernelGGL(large_final, dim3((unsigned)((nfin + 255) / 256)), dim3(256), 0, st, M, A.ER, 1, A.T,
                           A.mu, A.acc, B.gpart, B.spart, B.cpart_, A.loglik, A.g_mu,
                           A.g_alpha ? A.g_alpha + k * MM : nullptr, A.g_beta, A.grad ? 1 : 0, 0, K, k);
        if (!A.grad) break;   // the log-likelihood needs one launch
    }
    return hipGetLastError() == hipSuccess ? HAWKES_OK : HAWKES_EDEVICE;
}

hawkes_status run_large(LargeArgs& A, hipStream_t st) {
    if (A.per_target) return run_large_pt(A, st);
    if (A.K > 1) return run_large_multi(A, st);
    const int32_t M = A.M;
    const int64_t MM = (int64_t)M * M;
    const unsigned gM = (unsigned)((M + 255) / 256);
    const size_t lds_agg = (size_t)2 * M * sizeof(double);
    const size_t lds_fwd = (size_t)M * (sizeof(uint64_t) + 2 * sizeof(double));
    if (allow_lds((const void*)large_seg_agg, lds_agg) != HAWKES_OK ||
        allow_lds((const void*)large_forward<true, false, false, HK_FWW>, lds_fwd) != HAWKES_OK ||
        allow_lds((const void*)large_forward<true, false, true, 1>, lds_fwd) != HAWKES_OK ||
        allow_lds((const void*)large_forward<false, true, false, HK_FWW>, lds_fwd) != HAWKES_OK ||
        allow_lds((const void*)large_forward<false, false, false, HK_FWW>, lds_fwd) != HAWKES_OK)
        return HAWKES_EUNSUPPORTED;
    if (A.grad && !A.support && dense_allow_lds(A) != HAWKES_OK) return HAWKES_EUNSUPPORTED;
    const bool sup = A.grad && A.support;
    // support-restricted: the first term's copies (CSR order) take the place
    // of the dense partials, min(8, ER) of them (ER is a power of two)
    const int32_t ncopy = A.ER < 8 ? A.ER : 8;
    if (sup) A.gsup = A.gpart;
    // the dense-gradient kernels address checkpoints and records with
    // 32-bit byte offsets
    if (A.grad && (uint64_t)A.nslot * (uint64_t)HK_SLOT_WORDS(A.CPL, A.NGW) * 8u >= (1ull << 32))
        return HAWKES_EUNSUPPORTED;
    // zero the carried state and accumulators
    hipLaunchKernelGGL(fill_d, dim3(1), dim3(256), 0, st, A.carry, (int64_t)2 * M, 0.0);
    hipLaunchKernelGGL(fill_d, dim3(1), dim3(64), 0, st, A.acc, (int64_t)4, 0.0);
    // per-segment-slot sums of the forward pass, accumulated over the chunks
    // (one reduction after the last chunk instead of one launch per chunk)
    hipLaunchKernelGGL(fill_d, dim3(4), dim3(256), 0, st, A.seg_part, (int64_t)A.nseg * 4, 0.0);
    // the forward pass adds the scan's group carries itself (the scan's
    // apply pass is left out) and counts the partition (by blocks of 2^DRB
    // nodes, when the gradient needs them and they fit its LDS).  Measured
    // at c4: 6.483 -> 6.439 ms per step; also summing the chunk in the
    // forward pass's last workgroup instead of large_chunk_acc cost 0.17 ms.
    FwdExtra X;
    X.rtau = A.agg;   // free once the scan has run
    X.gcarry = A.gcarry;
    X.seg_off = A.seg_off;
    X.seg_offdec = A.seg_offdec;
    X.bs = A.DRB;
    X.nbo = A.NBO;
    X.bcnt = nullptr;
    size_t lds_fwdc = lds_fwd;   // the gradient's forward pass, with the partition counts if they fit
    if (A.grad && A.NBO <= HK_NBO_MAX) {
        const void* kf = sup ? (const void*)large_forward<true, false, true, 1>
                             : (const void*)large_forward<true, false, false, HK_FWW>;
        if (allow_lds(kf, lds_fwd + (size_t)A.NBO * sizeof(int32_t)) == HAWKES_OK) {
            X.bcnt = A.bo_cnt;
            lds_fwdc = lds_fwd + (size_t)A.NBO * sizeof(int32_t);
        }
    }
    A.carry_prefix = true;
    if (A.grad) {
        // the dense partials, or (support-restricted) the CSR-ordered sums
        const int64_t ng = (sup ? ncopy : A.ER) * MM;
        hipLaunchKernelGGL(fill_d, dim3((unsigned)((ng + 255) / 256 < 65535 ? (ng + 255) / 256 : 65535)),
                           dim3(256), 0, st, sup ? A.gsup : A.gpart, ng, 0.0);
        hipLaunchKernelGGL(fill_d, dim3(64), dim3(256), 0, st, A.spart, (int64_t)A.NRUN * M, 0.0);
        hipLaunchKernelGGL(fill_d, dim3(64), dim3(256), 0, st, A.cpart_, (int64_t)A.NRUN * M, 0.0);
    }
    hipLaunchKernelGGL(large_colsum, dim3((unsigned)((M + 63) / 64)), dim3(1024), 0, st, M, A.alpha, A.colsum);
    large_build_index(M, A.alpha, 0, A.csr_ptr, A.csr_cv, st);
    hipLaunchKernelGGL(large_node_info, dim3(gM), dim3(256), 0, st, M, A.csr_ptr, A.mu, A.colsum, A.node_info);
    for (int64_t ch = 0; ch < A.nchunks; ++ch) {
        const int64_t c0 = ch * A.CH;
        const int64_t c1 = c0 + A.CH < A.n ? c0 + A.CH : A.n;
        const int32_t nseg = (int32_t)((c1 - c0 + HK_SEG - 1) / HK_SEG);
        {
            TimedScope ts(2, st);
            hipLaunchKernelGGL(large_seg_agg, dim3(nseg), dim3(64), lds_agg, st, c0, c1, M, A.t, A.marks, A.beta,
                               A.agg, A.seg_span, A.seg_dec);
        }
        {
            TimedScope ts(3, st);
            large_scan(A, nseg, nullptr, st, false);
        }
        {
            TimedScope ts(1, st);
            if (sup)
                hipLaunchKernelGGL((large_forward<true, false, true, 1>), dim3(nseg), dim3(64), lds_fwdc, st, c0, c1,
                                   M, A.T, A.t, A.marks, A.mu, A.beta, A.node_info, A.csr_cv,
                                   A.carry_seg, A.seg_part, A.wchunk, (float*)nullptr, A.gsup, ncopy - 1,
                                   (double*)nullptr, (double*)nullptr, X);
            else if (A.grad)
                hipLaunchKernelGGL((large_forward<true, false, false, HK_FWW>), dim3(nseg), dim3(64 * HK_FWW), lds_fwdc,
                                   st, c0, c1,
                                   M, A.T, A.t, A.marks, A.mu, A.beta, A.node_info, A.csr_cv,
                                   A.carry_seg, A.seg_part, A.wchunk, (float*)nullptr, (double*)nullptr, 0,
                                   (double*)nullptr, (double*)nullptr, X);
            else if (A.lambda_out)
                hipLaunchKernelGGL((large_forward<false, true, false, HK_FWW>), dim3(nseg), dim3(64 * HK_FWW), lds_fwd,
                                   st, c0, c1,
                                   M, A.T, A.t, A.marks, A.mu, A.beta, A.node_info, A.csr_cv,
                                   A.carry_seg, A.seg_part, A.wchunk, A.lambda_out, (double*)nullptr, 0,
                                   (double*)nullptr, (double*)nullptr, X);
            else
                hipLaunchKernelGGL((large_forward<false, false, false, HK_FWW>), dim3(nseg), dim3(64 * HK_FWW), lds_fwd,
                                   st, c0, c1,
                                   M, A.T, A.t, A.marks, A.mu, A.beta, A.node_info, A.csr_cv,
                                   A.carry_seg, A.seg_part, A.wchunk, (float*)nullptr, (double*)nullptr, 0,
                                   (double*)nullptr, (double*)nullptr, X);
        }
        if (A.grad) {
            {
                TimedScope tb(6, st);
                bucket_chunk_into(A, c0, c1, nseg, A.wchunk, A.DRB, A.bo_cnt, A.bo_off, A.bo_base, A.bo_key, A.bo_t,
                                  A.bo_w, st, X.bcnt != nullptr);
            }
            // support-restricted: only the checkpoint kernel's per-column
            // sums (dL/dmu, compensator) are needed
            large_dense_launch(A, c0, c1, nseg, st, sup);
        }
    }
    hipLaunchKernelGGL(large_chunk_acc, dim3(1), dim3(256), 0, st, A.nseg, 4, A.seg_part, A.acc);
    const int64_t nfin = A.grad ? (MM > M ? MM : M) : 1;
    if (A.grad) hipLaunchKernelGGL(large_colfold, dim3(gM), dim3(256), 0, st, M, A.NRUN, A.spart, A.cpart_);
    hipLaunchKernelGGL(large_final, dim3((unsigned)((nfin + 255) / 256)), dim3(256), 0, st, M, A.ER, 1, A.T, A.mu,
                       A.acc, A.gpart, A.spart, A.cpart_, A.loglik, A.g_mu, A.g_alpha, A.g_beta, A.grad ? 1 : 0,
                       sup ? 1 : 0, 1, 0);
    if (sup && A.g_alpha)
        hipLaunchKernelGGL(large_sup_scatter, dim3((unsigned)M), dim3(64), 0, st, M, ncopy, A.csr_ptr, A.csr_cv,
                           A.gsup, A.cpart_, A.g_alpha);
    return hipGetLastError() == hipSuccess ? HAWKES_OK : HAWKES_EDEVICE;
}

}  // namespace hk
