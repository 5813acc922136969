// Dense dL/dalpha of the shared-decay large-M path (eq. 9): sum over events
// of beta w_i K(t_i) into row m_i, from the bucketed event streams.
#include "hk_device.h"
#include "hk_large.h"
#include "hk_stream.h"

namespace hk {

// ------------------------------------------------------------------ dense dL/dalpha
// Block = (row block of HK_DR rows, column block of W = 64 CPL columns, event
// range er), one wave.  LDS G[HK_DR][W] float64 accumulates
// sum_i beta w_i K_q(t_i) for the block's rows p (targets m_i) and columns q
// (sources); lane c owns columns s0 + c + 64 j (j < CPL) and their state K
// (float64), kept in the frame of an anchor time.  Events are bucketed by
// node blocks of W nodes; the block reads only two bucket streams: the node
// block holding its rows (the events in its rows are the "own" events) and
// its column block ("slab" events), merged by event index in windows of up to
// 64 + 64 records:
//   - the window ends where either list's 64th record ends (hi), so every own
//     event of the window sees all earlier slab events either in K or in the
//     window;
//   - K moves to the window's first event time tw; own event k adds c_k * K to
//     row m_k (c_k = beta w_k e^{-beta (t_k - tw)}, CPL ds_add_f64 over the
//     W columns) plus c_k * b_j at (m_k, m_j) for the window's slab events j
//     before it (b_j = e^{beta (t_j - tw)}, one masked ds_add_f64 over those
//     lanes): together c_k times K just before event k;
//   - then the slab events enter K in one vector step (scatter-add into LDS by
//     column, read back by each column's lane), and row block 0 sums w and the
//     compensator terms 1 - e^{-beta (T - t_j)} per column the same way.
// A window whose time span exceeds HK_WIDE / beta (anchored factors would
// leave float32 range) is walked event by event with per-event decays.
// Blocks of one event range are placed on one XCD (blockIdx % 8).  With
// HK_DR = 16 rows and W = 128 a block uses 19 KiB of LDS.
template <int CPL>
__global__ __launch_bounds__(64) void large_dense(int64_t c0, int64_t c1, int32_t M, int32_t NBC, int32_t NBR,
                                                  int32_t ER, int32_t segs_per_range, int32_t nseg, double T,
                                                  const double* __restrict__ t, const float* __restrict__ beta,
                                                  const double* __restrict__ carry_seg,
                                                  const int32_t* __restrict__ bk_off,
                                                  const int32_t* __restrict__ bk_base,
                                                  const uint32_t* __restrict__ bk_key, const double* __restrict__ bk_t,
                                                  const float* __restrict__ bk_w, double* __restrict__ gpart,
                                                  double* __restrict__ spart, double* __restrict__ cpart) {
    constexpr int W = 64 * CPL;
    __shared__ double G[HK_DR * W];
    __shared__ double KhL[W], SL[W], CL[W];
    const int lane = threadIdx.x;
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        KhL[j * 64 + lane] = 0.0;
        SL[j * 64 + lane] = 0.0;
        CL[j * 64 + lane] = 0.0;
    }
    const int32_t blk = blockIdx.x;
    const int32_t nbb = NBR * NBC;
    int32_t er, local;
    if (ER >= 8) {
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
    const int32_t sb = local % NBC;
    const int32_t rb = local / NBC;
    const int32_t r0 = rb * HK_DR, s0 = sb * W;
    // own events: the node block holding rows [r0, r0 + HK_DR), part `hf` of it
    const int32_t ob = r0 / W;
    const uint32_t hf = (uint32_t)((r0 % W) / HK_DR);
    const int32_t sA = er * segs_per_range;
    if (sA >= nseg) return;
    const int32_t sB = sA + segs_per_range < nseg ? sA + segs_per_range : nseg;
    const int64_t a = c0 + (int64_t)sA * HK_SEG;
    double* gp = gpart + (int64_t)er * M * M;
    {
        // branch-free block load (all loads in flight together); out-of-range
        // rows/columns read a clamped valid address and are zeroed
#pragma unroll
        for (int j = 0; j < CPL; ++j) {
            const int32_t col = s0 + j * 64 + lane;
            const int32_t cc = col < M ? col : M - 1;
            for (int rg = 0; rg < HK_DR; rg += 16) {
                double v[16];
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int32_t row = r0 + rg + i;
                    const int32_t rr = row < M ? row : M - 1;
                    v[i] = gp[(int64_t)rr * M + cc];
                }
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int32_t row = r0 + rg + i;
                    G[(rg + i) * W + j * 64 + lane] = (row < M && col < M) ? v[i] : 0.0;
                }
            }
        }
    }
    const double bet = (double)beta[0];
    // K at the range start (just after the event before it)
    double Kh[CPL];
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const int32_t col = s0 + j * 64 + lane;
        Kh[j] = col < M ? carry_seg[(int64_t)sA * 2 * M + col] : 0.0;
    }
    double tau = a > 0 ? t[a - 1] : t[a];
    double Sacc[CPL], Cacc[CPL];
#pragma unroll
    for (int j = 0; j < CPL; ++j) Sacc[j] = Cacc[j] = 0.0;
    const bool diag_owner = rb == 0;
    RecStream<false> O, S;
    O.init(bk_key, bk_t, bk_w, (int64_t)bk_base[ob] + bk_off[(int64_t)ob * (nseg + 1) + sA],
           (int64_t)bk_base[ob] + bk_off[(int64_t)ob * (nseg + 1) + sB]);
    S.init(bk_key, bk_t, bk_w, (int64_t)bk_base[sb] + bk_off[(int64_t)sb * (nseg + 1) + sA],
           (int64_t)bk_base[sb] + bk_off[(int64_t)sb * (nseg + 1) + sB]);
    constexpr int SH = CPL == 2 ? 7 : 6;   // bits of the local mark in a record key
    __syncthreads();
    for (;;) {
        const int64_t ao = O.avail(), as = S.avail();
        if (ao <= 0 && as <= 0) break;
        const int io = (int)(O.ck >> SH), is = (int)(S.ck >> SH);
        const int lim_o = ao > 64 ? rl_i(io, 63) : 0x7fffffff;
        const int lim_s = as > 64 ? rl_i(is, 63) : 0x7fffffff;
        const int hi = lim_o < lim_s ? lim_o : lim_s;
        const bool inw = lane < ao && io <= hi;   // record of the window (any part of the block)
        const bool own = inw && ((O.ck & (uint32_t)(W - 1)) / HK_DR) == hf;
        const bool sl = lane < as && is <= hi;
        const uint64_t om = __ballot(own);
        const int nw = __builtin_popcountll(__ballot(inw));
        const int ns = __builtin_popcountll(__ballot(sl));
        double tw = 1e300, te = -1e300;
        if (nw) { tw = rl_d(O.ct, 0); te = rl_d(O.ct, nw - 1); }
        if (ns) {
            const double a0 = rl_d(S.ct, 0), a1 = rl_d(S.ct, ns - 1);
            tw = a0 < tw ? a0 : tw;
            te = a1 > te ? a1 : te;
        }
        {
            const double f = (double)exp_f64arg(-bet * (tw - tau));
#pragma unroll
            for (int j = 0; j < CPL; ++j) Kh[j] *= f;
        }
        tau = tw;
        const int colj = (int)(S.ck & (uint32_t)(W - 1));
        if (bet * (te - tw) <= HK_WIDE) {
            const float cf = own ? (float)(bet * (double)O.cw) * exp_f64arg(-bet * (O.ct - tw)) : 0.0f;
            const double bj = sl ? (double)exp_f64arg(bet * (S.ct - tw)) : 0.0;
            // own events two at a time: two independent update chains
            const int rowl = (int)(O.ck & (HK_DR - 1));
            uint64_t mo = om;
            while (mo) {
                const int k1 = __builtin_ctzll(mo);
                mo &= mo - 1;
                const int r1 = rl_i(rowl, k1) * W, i1 = rl_i(io, k1);
                const double c1 = (double)rl_f(cf, k1);
                if (mo) {
                    const int k2 = __builtin_ctzll(mo);
                    mo &= mo - 1;
                    const int r2 = rl_i(rowl, k2) * W, i2 = rl_i(io, k2);
                    const double c2 = (double)rl_f(cf, k2);
#pragma unroll
                    for (int j = 0; j < CPL; ++j) {
                        atomicAdd(&G[r1 + j * 64 + lane], c1 * Kh[j]);
                        atomicAdd(&G[r2 + j * 64 + lane], c2 * Kh[j]);
                    }
                    if (sl && is < i1) atomicAdd(&G[r1 + colj], c1 * bj);
                    if (sl && is < i2) atomicAdd(&G[r2 + colj], c2 * bj);
                } else {
#pragma unroll
                    for (int j = 0; j < CPL; ++j) atomicAdd(&G[r1 + j * 64 + lane], c1 * Kh[j]);
                    if (sl && is < i1) atomicAdd(&G[r1 + colj], c1 * bj);
                }
            }
            if (ns) {
                if (sl) {
                    atomicAdd(&KhL[colj], bj);
                    if (diag_owner) {
                        atomicAdd(&SL[colj], (double)S.cw);
                        atomicAdd(&CL[colj], -expm1(-bet * (T - S.ct)));
                    }
                }
                __syncthreads();
#pragma unroll
                for (int j = 0; j < CPL; ++j) {
                    Kh[j] += KhL[j * 64 + lane];
                    KhL[j * 64 + lane] = 0.0;
                }
            }
        } else {
            int ko = 0, ks = 0;
            while (ko < nw || ks < ns) {
                const int iko = ko < nw ? rl_i(io, ko) : 0x7fffffff;
                const int iks = ks < ns ? rl_i(is, ks) : 0x7fffffff;
                if (iko <= iks) {
                    // own first on a tie: the same event as slab event comes after
                    const double tk = rl_d(O.ct, ko);
                    const double f = (double)exp_f64arg(-bet * (tk - tau));
#pragma unroll
                    for (int j = 0; j < CPL; ++j) Kh[j] *= f;
                    tau = tk;
                    if ((om >> ko) & 1ull) {
                        const int r = (int)(rl_i((int)O.ck, ko) & (HK_DR - 1));
                        const double cw = bet * (double)rl_f(O.cw, ko);
#pragma unroll
                        for (int j = 0; j < CPL; ++j) atomicAdd(&G[r * W + j * 64 + lane], cw * Kh[j]);
                    }
                    ++ko;
                } else {
                    const double tk = rl_d(S.ct, ks);
                    const double f = (double)exp_f64arg(-bet * (tk - tau));
#pragma unroll
                    for (int j = 0; j < CPL; ++j) Kh[j] *= f;
                    tau = tk;
                    const int ck = (int)(rl_i((int)S.ck, ks) & (W - 1));
#pragma unroll
                    for (int j = 0; j < CPL; ++j) {
                        if (j * 64 + lane == ck) {
                            Kh[j] += 1.0;
                            if (diag_owner) {
                                Sacc[j] += (double)rl_f(S.cw, ks);
                                Cacc[j] += -expm1(-bet * (T - tk));
                            }
                        }
                    }
                    ++ks;
                }
            }
        }
        O.consume(nw);
        S.consume(ns);
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < CPL; ++j) {
        const int32_t col = s0 + j * 64 + lane;
        if (col < M) {
#pragma unroll
            for (int r = 0; r < HK_DR; ++r) {
                const int32_t row = r0 + r;
                if (row < M) gp[(int64_t)row * M + col] = G[r * W + j * 64 + lane];
            }
            if (diag_owner) {
                spart[(int64_t)er * M + col] += Sacc[j] + SL[j * 64 + lane];
                cpart[(int64_t)er * M + col] += Cacc[j] + CL[j * 64 + lane];
            }
        }
    }
}

void large_dense_launch(LargeArgs& A, int64_t c0, int64_t c1, int32_t nseg, hipStream_t st) {
    const int32_t spr = (nseg + A.ER - 1) / A.ER;
    const int32_t nbb = A.NBR * A.NBC;
    const unsigned nblk = A.ER >= 8 ? (unsigned)(nbb * ((A.ER + 7) / 8) * 8)
                                    : (unsigned)(((nbb + 8 / A.ER - 1) / (8 / A.ER)) * 8);
    if (A.CPL == 2)
        hipLaunchKernelGGL(large_dense<2>, dim3(nblk), dim3(64), 0, st, c0, c1, A.M, A.NBC, A.NBR, A.ER, spr, nseg,
                           A.T, A.t, A.beta, A.carry_seg, A.bk_off, A.bk_base, A.bk_key, A.bk_t, A.bk_w, A.gpart,
                           A.spart, A.cpart_);
    else
        hipLaunchKernelGGL(large_dense<1>, dim3(nblk), dim3(64), 0, st, c0, c1, A.M, A.NBC, A.NBR, A.ER, spr, nseg,
                           A.T, A.t, A.beta, A.carry_seg, A.bk_off, A.bk_base, A.bk_key, A.bk_t, A.bk_w, A.gpart,
                           A.spart, A.cpart_);
}

}  // namespace hk
