// Large-M engine with one decay per target node (beta[M], one kernel).
//
// With beta_p depending on the target, the intensity state is target-indexed
// (R-form): R_p(t) = sum_{j: t_j < t} alpha_{p,m_j} e^{-beta_p (t - t_j)}, so
// lambda_p(t) = mu_p + beta_p R_p(t) (eq. 1 with gamma -> beta_p).  Its
// transition map is affine with a diagonal decay diag(e^{-beta_p dt}) instead
// of a scalar one (eq. 6 with a per-component decay); segment maps compose in
// closed form per component, so the segmented scan of the shared-decay path
// carries over with exp(-beta_p span) per (segment, p).
//
// Gradient (eqs. 8-10 with beta_p):
//   dL/dmu_p    = S_p - T,                S_p = sum_{i: m_i = p} w_i, w_i = 1/lambda_i
//   dL/dbeta_p  = sum_{i: m_i = p} w_i (R_p(t_i) - beta_p D_p(t_i))
//                 - sum_j alpha_{p,m_j} (T - t_j) e^{-beta_p (T - t_j)},
//                 D_p(t) = sum_j alpha_{p,m_j} (t - t_j) e^{-beta_p (t - t_j)}
//   dL/dalpha_pq = sum_{j: m_j = q} beta_p A_p(t_j) - N_q
// where A_p(t) = sum_{i > j, m_i = p} w_i e^{-beta_p (t_i - t)} + e^{-beta_p (T - t)} / beta_p
// is the reverse (adjoint) state: the second term, a seed 1/beta_p at T,
// folds the compensator's alpha-derivative sum_j (1 - e^{-beta_p (T - t_j)})
// into the sum, and N_q is the number of q-events.  The dense alpha-gradient
// is then a column update per source event, with target-indexed state in the
// lanes, so each lane keeps its own decay.
//
// Pass 1 (chunks in order): R-form segment maps, their scan, the forward pass
// (log-likelihood, w_i per event, per-target sums for dL/dbeta), compensator
// terms.  Decays in this pass use float64 exp: dL/dbeta_p is a difference of
// near-equal sums, and with float32 decays its error reached 2e-6 on a small
// dense-alpha case.
// Pass 2 (chunks in reverse): reverse segment maps of A, their scan from the
// right (seeded at T), and the dense adjoint kernel.
#include "hk_device.h"
#include "hk_large.h"
#include "hk_stream.h"

namespace hk {

// capacity of the per-batch staging of alpha columns in the forward kernel
// (16 bytes an entry); the forward kernel's batch area (event times, shares,
// events per own target) takes PT_BATCH_LDS, its table of own targets one
// byte per node; PT_U column entries a lane per pass of its pushes
#define PT_STAGE 1136
#define PT_BATCH_LDS (64 * 4 * 8)
#define PT_U 4
// column entries a lane per pass in the segment aggregation and the chunk chain
// (measured at c5: 2 against 4 took their time from 3.66 to 3.27 ms per call)
#define PT_UA 2
// capacity of the segment aggregation's stage (16 bytes an entry)
#define PT_STAGE_AGG 2048
// events per workgroup of the chunk chain (512 workgroups for 2^20 events;
// measured at c5 against 1024 and 4096), and its stage (two workgroups a CU
// at M = 4096)
#define PT_CHAIN_EV 2048
#define PT_STAGE_CHAIN 960
// waves per workgroup of the dense kernel: eight share the 64 x 64 LDS tile,
// three workgroups a CU (measured at c5: 3.36 ms per launch against 4.01 with
// four waves, 4.19 with seven, 4.49 with nine)
#ifndef HK_DWP
#define HK_DWP 8
#endif
// largest beta_max (t_first - t_last) of a dense-kernel window that takes the
// merged path: e^64 and e^-64 stay well inside float32's range
#define HK_PT_MERGE_SPAN 64.0

// Inclusive prefix sum over the 64 lanes of a wave on the vector ALU (DPP):
// shifts within rows of 16 lanes (row_shr 1, 2, 4, 8), then each row's total
// carried forward (row_bcast 15 into rows 1 and 3, row_bcast 31 into rows 2
// and 3).  A lane that a shift or broadcast does not reach adds 0.  Every
// lane of the wave must be active.
__device__ __forceinline__ int32_t wave_incl_scan_dpp(int32_t v) {
    v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xF, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xA, 0xF, false);
    v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xC, 0xF, false);
    return v;
}

__global__ void pt_fill(double* p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// dst[i] = src[i] (a chunk-start state into or out of a checkpoint slot)
__global__ void pt_copy(double* __restrict__ dst, const double* __restrict__ src, int64_t n) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

// csc_b[k] = beta of the target of column entry k (the decay that entry's
// push uses, so a pass reads it with the entry instead of a second gather)
__global__ void pt_csc_beta(int32_t M, const int32_t* __restrict__ csc_ptr, const int2* __restrict__ csc_cv,
                            const float* __restrict__ beta, float* __restrict__ csc_b) {
    const int32_t nnz = csc_ptr[M];
    for (int32_t k = blockIdx.x * blockDim.x + threadIdx.x; k < nnz; k += gridDim.x * blockDim.x)
        csc_b[k] = beta[csc_cv[k].x];
}

// adjoint seed at T: A_p(T) = 1 / beta_p
__global__ void pt_seed(int32_t M, const float* __restrict__ beta, double* __restrict__ a) {
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < M) a[p] = 1.0 / (double)beta[p];
}

__device__ __forceinline__ int pt_rdl(int v, int k) { return __builtin_amdgcn_readlane(v, k); }
__device__ __forceinline__ double pt_rdl_d(double v, int k) {
    const int64_t b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((int64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// ------------------------------------------------------------------ pass 1
// Segment map in R-form: R and D just after the segment's last event, from the
// segment's own events.  Also the two compensator sums of the segment:
// sum_j sum_p alpha_{p,m_j} (1 - e^{-beta_p (T - t_j)}) into seg_part[s][1]
// and, per target, sum_j alpha_{p,m_j} (T - t_j) e^{-beta_p (T - t_j)}.
// One wave per segment.  The terms are plain sums, so the alpha-column entries
// of 64 events at a time are staged in LDS and taken PT_UA a lane per pass
// (lanes over entries, not events: a column averages a few entries).  An
// entry's compensator terms need e^{-beta_p (T - t_j)}, zero in float64 past
// an exponent of 745: then the entry adds its alpha to the sum and nothing
// to the per-target one, with no exponential (every entry of a segment far
// from T).  LDS: aR[M], aD[M], aE[M] (float64), the batch's event times and
// the stage.
// FAR: the variant for a chunk in which every entry's e^{-beta_p (T - t_j)}
// is zero (beta_min (T - t_last) > 745, decided on the device into *near):
// no per-target compensator array, so two workgroups share a CU at M = 4096;
// of the two variants launched for a chunk, the one that does not apply
// returns at once.
template <bool FAR, int STG>
__global__ __launch_bounds__(64) void pt_seg_agg(int64_t c0, int64_t c1, int32_t M, double T,
                                                 const double* __restrict__ t, const int32_t* __restrict__ marks,
                                                 const float* __restrict__ beta, const int32_t* __restrict__ csc_ptr,
                                                 const int2* __restrict__ csc_cv, const float* __restrict__ csc_b,
                                                 double* __restrict__ agg, double* __restrict__ seg_span,
                                                 double* __restrict__ ebseg, double* __restrict__ seg_part,
                                                 const int32_t* __restrict__ near) {
    if ((*near != 0) == FAR) return;   // the other variant takes this chunk
    extern __shared__ double lds[];
    double* aR = lds;
    double* aD = lds + M;
    double* aE = lds + 2 * M;                  // (unused when FAR)
    double* ev_t = lds + (FAR ? 2 : 3) * M;    // [64]
    int4* stg = (int4*)(ev_t + 64);            // [STG] (target, alpha, event, beta)
    const int32_t s = blockIdx.x;
    const int64_t a = c0 + (int64_t)s * HK_SEG;
    const int64_t b = a + HK_SEG < c1 ? a + HK_SEG : c1;
    const int lane = threadIdx.x;
    for (int32_t q = lane; q < M; q += 64) {
        aR[q] = 0.0;
        aD[q] = 0.0;
        if (!FAR) aE[q] = 0.0;
    }
    const double te = t[b - 1];
    double comp = 0.0;
    // the next batch's events and column extents are loaded one batch ahead
    double tv_n;
    int32_t cb_n, ce_n;
    {
        const int64_t ic = a + lane < b ? a + lane : b - 1;
        tv_n = t[ic];
        const int q = clamp_mark(marks[ic], M);
        cb_n = csc_ptr[q];
        ce_n = csc_ptr[q + 1];
    }
    for (int64_t base = a; base < b; base += 64) {
        const int64_t i = base + lane;
        const bool ve = i < b;
        const double tv = tv_n;
        const int32_t cb = cb_n;
        const int32_t cn = ve ? ce_n - cb : 0;
        int mraw_n;
        {
            const int64_t i2 = base + 64 + lane;
            const int64_t ic2 = i2 < b ? i2 : b - 1;
            tv_n = t[ic2];
            mraw_n = marks[ic2];
        }
        const int32_t off = wave_incl_scan_dpp(cn) - cn;   // exclusive
        const int32_t cend = off + cn;
        const int nb = (int)(b - base < 64 ? b - base : 64);
        __syncthreads();   // the previous batch is done with ev_t and the stage
        ev_t[lane] = tv;
        int k = 0;
        while (k < nb) {
            const int32_t o0 = pt_rdl(off, k);
            const int nfit = __builtin_popcountll(
                __builtin_amdgcn_ballot_w64(lane >= k && lane < nb && cend - o0 <= STG));
            const bool staged = nfit > 0;
            const int k2 = staged ? k + nfit : k + 1;
            const int32_t ne = pt_rdl(cend, k2 - 1) - o0;
            const int32_t cbk = pt_rdl(cb, k);
            if (staged) {
                const bool mine = lane >= k && lane < k2;
                if (mine && cn <= 32) {
                    for (int32_t j0 = 0; j0 < cn; j0 += 8) {
                        int2 e[8];
                        float bb[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int32_t kq = cb + (j0 + u < cn ? j0 + u : cn - 1);
                            e[u] = csc_cv[kq];
                            bb[u] = csc_b[kq];
                        }
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            if (j0 + u < cn)
                                stg[off - o0 + j0 + u] = make_int4(e[u].x, e[u].y, lane, __float_as_int(bb[u]));
                    }
                }
                uint64_t big = __ballot(mine && cn > 32);
                while (big) {
                    const int kk = __builtin_ctzll(big);
                    big &= big - 1;
                    const int32_t nk = pt_rdl(cn, kk), ok = pt_rdl(off, kk) - o0, bk = pt_rdl(cb, kk);
                    for (int32_t j = lane; j < nk; j += 64) {
                        const int2 e = csc_cv[bk + j];
                        stg[ok + j] = make_int4(e.x, e.y, kk, __float_as_int(csc_b[bk + j]));
                    }
                }
            }
            if (k == 0) {
                const int qn = clamp_mark(mraw_n, M);
                cb_n = csc_ptr[qn];
                ce_n = csc_ptr[qn + 1];
            }
            __syncthreads();
            for (int32_t g = 0; g < ne; g += 64 * PT_UA) {
                int32_t tp[PT_UA];
                double al[PT_UA], bt[PT_UA], tj[PT_UA];
#pragma unroll
                for (int u = 0; u < PT_UA; ++u) {
                    const int32_t f = g + 64 * u + lane;
                    const bool vf = f < ne;
                    int ej = k;
                    if (staged) {
                        const int4 r = stg[vf ? f : 0];
                        tp[u] = r.x;
                        al[u] = vf ? (double)__int_as_float(r.y) : 0.0;
                        ej = r.z;
                        bt[u] = (double)__int_as_float(r.w);
                    } else {
                        const int32_t kq = cbk + (vf ? f : 0);
                        const int2 e = csc_cv[kq];
                        tp[u] = e.x;
                        al[u] = vf ? (double)__int_as_float(e.y) : 0.0;
                        bt[u] = (double)csc_b[kq];
                    }
                    tj[u] = ev_t[ej];
                }
                // entries past the list carry alpha = 0 and add zeros
#pragma unroll
                for (int u = 0; u < PT_UA; ++u) {
                    const double d = te - tj[u], x0 = T - tj[u];
                    const double e = exp_f64(-bt[u] * d);
                    atomicAdd(&aR[tp[u]], al[u] * e);
                    atomicAdd(&aD[tp[u]], al[u] * d * e);
                    const double x = bt[u] * x0;
                    if (!FAR && x <= 745.0) {
                        atomicAdd(&aE[tp[u]], al[u] * x0 * exp_f64(-x));
                        comp += al[u] * -expm1(-x);
                    } else {
                        comp += al[u];
                    }
                }
            }
            __syncthreads();   // the stage is free again
            k = k2;
        }
    }
    __syncthreads();
    double* o = agg + (int64_t)s * 2 * M;
    double* oe = ebseg + (int64_t)s * M;
    for (int32_t q = lane; q < M; q += 64) {
        o[q] = aR[q];
        o[M + q] = aD[q];
        oe[q] = FAR ? 0.0 : aE[q];
    }
    for (int off = 32; off > 0; off >>= 1) comp += __shfl_down(comp, off, 64);
    if (lane == 0) {
        const double tr = a > 0 ? t[a - 1] : t[a];
        seg_span[s] = te - tr;
        seg_part[(int64_t)s * 4 + 1] = comp;
    }
}

// beta_min over the targets, into flags[0] (a float), once per call
__global__ __launch_bounds__(256) void pt_bmin(int32_t M, const float* __restrict__ beta, float* __restrict__ flags) {
    __shared__ float sm[256];
    float v = 3.0e38f;
    for (int32_t p = threadIdx.x; p < M; p += 256) v = beta[p] < v ? beta[p] : v;
    sm[threadIdx.x] = v;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h && sm[threadIdx.x + h] < sm[threadIdx.x]) sm[threadIdx.x] = sm[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) flags[0] = sm[0];
}

// flags[1] (an int): 1 when some entry of the chunk [c0, c1) can have
// beta_p (T - t_j) <= 745 (its compensator terms are not all zero)
__global__ void pt_near(int64_t c1, double T, const double* __restrict__ t, float* __restrict__ flags) {
    if (threadIdx.x == 0)
        reinterpret_cast<int32_t*>(flags)[1] = (double)flags[0] * (T - t[c1 - 1]) <= 745.0 ? 1 : 0;
}

// Pass 1 of the constant-memory gradient only carries the state from chunk to
// chunk: the state just after the chunk's last event t_e from the state just
// after the previous chunk's last event, with no per-segment maps and no
// scan.  pt_chain_part: a workgroup (one wave) takes PT_CHAIN_EV events of the
// chunk and sums their alpha-column pushes anchored at t_e in LDS, R_p +=
// alpha e^{-beta_p (t_e - t_j)} and D_p += (t_e - t_j) alpha e^{...}, lanes
// over staged column entries as in pt_seg_agg, and writes its partials.
// pt_chain_fold moves the carry to t_e and adds the partials in workgroup
// order (fixed order: the state, and every result after it, repeat bitwise).
template <int STG>
__global__ __launch_bounds__(64) void pt_chain_part(int64_t c0, int64_t c1, int32_t M, const double* __restrict__ t,
                                                    const int32_t* __restrict__ marks,
                                                    const int32_t* __restrict__ csc_ptr,
                                                    const int2* __restrict__ csc_cv, const float* __restrict__ csc_b,
                                                    double* __restrict__ part) {
    extern __shared__ double lds[];
    double* aR = lds;
    double* aD = lds + M;
    double* ev_t = lds + 2 * M;          // [64]
    int4* stg = (int4*)(ev_t + 64);      // [STG] (target, alpha, event, beta)
    const int32_t w = blockIdx.x;
    const int64_t a = c0 + (int64_t)w * PT_CHAIN_EV;
    const int64_t b = a + PT_CHAIN_EV < c1 ? a + PT_CHAIN_EV : c1;
    const int lane = threadIdx.x;
    for (int32_t q = lane; q < M; q += 64) { aR[q] = 0.0; aD[q] = 0.0; }
    const double te = t[c1 - 1];
    double tv_n;
    int32_t cb_n, ce_n;
    {
        const int64_t ic = a + lane < b ? a + lane : b - 1;
        tv_n = t[ic];
        const int q = clamp_mark(marks[ic], M);
        cb_n = csc_ptr[q];
        ce_n = csc_ptr[q + 1];
    }
    for (int64_t base = a; base < b; base += 64) {
        const bool ve = base + lane < b;
        const double tv = tv_n;
        const int32_t cb = cb_n;
        const int32_t cn = ve ? ce_n - cb : 0;
        int mraw_n;
        {
            const int64_t i2 = base + 64 + lane;
            const int64_t ic2 = i2 < b ? i2 : b - 1;
            tv_n = t[ic2];
            mraw_n = marks[ic2];
        }
        const int32_t off = wave_incl_scan_dpp(cn) - cn;   // exclusive
        const int32_t cend = off + cn;
        const int nb = (int)(b - base < 64 ? b - base : 64);
        __syncthreads();   // the previous batch is done with ev_t and the stage
        ev_t[lane] = tv;
        int k = 0;
        while (k < nb) {
            const int32_t o0 = pt_rdl(off, k);
            const int nfit = __builtin_popcountll(
                __builtin_amdgcn_ballot_w64(lane >= k && lane < nb && cend - o0 <= STG));
            const bool staged = nfit > 0;
            const int k2 = staged ? k + nfit : k + 1;
            const int32_t ne = pt_rdl(cend, k2 - 1) - o0;
            const int32_t cbk = pt_rdl(cb, k);
            if (staged) {
                const bool mine = lane >= k && lane < k2;
                if (mine && cn <= 32) {
                    for (int32_t j0 = 0; j0 < cn; j0 += 8) {
                        int2 e[8];
                        float bb[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int32_t kq = cb + (j0 + u < cn ? j0 + u : cn - 1);
                            e[u] = csc_cv[kq];
                            bb[u] = csc_b[kq];
                        }
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            if (j0 + u < cn)
                                stg[off - o0 + j0 + u] = make_int4(e[u].x, e[u].y, lane, __float_as_int(bb[u]));
                    }
                }
                uint64_t big = __ballot(mine && cn > 32);
                while (big) {
                    const int kk = __builtin_ctzll(big);
                    big &= big - 1;
                    const int32_t nk = pt_rdl(cn, kk), ok = pt_rdl(off, kk) - o0, bk = pt_rdl(cb, kk);
                    for (int32_t j = lane; j < nk; j += 64) {
                        const int2 e = csc_cv[bk + j];
                        stg[ok + j] = make_int4(e.x, e.y, kk, __float_as_int(csc_b[bk + j]));
                    }
                }
            }
            if (k == 0) {
                const int qn = clamp_mark(mraw_n, M);
                cb_n = csc_ptr[qn];
                ce_n = csc_ptr[qn + 1];
            }
            __syncthreads();
            for (int32_t g = 0; g < ne; g += 64 * PT_UA) {
                int32_t tp[PT_UA];
                double al[PT_UA], bt[PT_UA], tj[PT_UA];
#pragma unroll
                for (int u = 0; u < PT_UA; ++u) {
                    const int32_t f = g + 64 * u + lane;
                    const bool vf = f < ne;
                    int ej = k;
                    if (staged) {
                        const int4 r = stg[vf ? f : 0];
                        tp[u] = r.x;
                        al[u] = vf ? (double)__int_as_float(r.y) : 0.0;
                        ej = r.z;
                        bt[u] = (double)__int_as_float(r.w);
                    } else {
                        const int32_t kq = cbk + (vf ? f : 0);
                        const int2 e = csc_cv[kq];
                        tp[u] = e.x;
                        al[u] = vf ? (double)__int_as_float(e.y) : 0.0;
                        bt[u] = (double)csc_b[kq];
                    }
                    tj[u] = ev_t[ej];
                }
                // entries past the list carry alpha = 0 and add zeros
#pragma unroll
                for (int u = 0; u < PT_UA; ++u) {
                    const double d = te - tj[u];
                    const double e = exp_f64(-bt[u] * d);
                    atomicAdd(&aR[tp[u]], al[u] * e);
                    atomicAdd(&aD[tp[u]], al[u] * d * e);
                }
            }
            __syncthreads();   // the stage is free again
            k = k2;
        }
    }
    __syncthreads();
    double* o = part + (int64_t)w * 2 * M;
    for (int32_t q = lane; q < M; q += 64) {
        o[q] = aR[q];
        o[M + q] = aD[q];
    }
}

// carry (R, D just after t_r, the previous chunk's last event; t_r = t_0 for
// the first chunk, whose carry is zero) moved to t_e and the nw partials
// added: a workgroup of 8 waves per 64 targets, wave g sums its eighth of the
// partials in order, wave 0 adds the eighths in order
__global__ __launch_bounds__(512) void pt_chain_fold(int64_t c0, int64_t c1, int32_t M, int32_t nw,
                                                     const double* __restrict__ t, const float* __restrict__ beta,
                                                     const double* __restrict__ part, double* __restrict__ carry) {
    __shared__ double sR[8][64], sD[8][64];
    const int lane = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int32_t p = blockIdx.x * 64 + lane;
    const int32_t pc = p < M ? p : M - 1;
    const int32_t w0 = (int32_t)(((int64_t)g * nw) / 8), w1 = (int32_t)(((int64_t)(g + 1) * nw) / 8);
    double r = 0.0, d = 0.0;
    for (int32_t w = w0; w < w1; ++w) {
        r += part[(int64_t)w * 2 * M + pc];
        d += part[(int64_t)w * 2 * M + M + pc];
    }
    sR[g][lane] = r;
    sD[g][lane] = d;
    __syncthreads();
    if (g != 0 || p >= M) return;
    const double tr = c0 > 0 ? t[c0 - 1] : t[c0], te = t[c1 - 1];
    const double span = te - tr;
    const double ex = exp(-(double)beta[p] * span);
    const double k0 = carry[p];
    double R = ex * k0, D = ex * __builtin_fma(span, k0, carry[M + p]);
    for (int h = 0; h < 8; ++h) {
        R += sR[h][lane];
        D += sD[h][lane];
    }
    carry[p] = R;
    carry[M + p] = D;
}

// Forward pass over one segment (one wave), 64 events per batch.  LDS keeps
// one lazy record per target (time tau_p, R_p and D_p at tau_p), initialised
// from the scanned carry.  Per batch:
//  1. read: lane i moves its own target's record to t_i: R_p(t_i), D_p(t_i)
//     from the events before the batch;
//  2. push: the batch's alpha-column entries (event j, target p, alpha),
//     staged in LDS, PT_U a lane per pass, lanes over entries.  The first
//     entry of a target in the batch moves its record to the batch's last
//     time t_B (it claims the record by exchanging tau_p for t_B); then every
//     entry adds alpha e^{-beta_p (t_B - t_j)} to R_p and (t_B - t_j) times
//     that to D_p (in a segment short enough for anchored records, below,
//     the entry only adds to its target's sums).  An entry whose target is
//     the own target of a later event
//     i of the batch (a byte per node names one batch event with that own
//     target, a mask per event all of them) adds its share at t_i,
//     alpha e^{-beta_p (t_i - t_j)}, to that event;
//  3. finish: lane i adds its shares, lambda_i = mu_p + beta_p R_p(t_i).
// Events tied in time keep index order (a later event sees an earlier one's
// push at distance 0), as in the recurrence.
template <bool GRAD, bool INTENS>
__global__ __launch_bounds__(64) void pt_forward(int64_t c0, int64_t c1, int32_t M, double T,
                                                 const double* __restrict__ t, const int32_t* __restrict__ marks,
                                                 const float* __restrict__ mu, const float* __restrict__ beta,
                                                 const int32_t* __restrict__ csc_ptr,
                                                 const int2* __restrict__ csc_cv, const float* __restrict__ csc_b,
                                                 const double* __restrict__ carry_seg, double* __restrict__ seg_part,
                                                 double* __restrict__ ebseg, float* __restrict__ wv,
                                                 float* __restrict__ lambda_out) {
    // wv: 1/lambda of the chunk's events, indexed from the chunk start c0
    extern __shared__ double lds[];
    double* rtau = lds;
    double* rR = lds + M;
    double* rD = lds + 2 * M;
    double* gbl = lds + 3 * M;   // per-target sum of w_i (R_i - beta_p D_i) over the segment
    double* ev_t = lds + 4 * M;  // [64] the batch's event times
    double* shR = ev_t + 64;     // [64] the batch's in-batch shares of R and D
    double* shD = shR + 64;
    uint64_t* smask = (uint64_t*)(shD + 64);   // [64] events of the batch with event i's own target
    int4* stg = (int4*)(smask + 64);           // [PT_STAGE] (target, alpha, event, beta)
    // [M] per target: an event of the batch with that own target, 0xff none
    uint8_t* tev = (uint8_t*)(stg + PT_STAGE);
    const int32_t s = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t a = c0 + (int64_t)s * HK_SEG;
    const int64_t b = a + HK_SEG < c1 ? a + HK_SEG : c1;
    const double tref = a > 0 ? t[a - 1] : t[a];
    const double* cs = carry_seg + (int64_t)s * 2 * M;
    // Anchored records when the segment's span allows, beta_max (t_last -
    // t_ref) <= 600: with u = t - t_ref, rR[p] = S0_p = sum_j alpha e^{beta_p u_j}
    // and rD[p] = S1_p = sum_j alpha u_j e^{beta_p u_j} over the pushes so far
    // (the carry enters as S0 = R(t_ref), S1 = -D(t_ref)); then R_p(t) =
    // e^{-beta_p u} S0_p and D_p(t) = e^{-beta_p u} (u S0_p - S1_p), pushes are
    // plain additions and no record is claimed or moved.  Otherwise each
    // record keeps its own time rtau[p] and is moved on use.
    float bmx = 0.0f;
    for (int32_t q = lane; q < M; q += 64) bmx = beta[q] > bmx ? beta[q] : bmx;
    for (int o = 32; o > 0; o >>= 1) {
        const float v = __shfl_xor(bmx, o, 64);
        bmx = v > bmx ? v : bmx;
    }
    const bool anch = __builtin_amdgcn_readfirstlane((int)((double)bmx * (t[b - 1] - tref) <= 600.0)) != 0;
    // records from the carry, eight rows of 64 in flight at a time
    for (int32_t q0 = 0; q0 < M; q0 += 512) {
        double r[8], d[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int32_t q = q0 + 64 * u + lane < M ? q0 + 64 * u + lane : M - 1;
            r[u] = cs[q];
            d[u] = cs[M + q];
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int32_t q = q0 + 64 * u + lane;
            if (q < M) {
                rtau[q] = tref;
                rR[q] = r[u];
                rD[q] = anch ? -d[u] : d[u];
                gbl[q] = 0.0;
            }
        }
    }
    for (int32_t q = lane; q < M; q += 64) tev[q] = 0xff;
    double logsum = 0.0;
    // the next batch's event, its column extent, decay and base rate are
    // loaded one batch ahead (one wave per CU: nothing else hides the
    // latency of global memory)
    double tv_n;
    int mv_n;
    int32_t cb_n, ce_n;
    float bm_n, mu_n;
    {
        const int64_t ic = a + lane < b ? a + lane : b - 1;
        tv_n = t[ic];
        mv_n = clamp_mark(marks[ic], M);
        cb_n = csc_ptr[mv_n];
        ce_n = csc_ptr[mv_n + 1];
        bm_n = beta[mv_n];
        mu_n = mu[mv_n];
    }
    for (int64_t base = a; base < b; base += 64) {
        const int64_t ie = base + lane;
        const bool ve = ie < b;
        const double tv = tv_n;
        const int mv = mv_n;
        const int nb = (int)(b - base < 64 ? b - base : 64);
        const double tB = pt_rdl_d(tv, nb - 1);
        const double bm = (double)bm_n, mub = (double)mu_n;
        // column extents of the batch's marks and their exclusive prefix
        const int32_t cb = cb_n;
        const int32_t cn = ve ? ce_n - cb : 0;
        int mraw_n = 0;
        {
            const int64_t i2 = base + 64 + lane;
            const int64_t ic2 = i2 < b ? i2 : b - 1;
            tv_n = t[ic2];
            mraw_n = marks[ic2];
        }
        const int32_t off = wave_incl_scan_dpp(cn) - cn;   // exclusive
        ev_t[lane] = tv;
        shR[lane] = 0.0;
        shD[lane] = 0.0;
        smask[lane] = 0ull;
        __syncthreads();   // also orders the previous batch's pushes before the reads
        // 1. own target's record at t_i, and the table of own targets
        double Rk, Dk;
        if (anch) {
            const double u = tv - tref;
            const double e = exp_f64(-bm * u);
            const double s0 = rR[mv];
            Rk = e * s0;
            Dk = e * __builtin_fma(u, s0, -rD[mv]);
        } else {
            const double d = tv - rtau[mv];
            const double e = exp_f64(-bm * d);
            const double r = rR[mv];
            Rk = e * r;
            Dk = e * __builtin_fma(d, r, rD[mv]);
        }
        // one event per own target stands for all of them (the store that
        // lands last), and collects their mask
        if (ve) tev[mv] = (uint8_t)lane;
        lds_wait();
        if (ve) atomicOr((unsigned long long*)&smask[tev[mv]], 1ull << lane);
        mv_n = clamp_mark(mraw_n, M);
        cb_n = csc_ptr[mv_n];
        ce_n = csc_ptr[mv_n + 1];
        bm_n = beta[mv_n];
        mu_n = mu[mv_n];
        __syncthreads();
        // 2. pushes, in stretches of events [k, k2) whose entries fit the stage
        const int32_t cend = off + cn;   // end of the event's entries in the batch
        int k = 0;
        while (k < nb) {
            const int32_t o0 = pt_rdl(off, k);
            // events from k on whose entries end inside the stage (a prefix,
            // the ends grow with the lane); at least event k
            const int nfit = __builtin_popcountll(
                __builtin_amdgcn_ballot_w64(lane >= k && lane < nb && cend - o0 <= PT_STAGE));
            const bool staged = nfit > 0;
            const int k2 = staged ? k + nfit : k + 1;
            const int32_t ne = pt_rdl(cend, k2 - 1) - o0;
            const int32_t cbk = pt_rdl(cb, k);
            if (staged) {
                // short columns: each lane copies its own event's column;
                // long ones: all lanes copy one column at a time (coalesced)
                const bool mine = lane >= k && lane < k2;
                if (mine && cn <= 32) {
                    for (int32_t j0 = 0; j0 < cn; j0 += 8) {
                        // eight entries and their targets' decays in flight
                        int2 e[8];
                        float bb[8];
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            const int32_t kq = cb + (j0 + u < cn ? j0 + u : cn - 1);
                            e[u] = csc_cv[kq];
                            bb[u] = csc_b[kq];
                        }
#pragma unroll
                        for (int u = 0; u < 8; ++u)
                            if (j0 + u < cn)
                                stg[off - o0 + j0 + u] = make_int4(e[u].x, e[u].y, lane, __float_as_int(bb[u]));
                    }
                }
                uint64_t big = __ballot(mine && cn > 32);
                while (big) {
                    const int kk = __builtin_ctzll(big);
                    big &= big - 1;
                    const int32_t nk = pt_rdl(cn, kk), ok = pt_rdl(off, kk) - o0, bk = pt_rdl(cb, kk);
                    for (int32_t j = lane; j < nk; j += 64) {
                        const int2 e = csc_cv[bk + j];
                        stg[ok + j] = make_int4(e.x, e.y, kk, __float_as_int(csc_b[bk + j]));
                    }
                }
                __syncthreads();
            }
            // PT_U entries a lane per pass: their loads, claims and table
            // probes in flight together, their decays as straight-line code
            for (int32_t g = 0; g < ne; g += 64 * PT_U) {
                int32_t tp[PT_U], ej[PT_U];
                double av[PT_U], bt[PT_U];
                bool vf[PT_U];
#pragma unroll
                for (int u = 0; u < PT_U; ++u) {
                    const int32_t f = g + 64 * u + lane;
                    vf[u] = f < ne;
                    if (staged) {
                        const int4 r = stg[vf[u] ? f : 0];
                        tp[u] = r.x;
                        av[u] = (double)__int_as_float(r.y);
                        ej[u] = r.z;
                        bt[u] = (double)__int_as_float(r.w);
                    } else {
                        const int32_t kq = cbk + (vf[u] ? f : 0);
                        const int2 e = csc_cv[kq];
                        tp[u] = e.x;
                        av[u] = (double)__int_as_float(e.y);
                        ej[u] = k;
                        bt[u] = (double)csc_b[kq];
                    }
                }
                double tj[PT_U];
                int rep[PT_U];
                uint64_t mk[PT_U];
                if (anch) {
                    // anchored: every entry adds alpha e^{beta u_j} (and u_j
                    // times that) to its target's sums
#pragma unroll
                    for (int u = 0; u < PT_U; ++u) {
                        tj[u] = ev_t[ej[u]];
                        rep[u] = tev[tp[u]];
                    }
                    double g[PT_U], uj[PT_U];
#pragma unroll
                    for (int u = 0; u < PT_U; ++u) {
                        uj[u] = tj[u] - tref;
                        g[u] = av[u] * exp_f64(bt[u] * uj[u]);
                    }
#pragma unroll
                    for (int u = 0; u < PT_U; ++u) {
                        if (vf[u]) {
                            atomicAdd(&rR[tp[u]], g[u]);
                            atomicAdd(&rD[tp[u]], uj[u] * g[u]);
                        }
                    }
                } else {
                    // claim: the first entry of its target moves the record to tB
                    double told[PT_U];
#pragma unroll
                    for (int u = 0; u < PT_U; ++u) {
                        tj[u] = ev_t[ej[u]];
                        told[u] = tB;
                        if (vf[u])
                            told[u] = __longlong_as_double((long long)atomicExch(
                                (unsigned long long*)&rtau[tp[u]], (unsigned long long)__double_as_longlong(tB)));
                        rep[u] = tev[tp[u]];
                    }
                    double e0[PT_U], c[PT_U], dB[PT_U];
#pragma unroll
                    for (int u = 0; u < PT_U; ++u) {
                        e0[u] = exp_f64(-bt[u] * (tB - told[u]));   // 1 unless claimed
                        dB[u] = tB - tj[u];
                        c[u] = av[u] * exp_f64(-bt[u] * dB[u]);
                    }
#pragma unroll
                    for (int u = 0; u < PT_U; ++u) {
                        if (vf[u] && told[u] != tB) {
                            const double d0 = tB - told[u];
                            const double r0 = rR[tp[u]];
                            rD[tp[u]] = e0[u] * __builtin_fma(d0, r0, rD[tp[u]]);
                            rR[tp[u]] = e0[u] * r0;
                        }
                    }
                    lds_wait();   // the moves land before any entry's add
#pragma unroll
                    for (int u = 0; u < PT_U; ++u) {
                        if (vf[u]) {
                            atomicAdd(&rR[tp[u]], c[u]);
                            atomicAdd(&rD[tp[u]], dB[u] * c[u]);
                        }
                    }
                }
                // events of the batch after the entry's event whose own
                // target is the entry's (rare: 64 own targets of M)
#pragma unroll
                for (int u = 0; u < PT_U; ++u)
                    mk[u] = vf[u] && rep[u] != 0xff ? smask[rep[u] & 63] & ~((2ull << ej[u]) - 1ull) : 0ull;
                // their shares at t_i, one (entry, event) pair a lane per round
                for (;;) {
                    int i = -1;
                    double tju = 0.0, avu = 0.0, btu = 0.0;
#pragma unroll
                    for (int u = PT_U - 1; u >= 0; --u) {
                        if (mk[u]) {
                            i = __builtin_ctzll(mk[u]);
                            tju = tj[u];
                            avu = av[u];
                            btu = bt[u];
                        }
                    }
                    if (!__builtin_amdgcn_ballot_w64(i >= 0)) break;
                    bool done = false;
#pragma unroll
                    for (int u = 0; u < PT_U; ++u) {
                        if (!done && mk[u]) {
                            mk[u] &= mk[u] - 1;
                            done = true;
                        }
                    }
                    if (i >= 0) {
                        const double di = ev_t[i] - tju;
                        const double ci = avu * exp_f64(-btu * di);
                        atomicAdd(&shR[i], ci);
                        atomicAdd(&shD[i], di * ci);
                    }
                }
            }
            if (staged) __syncthreads();   // the stage is free again
            k = k2;
        }
        __syncthreads();
        if (ve) tev[mv] = 0xff;   // the table is empty again for the next batch
        // 3. the event's intensity
        if (ve) {
            Rk += shR[lane];
            Dk += shD[lane];
            const double lam = mub + bm * Rk;
            logsum += log(lam);
            if (INTENS) lambda_out[ie] = (float)lam;
            if (GRAD) {
                const double w = 1.0 / lam;
                wv[ie - c0] = (float)w;
                atomicAdd(&gbl[mv], w * (Rk - bm * Dk));
            }
        }
    }
    if (GRAD) {
        // the segment's row of ebseg becomes EB - GB (minus its dL/dbeta share)
        __syncthreads();
        double* oe = ebseg + (int64_t)s * M;
        for (int32_t q0 = 0; q0 < M; q0 += 512) {
            double v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = oe[q0 + 64 * u + lane < M ? q0 + 64 * u + lane : M - 1];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int32_t q = q0 + 64 * u + lane;
                if (q < M) oe[q] = v[u] - gbl[q];
            }
        }
    }
    for (int off = 32; off > 0; off >>= 1) logsum += __shfl_down(logsum, off, 64);
    if (lane == 0) {
        double* o = seg_part + (int64_t)s * 4;
        o[0] = logsum;
        o[2] = 0.0;
        o[3] = 0.0;
    }
}

// ebacc[p] += sum over the chunk's segments: a workgroup per 64 targets,
// 16 slices of the segments summed side by side (each in segment order),
// then the slices in order (a fixed order: repeatable)
__global__ __launch_bounds__(1024) void pt_eb_reduce(int32_t nseg, int32_t M, const double* __restrict__ ebseg,
                                                     double* __restrict__ ebacc) {
    __shared__ double part[16][64];
    const int lane = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const int32_t p = blockIdx.x * 64 + lane;
    const int32_t per = (nseg + 15) / 16;
    const int32_t s0 = sl * per, s1 = s0 + per < nseg ? s0 + per : nseg;
    double v = 0.0;
    if (p < M)
        for (int32_t s = s0; s < s1; ++s) v += ebseg[(int64_t)s * M + p];
    part[sl][lane] = v;
    __syncthreads();
    if (sl == 0 && p < M) {
        double tot = 0.0;
        for (int k = 0; k < 16; ++k) tot += part[k][lane];
        ebacc[p] += tot;
    }
}

// ------------------------------------------------------------------ pass 2
// time of segment s's first event; for s == nseg, the time the chunk's right
// carry refers to (the next chunk's first event, or T after the last chunk)
__device__ __forceinline__ double seg_first_time(const double* __restrict__ t, int64_t c0, int64_t c1, int64_t n,
                                                 int32_t nseg, int32_t s, double T) {
    if (s >= nseg) return c1 < n ? t[c1] : T;
    return t[c0 + (int64_t)s * HK_SEG];
}

// aggA[s][p] = sum_{i in segment s, m_i = p} w_i e^{-beta_p (t_i - t_first(s))}
// (wv indexed from the chunk start c0); one wave per segment, LDS aA[M]
__global__ __launch_bounds__(64) void pt_rev_agg(int64_t c0, int64_t c1, int32_t M, const double* __restrict__ t,
                                                 const int32_t* __restrict__ marks, const float* __restrict__ beta,
                                                 const float* __restrict__ wv, double* __restrict__ aggA) {
    extern __shared__ double lds[];
    double* aA = lds;
    const int32_t s = blockIdx.x;
    const int64_t a = c0 + (int64_t)s * HK_SEG;
    const int64_t b = a + HK_SEG < c1 ? a + HK_SEG : c1;
    const int lane = threadIdx.x;
    for (int32_t q = lane; q < M; q += 64) aA[q] = 0.0;
    __syncthreads();
    const double tf = t[a];
    for (int64_t base = a; base < b; base += 64) {
        const int64_t i = base + lane;
        if (i < b) {
            const int p = clamp_mark(marks[i], M);
            const double w = (double)wv[i - c0];
            atomicAdd(&aA[p], w * (double)exp2_f64arg((tf - t[i]) * ((double)beta[p] * HK_LOG2E)));
        }
    }
    __syncthreads();
    double* o = aggA + (int64_t)s * M;
    for (int32_t q = lane; q < M; q += 64) o[q] = aA[q];
}

// Reverse scan in three parallel steps, mirroring the forward one:
//   local   1 thread per (group, target): suffix inside the group
//   groups  1 thread per target: chain the groups from the chunk's right carry
//   apply   1 thread per (segment, target): add the group's right carry
// rcarry_seg[s][p] ends as A_p at t_first(s) from the events of segment s on
// (this and later chunks, plus the seed).
__global__ void pt_rscan_local(int64_t c0, int64_t c1, int64_t n, double T, int32_t nseg, int32_t M,
                               const double* __restrict__ t, const float* __restrict__ beta,
                               const double* __restrict__ aggA, double* __restrict__ rcarry_seg,
                               double* __restrict__ rgagg) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int32_t ngr = (nseg + HK_SG - 1) / HK_SG;
    if (gid >= (int64_t)ngr * M) return;
    const int32_t g = (int32_t)(gid / M), p = (int32_t)(gid % M);
    const int32_t s0 = g * HK_SG, s1 = s0 + HK_SG < nseg ? s0 + HK_SG : nseg;
    const double bp = (double)beta[p];
    double A = 0.0, tn = seg_first_time(t, c0, c1, n, nseg, s1, T);
    for (int32_t s = s1 - 1; s >= s0; --s) {
        const double ts = seg_first_time(t, c0, c1, n, nseg, s, T);
        A = __builtin_fma(exp(-bp * (tn - ts)), A, aggA[(int64_t)s * M + p]);
        rcarry_seg[(int64_t)s * M + p] = A;
        tn = ts;
    }
    rgagg[(int64_t)g * M + p] = A;
}

__global__ void pt_rscan_groups(int64_t c0, int64_t c1, int64_t n, double T, int32_t nseg, int32_t M,
                                const double* __restrict__ t, const float* __restrict__ beta,
                                const double* __restrict__ rgagg, double* __restrict__ rgcarry,
                                double* __restrict__ achunk) {
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    const int32_t ngr = (nseg + HK_SG - 1) / HK_SG;
    const double bp = (double)beta[p];
    double A = achunk[p], tn = seg_first_time(t, c0, c1, n, nseg, nseg, T);
    for (int32_t g = ngr - 1; g >= 0; --g) {
        rgcarry[(int64_t)g * M + p] = A;
        const double ts = seg_first_time(t, c0, c1, n, nseg, g * HK_SG, T);
        A = __builtin_fma(exp(-bp * (tn - ts)), A, rgagg[(int64_t)g * M + p]);
        tn = ts;
    }
    achunk[p] = A;
}

__global__ void pt_rscan_apply(int64_t c0, int64_t c1, int64_t n, double T, int32_t nseg, int32_t M,
                               const double* __restrict__ t, const float* __restrict__ beta,
                               const double* __restrict__ rgcarry, double* __restrict__ rcarry_seg) {
    const int64_t gid = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (gid >= (int64_t)nseg * M) return;
    const int32_t s = (int32_t)(gid / M), p = (int32_t)(gid % M);
    const int32_t g = s / HK_SG;
    const int32_t s1 = (g + 1) * HK_SG < nseg ? (g + 1) * HK_SG : nseg;
    const double te = seg_first_time(t, c0, c1, n, nseg, s1, T);
    const double ts = seg_first_time(t, c0, c1, n, nseg, s, T);
    rcarry_seg[(int64_t)s * M + p] += exp(-(double)beta[p] * (te - ts)) * rgcarry[(int64_t)g * M + p];
}

// Dense adjoint kernel.  Block = (target block rb, source block sb, event
// range er), HK_DWP waves, each over its share of the range's segments; lane
// l owns target p = r0 + l and beta_p A_p (float64), A_p the adjoint state
// from the events after the current read position, kept at an anchor time.
// The block reads only the bucketed records of its two node blocks ("own":
// targets in rb; "slab": sources in sb), from the end of the range
// backwards, merged by event index in windows of up to 64 + 64 records (the
// window starts where either list's 64th record from the end is).  Per
// window: A moves to the window's latest event time tw; every slab event k
// adds beta_p A_p(t_k) to column m_k of the block: the state decayed to t_k
// plus the window's own-target events after k.  Three forms, by the window's
// largest decay exponent beta_max (tw - t_last): short windows (<= 0.5) and
// windows past HK_PT_MERGE_SPAN add the own events' part pairwise (one
// masked ds_add per slab event) and then enter the own events into A at the
// window's earliest time; the windows between enter them into A in event
// order inside the slab loop.  G is kept in LDS column-major (stride 65
// against bank conflicts).  Blocks with sb == 0 also sum w_i per target,
// blocks with rb == 0 count the events per source.
__global__ __launch_bounds__(64 * HK_DWP) void pt_dense(int64_t c0, int64_t c1, int64_t n, double T, int32_t M, int32_t NB,
                                               int32_t ER, int32_t segs_per_range, int32_t nseg,
                                               const double* __restrict__ t, const float* __restrict__ beta,
                                               const double* __restrict__ rcarry_seg,
                                               const double* __restrict__ rgcarry,
                                               const int32_t* __restrict__ bk_off,
                                               const int32_t* __restrict__ bk_base,
                                               const uint32_t* __restrict__ bk_key, const double* __restrict__ bk_t,
                                               const float* __restrict__ bk_w, double* __restrict__ gpart,
                                               double* __restrict__ spart, double* __restrict__ npart) {
    __shared__ double G[HK_SLAB * 65];   // shared by the group's waves
    __shared__ double ALs[HK_DWP][64], SLs[HK_DWP][64], NLs[HK_DWP][64];
    __shared__ float BL[64];
    const int lane = threadIdx.x & 63;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);   // wave-uniform
    double* AL = ALs[wv];
    double* SL = SLs[wv];
    double* NL = NLs[wv];
    AL[lane] = 0.0;
    SL[lane] = 0.0;
    NL[lane] = 0.0;
    const int32_t blk = blockIdx.x;
    const int32_t nbb = NB * NB;
    int32_t er, local;
    if (ER >= 8) {
        const int32_t slot = blk >> 3;
        er = (slot / nbb) * 8 + (blk & 7);
        local = slot % nbb;
    } else {
        const int32_t per = 8 / ER, x = blk & 7;
        er = x / per;
        local = (blk >> 3) * per + x % per;
        if (local >= nbb) return;
    }
    if (er >= ER) return;
    const int32_t sb = local % NB;
    const int32_t rb = local / NB;
    const int32_t r0 = rb * HK_RB, s0 = sb * HK_SLAB;
    const int32_t gA = er * segs_per_range;
    if (gA >= nseg) return;
    const int32_t gB = gA + segs_per_range < nseg ? gA + segs_per_range : nseg;
    // this wave's share of the range's segments (possibly none)
    const int32_t sA = gA + (wv * (gB - gA)) / HK_DWP;
    const int32_t sB = gA + ((wv + 1) * (gB - gA)) / HK_DWP;
    const int32_t p = r0 + lane;
    const bool pv = p < M;
    BL[lane] = pv ? beta[p] : 0.0f;
    double* gp = gpart + (int64_t)er * M * M;
    {
        // lanes over the block's columns (coalesced rows of gpart)
        const int32_t col = s0 + lane;
        const int32_t cc = col < M ? col : M - 1;
        for (int rg = wv * 16; rg < HK_RB; rg += 16 * HK_DWP) {
            double v[16];
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int32_t row = r0 + rg + j;
                const int32_t rr = row < M ? row : M - 1;
                v[j] = gp[(int64_t)rr * M + cc];
            }
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                const int32_t row = r0 + rg + j;
                G[lane * 65 + rg + j] = (row < M && col < M) ? v[j] : 0.0;
            }
        }
    }
    const double bp = pv ? (double)beta[p] : 0.0;
    const double bp2 = bp * HK_LOG2E;                      // beta_p log2(e)
    const float bpl = (float)bp2;
    const float bpl_lo = (float)(bp2 - (double)bpl);       // bp2 = bpl + bpl_lo to ~2^-48
    // largest decay of the block's targets
    double bmax = bp;
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(bmax, off, 64);
        bmax = o > bmax ? o : bmax;
    }
    // adjoint state from the events after the range (and the seed) at tau
    const bool at_end = sB >= nseg;
    double tau = seg_first_time(t, c0, c1, n, nseg, at_end ? nseg : sB, T);
    double Ab = 0.0;   // beta_p A_p at the anchor tau
    if (pv) {
        const int32_t ngr = (nseg + HK_SG - 1) / HK_SG;
        Ab = bp * (at_end ? rgcarry[(int64_t)(ngr - 1) * M + p] : rcarry_seg[(int64_t)sB * M + p]);
    }
    RecStream<true> O, S;
    O.init(bk_key, bk_t, bk_w, (int64_t)bk_base[rb] + bk_off[(int64_t)rb * (nseg + 1) + sA],
           (int64_t)bk_base[rb] + bk_off[(int64_t)rb * (nseg + 1) + sB]);
    S.init(bk_key, bk_t, bk_w, (int64_t)bk_base[sb] + bk_off[(int64_t)sb * (nseg + 1) + sA],
           (int64_t)bk_base[sb] + bk_off[(int64_t)sb * (nseg + 1) + sB]);
    O.settle();
    S.settle();
    __syncthreads();
    for (;;) {
        if (sA >= sB) break;
        const int64_t ao = O.avail(), as = S.avail();
        if (ao <= 0 && as <= 0) break;
        const int io = (int)(O.ck >> 6), is = (int)(S.ck >> 6);
        const int lim_o = ao > 64 ? rl_i(io, 63) : -1;
        const int lim_s = as > 64 ? rl_i(is, 63) : -1;
        const int lo = lim_o > lim_s ? lim_o : lim_s;
        const bool own = lane < ao && io >= lo;
        const bool sl = lane < as && is >= lo;
        const int no = __builtin_popcountll(__ballot(own));
        const int ns = __builtin_popcountll(__ballot(sl));
        double tw = -1e300, tl = 1e300;
        if (no) { tw = rl_d(O.ct, 0); tl = rl_d(O.ct, no - 1); }
        if (ns) {
            const double a0 = rl_d(S.ct, 0), a1 = rl_d(S.ct, ns - 1);
            tw = a0 > tw ? a0 : tw;
            tl = a1 < tl ? a1 : tl;
        }
        Ab *= (double)exp2_f64arg((tw - tau) * bp2);
        const int pi = (int)(O.ck & 63u);
        const double bo = (double)BL[pi];
        const double bo2 = bo * HK_LOG2E;
        const float bol = (float)bo2;
        const double wi = (double)O.cw;
        bool merged = false;
        if (bmax * (tw - tl) <= 0.5) {
            // short window: every decay exponent is at most 0.5 in magnitude,
            // so float32 arguments cost at most 2.5e-7 relative and the
            // hardware exp2 applies directly.  The time differences are taken
            // in float64 once per lane (slab lane k: tw - t_k; own lane:
            // t_i - tw, folded into the exponent's constant), then each slab
            // event's offset and key are broadcast by one readlane apiece.
            // Lanes without an own event add 0 to their own column slot (a
            // finite 0: their exponent constant is 0, not a stale record's).
            const float dks = (float)(tw - S.ct);
            const float c2 = own ? -bol * (float)(O.ct - tw) : 0.0f;
            const int pa = own ? pi : lane;
            const double bA = Ab, bw = own ? bo * wi : 0.0;
            const int keys = (int)S.ck;
            for (int k = 0; k < ns; ++k) {
                const uint32_t key = (uint32_t)rl_i(keys, k);
                const float dk = rl_f(dks, k);
                const int qoff = (int)(key & 63u) * 65;
                const float e1 = __builtin_amdgcn_exp2f(-bpl * dk);
                const float e2 = __builtin_amdgcn_exp2f(__builtin_fmaf(-bol, dk, c2));
                atomicAdd(&G[qoff + lane], bA * (double)e1);
                // own event later than slab event k (both lists newest first)
                atomicAdd(&G[qoff + pa], bw * (double)(io > (int)(key >> 6) ? e2 : 0.0f));
            }
        } else if (bmax * (tw - tl) <= HK_PT_MERGE_SPAN) {
            // long window, merged: A is moved to the anchor tw, and the
            // window's own events enter it in event order between the slab
            // events (newest first), each as beta_{m_i} w_i e^{beta_{m_i}
            // (tw - t_i)} on its target's lane, so every slab event needs one decay
            // e^{-beta_p (tw - t_k)} per lane and one ds_add.  The span bound
            // keeps both factors inside float32's exponent range.  The decay's
            // exponent is split in two floats (tw - t_k = dh + dl, beta_p
            // log2(e) = bpl + bpl_lo, and the product's rounding error by an
            // fma), so 2^-x = 2^-xh (1 - xl ln2) is as accurate as the
            // hardware exp2 at any x in range.
            merged = true;
            const double dd = tw - S.ct;
            const float dh = (float)dd, dl0 = (float)(dd - (double)dh);
            // per slab lane k: the own events later than it, the first dcnt of
            // the own list (both lists newest first: a binary search over the
            // own indices), and with its column in the 13 low mantissa bits of
            // the low part of its offset (dl changes by at most 2^-10 of
            // itself, 2^-34 of the offset), so that one readlane gives all
            int dcnt = 0;
#pragma unroll
            for (int step = 64; step >= 1; step >>= 1) {
                const int probe = dcnt + step - 1;
                const int ov = __shfl(io, probe & 63, 64);
                if (probe < no && ov > is) dcnt += step;
            }
            const float dl = __int_as_float((__float_as_int(dl0) & ~8191) | (dcnt << 6) | (int)(S.ck & 63u));
            // the own event's target lane rides in the 6 low mantissa bits of
            // its weight (a change of at most 2^-46 relative), so one pair
            // of readlanes gives both
            const double fo = own ? bo * wi * (double)exp2_f64arg((tw - O.ct) * bo2) : 0.0;
            const double fop = __longlong_as_double((__double_as_longlong(fo) & ~63ll) | (long long)pi);
            int j = 0;
            for (int k = 0; k < ns; ++k) {
                const float xl0 = rl_f(dl, k);
                const int kb = __float_as_int(xl0);
                // own events later than slab event k (the first dk of the
                // list, newest first) join A before it
                const int dk = (kb >> 6) & 127;
                for (; j < dk; ++j) {
                    const double f = rl_d(fop, j);
                    if (lane == (int)(__double_as_longlong(f) & 63)) {
                        Ab += f;
                        // keeps the add under the lane's exec mask (else the
                        // compiler adds on every lane and selects: two more
                        // vector instructions per own event)
                        __asm__ volatile("" : "+v"(Ab));
                    }
                }
                const float xh0 = rl_f(dh, k);
                const float xh = bpl * xh0;
                const float xl = __builtin_fmaf(bpl, xl0, __builtin_fmaf(bpl_lo, xh0, __builtin_fmaf(bpl, xh0, -xh)));
                const float e0 = __builtin_amdgcn_exp2f(-xh);
                const float e = __builtin_fmaf(e0, xl * -0.69314718f, e0);
                atomicAdd(&G[(kb & 63) * 65 + lane], Ab * (double)e);
            }
            // own events older than every slab event of the window
            for (; j < no; ++j) {
                const double f = rl_d(fop, j);
                if (lane == (int)(__double_as_longlong(f) & 63)) {
                    Ab += f;
                    __asm__ volatile("" : "+v"(Ab));
                }
            }
        } else {
            for (int k = 0; k < ns; ++k) {
                const int qoff = (int)(rl_i((int)S.ck, k) & 63) * 65;
                const double tk = rl_d(S.ct, k);
                const int ik = rl_i(is, k);
                atomicAdd(&G[qoff + lane], Ab * (double)exp2_f64arg((tk - tw) * bp2));
                if (own && io > ik) atomicAdd(&G[qoff + pi], bo * wi * (double)exp2_f64arg((tk - O.ct) * bo2));
            }
        }
        if (sb == 0 && own) atomicAdd(&SL[pi], wi);
        if (rb == 0 && sl) atomicAdd(&NL[S.ck & 63u], 1.0);
        if (merged) {
            tau = tw;   // A already holds the window's own events, anchored at tw
        } else {
            if (own) atomicAdd(&AL[pi], bo * wi * (double)exp2_f64arg((tl - O.ct) * bo2));
            // AL is this wave's; its atomics land before the read
            lds_wait();
            Ab = __builtin_fma(Ab, (double)exp2_f64arg((tl - tw) * bp2), AL[lane]);
            __builtin_amdgcn_wave_barrier();
            AL[lane] = 0.0;
            __builtin_amdgcn_wave_barrier();
            tau = tl;
        }
        O.shift(no);
        S.shift(ns);
        O.refill();
        S.refill();
    }
    __syncthreads();
    {
        const int32_t col = s0 + lane;
        if (col < M) {
#pragma unroll 16
            for (int r = wv; r < HK_RB; r += HK_DWP) {
                const int32_t row = r0 + r;
                if (row < M) gp[(int64_t)row * M + col] = G[lane * 65 + r];
            }
        }
    }
    if (wv != 0) return;
    // the waves' sums, in wave order
    double sl = 0.0, nl = 0.0;
    for (int v = 0; v < HK_DWP; ++v) {
        sl += SLs[v][lane];
        nl += NLs[v][lane];
    }
    if (sb == 0 && pv) spart[(int64_t)er * M + p] += sl;
    if (rb == 0 && s0 + lane < M) npart[(int64_t)er * M + s0 + lane] += nl;
}

__global__ __launch_bounds__(256) void pt_final(int32_t M, int32_t ER, double T, const float* __restrict__ mu,
                         const double* __restrict__ acc, const double* __restrict__ gpart,
                         const double* __restrict__ spart, const double* __restrict__ npart,
                         const double* __restrict__ ebacc,
                         double* __restrict__ loglik, double* __restrict__ g_mu, double* __restrict__ g_alpha,
                         double* __restrict__ g_beta, int grad) {
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
        if (threadIdx.x == 0) loglik[0] = acc[0] - T * ps[0] - acc[1];
    }
    if (!grad) return;
    if (x < MM && g_alpha) {
        const int32_t q = (int32_t)(x % M);
        double g = 0.0, c = 0.0;
        for (int32_t e = 0; e < ER; ++e) {
            g += gpart[(int64_t)e * MM + x];
            c += npart[(int64_t)e * M + q];
        }
        g_alpha[x] = g - c;
    }
    if (x < M) {
        double s = 0.0;
        for (int32_t e = 0; e < ER; ++e) s += spart[(int64_t)e * M + x];
        if (g_mu) g_mu[x] = s - T;
        if (g_beta) g_beta[x] = -ebacc[x];
    }
}

// ------------------------------------------------------------------ host
hawkes_status run_large_pt(LargeArgs& A, hipStream_t st) {
    const int32_t M = A.M;
    const int64_t MM = (int64_t)M * M;
    const unsigned gM = (unsigned)((M + 255) / 256);
    const size_t lds_agg = (size_t)3 * M * sizeof(double) + 64 * sizeof(double) + (size_t)PT_STAGE_AGG * 16;
    const size_t lds_agg_far = (size_t)2 * M * sizeof(double) + 64 * sizeof(double) + (size_t)PT_STAGE_CHAIN * 16;
    const size_t lds_fwd = (size_t)4 * M * sizeof(double) + PT_BATCH_LDS + (size_t)PT_STAGE * 16 +
                           (size_t)((M + 15) & ~15);
    const size_t lds_rev = (size_t)M * sizeof(double);
    const size_t lds_chain = (size_t)2 * M * sizeof(double) + 64 * sizeof(double) + (size_t)PT_STAGE_CHAIN * 16;
    if (allow_lds((const void*)pt_seg_agg<false, PT_STAGE_AGG>, lds_agg) != HAWKES_OK ||
        allow_lds((const void*)pt_seg_agg<true, PT_STAGE_CHAIN>, lds_agg_far) != HAWKES_OK ||
        allow_lds((const void*)pt_forward<true, false>, lds_fwd) != HAWKES_OK ||
        allow_lds((const void*)pt_forward<false, true>, lds_fwd) != HAWKES_OK ||
        allow_lds((const void*)pt_forward<false, false>, lds_fwd) != HAWKES_OK ||
        allow_lds((const void*)pt_rev_agg, lds_rev) != HAWKES_OK ||
        allow_lds((const void*)pt_chain_part<PT_STAGE_CHAIN>, lds_chain) != HAWKES_OK)
        return HAWKES_EUNSUPPORTED;
    // the gradient's two checkpoint levels hold at most HK_PTCK^2 chunks
    if (A.grad && A.pt_ckr > HK_PTCK) return HAWKES_EUNSUPPORTED;
    auto fill = [&](double* p, int64_t cnt, double v) {
        const int64_t nb = (cnt + 255) / 256;
        hipLaunchKernelGGL(pt_fill, dim3((unsigned)(nb < 65535 ? (nb > 0 ? nb : 1) : 65535)), dim3(256), 0, st, p,
                           cnt, v);
    };
    fill(A.carry, 2 * (int64_t)M, 0.0);
    fill(A.acc, 4, 0.0);
    fill(A.ebacc, M, 0.0);
    if (A.grad) {
        fill(A.gpart, (int64_t)A.ER * MM, 0.0);
        fill(A.spart, (int64_t)A.ER * M, 0.0);
        fill(A.cpart_, (int64_t)A.ER * M, 0.0);
    }
    large_build_index(M, A.alpha, 1, A.csc_ptr, A.csc_cv, st);
    // the per-target engine builds no row index: its buffer holds the decay
    // of every column entry's target
    float* csc_b = reinterpret_cast<float*>(A.csr_cv);
    hipLaunchKernelGGL(pt_csc_beta, dim3(1024), dim3(256), 0, st, M, A.csc_ptr, A.csc_cv, A.beta, csc_b);
    // beta_min and a chunk's flag (near T or not)
    float* flags = A.pt_flags;
    hipLaunchKernelGGL(pt_bmin, dim3(1), dim3(256), 0, st, M, A.beta, flags);
    const int64_t M2 = 2 * (int64_t)M;
    auto chunk_range = [&](int64_t ch, int64_t& c0, int64_t& c1) -> int32_t {
        c0 = ch * A.CH;
        c1 = c0 + A.CH < A.n ? c0 + A.CH : A.n;
        return (int32_t)((c1 - c0 + HK_SEG - 1) / HK_SEG);
    };
    // segment maps and their scan: carry_seg of the chunk from A.carry (its
    // start state), which moves to the chunk's end
    auto agg_scan = [&](int64_t c0, int64_t c1, int32_t nseg) {
        {
            TimedScope ts(2, st);
            hipLaunchKernelGGL(pt_near, dim3(1), dim3(64), 0, st, c1, A.T, A.t, flags);
            const int32_t* nearf = reinterpret_cast<const int32_t*>(flags) + 1;
            hipLaunchKernelGGL((pt_seg_agg<true, PT_STAGE_CHAIN>), dim3(nseg), dim3(64), lds_agg_far, st, c0, c1, M,
                               A.T, A.t, A.marks, A.beta, A.csc_ptr, A.csc_cv, csc_b, A.agg, A.seg_span, A.ebseg,
                               A.seg_part, nearf);
            hipLaunchKernelGGL((pt_seg_agg<false, PT_STAGE_AGG>), dim3(nseg), dim3(64), lds_agg, st, c0, c1, M, A.T,
                               A.t, A.marks, A.beta, A.csc_ptr, A.csc_cv, csc_b, A.agg, A.seg_span, A.ebseg,
                               A.seg_part, nearf);
        }
        TimedScope ts(3, st);
        large_scan(A, nseg, A.beta, st);
    };
    // the carry moved over a chunk (pass 1 of the gradient)
    auto chain = [&](int64_t c0, int64_t c1) {
        const int32_t nw = (int32_t)((c1 - c0 + PT_CHAIN_EV - 1) / PT_CHAIN_EV);
        {
            TimedScope ts(2, st);
            hipLaunchKernelGGL(pt_chain_part<PT_STAGE_CHAIN>, dim3(nw), dim3(64), lds_chain, st, c0, c1, M, A.t,
                               A.marks, A.csc_ptr, A.csc_cv, csc_b, A.agg);
        }
        TimedScope ts(3, st);
        hipLaunchKernelGGL(pt_chain_fold, dim3((unsigned)((M + 63) / 64)), dim3(512), 0, st, c0, c1, M, nw, A.t,
                           A.beta, A.agg, A.carry);
    };
    // the forward pass of a chunk (after agg_scan), then its call-level sums
    auto forward = [&](int64_t c0, int64_t c1, int32_t nseg) {
        {
            TimedScope ts(1, st);
            if (A.grad)
                hipLaunchKernelGGL((pt_forward<true, false>), dim3(nseg), dim3(64), lds_fwd, st, c0, c1, M, A.T, A.t,
                                   A.marks, A.mu, A.beta, A.csc_ptr, A.csc_cv, csc_b, A.carry_seg, A.seg_part,
                                   A.ebseg, A.wv, (float*)nullptr);
            else if (A.lambda_out)
                hipLaunchKernelGGL((pt_forward<false, true>), dim3(nseg), dim3(64), lds_fwd, st, c0, c1, M, A.T, A.t,
                                   A.marks, A.mu, A.beta, A.csc_ptr, A.csc_cv, csc_b, A.carry_seg, A.seg_part,
                                   A.ebseg, (float*)nullptr, A.lambda_out);
            else
                hipLaunchKernelGGL((pt_forward<false, false>), dim3(nseg), dim3(64), lds_fwd, st, c0, c1, M, A.T,
                                   A.t, A.marks, A.mu, A.beta, A.csc_ptr, A.csc_cv, csc_b, A.carry_seg,
                                   A.seg_part, A.ebseg, (float*)nullptr, (float*)nullptr);
        }
        large_chunk_acc_launch(nseg, 4, A.seg_part, A.acc, st);
        hipLaunchKernelGGL(pt_eb_reduce, dim3((unsigned)((M + 63) / 64)), dim3(1024), 0, st, nseg, M, A.ebseg,
                           A.ebacc);
    };
    auto copy = [&](double* dst, const double* src) {
        hipLaunchKernelGGL(pt_copy, dim3((unsigned)((M2 + 255) / 256)), dim3(256), 0, st, dst, src, M2);
    };
    if (!A.grad) {
        // log-likelihood (or intensities) only: one pass in order
        for (int64_t ch = 0; ch < A.nchunks; ++ch) {
            int64_t c0, c1;
            const int32_t nseg = chunk_range(ch, c0, c1);
            agg_scan(c0, c1, nseg);
            forward(c0, c1, nseg);
        }
    } else if (A.n > 0) {
        // Gradient in constant memory (the batches of Algorithm 2, each
        // forward pass followed by its backward pass; here the backward runs
        // right to left, so the chunks are visited in reverse).  Pass 1 only
        // carries the state over the chunks (pt_chain_*) and keeps it at the
        // start of every r-th chunk (one block of r chunks per level-1 slot);
        // pass 2 takes the blocks from the last: it carries the block's chunks
        // again from its slot into the level-2 slots, then per chunk from the last:
        // maps and scan from the chunk's start state, the forward pass (w_i
        // of the chunk's events, the chunk's log-likelihood terms), the
        // reverse scan of the adjoint state and the dense dL/dalpha.
        const int64_t r = A.pt_ckr;
        const int64_t nblk_c = (A.nchunks + r - 1) / r;
        double* ck1 = A.pt_ck;
        double* ck2 = A.pt_ck + (int64_t)HK_PTCK * M2;
        for (int64_t ch = 0; ch < A.nchunks; ++ch) {
            int64_t c0, c1;
            chunk_range(ch, c0, c1);
            if (ch % r == 0) copy(ck1 + (ch / r) * M2, A.carry);
            if (ch + 1 < A.nchunks) chain(c0, c1);
        }
        hipLaunchKernelGGL(pt_seed, dim3(gM), dim3(256), 0, st, M, A.beta, A.achunk);
        for (int64_t b = nblk_c - 1; b >= 0; --b) {
            const int64_t cb0 = b * r, cb1 = cb0 + r < A.nchunks ? cb0 + r : A.nchunks;
            double* starts = r == 1 ? ck1 + b * M2 : ck2;
            if (r > 1) {
                copy(A.carry, ck1 + b * M2);
                for (int64_t ch = cb0; ch < cb1; ++ch) {
                    int64_t c0, c1;
                    chunk_range(ch, c0, c1);
                    copy(ck2 + (ch - cb0) * M2, A.carry);
                    if (ch + 1 < cb1) chain(c0, c1);
                }
            }
            for (int64_t ch = cb1 - 1; ch >= cb0; --ch) {
                int64_t c0, c1;
                const int32_t nseg = chunk_range(ch, c0, c1);
                copy(A.carry, starts + (ch - cb0) * M2);
                agg_scan(c0, c1, nseg);
                forward(c0, c1, nseg);
                const int32_t ngr = (nseg + HK_SG - 1) / HK_SG;
                const int64_t nloc = (int64_t)ngr * M, napp = (int64_t)nseg * M;
                {
                    TimedScope ts(3, st);
                    hipLaunchKernelGGL(pt_rev_agg, dim3(nseg), dim3(64), lds_rev, st, c0, c1, M, A.t, A.marks,
                                       A.beta, A.wv, A.aggA);
                    hipLaunchKernelGGL(pt_rscan_local, dim3((unsigned)((nloc + 255) / 256)), dim3(256), 0, st, c0,
                                       c1, A.n, A.T, nseg, M, A.t, A.beta, A.aggA, A.rcarry_seg, A.rgagg);
                    hipLaunchKernelGGL(pt_rscan_groups, dim3(gM), dim3(256), 0, st, c0, c1, A.n, A.T, nseg, M, A.t,
                                       A.beta, A.rgagg, A.rgcarry, A.achunk);
                    hipLaunchKernelGGL(pt_rscan_apply, dim3((unsigned)((napp + 255) / 256)), dim3(256), 0, st, c0,
                                       c1, A.n, A.T, nseg, M, A.t, A.beta, A.rgcarry, A.rcarry_seg);
                }
                {
                    TimedScope tb(6, st);
                    bucket_chunk(A, c0, c1, nseg, A.wv, 6, st);
                }
                const int32_t spr = (nseg + A.ER - 1) / A.ER;
                const int32_t nbb = A.NB * A.NB;
                const unsigned nblk = A.ER >= 8 ? (unsigned)(nbb * ((A.ER + 7) / 8) * 8)
                                                : (unsigned)(((nbb + 8 / A.ER - 1) / (8 / A.ER)) * 8);
                TimedScope ts(0, st);
                hipLaunchKernelGGL(pt_dense, dim3(nblk), dim3(64 * HK_DWP), 0, st, c0, c1, A.n, A.T, M, A.NB, A.ER,
                                   spr, nseg, A.t, A.beta, A.rcarry_seg, A.rgcarry, A.bk_off, A.bk_base, A.bk_key,
                                   A.bk_t, A.bk_w, A.gpart, A.spart, A.cpart_);
            }
        }
    }
    const int64_t nfin = A.grad ? (MM > M ? MM : M) : 1;
    hipLaunchKernelGGL(pt_final, dim3((unsigned)((nfin + 255) / 256)), dim3(256), 0, st, M, A.ER, A.T, A.mu, A.acc,
                       A.gpart, A.spart, A.cpart_, A.ebacc, A.loglik, A.g_mu, A.g_alpha, A.g_beta,
                       A.grad ? 1 : 0);
    return hipGetLastError() == hipSuccess ? HAWKES_OK : HAWKES_EDEVICE;
}

}  // namespace hk
