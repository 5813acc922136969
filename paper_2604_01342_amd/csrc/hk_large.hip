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
//   forward  one wave per segment replays its events 64 at a time (one per
//            lane).  Each node keeps a lazily decayed record (tau_q, K_q, J_q)
//            in LDS; lambda_i needs only the nonzeros of alpha's row m_i
//            (R = alpha_{m_i,:} . K, eq. 3), read from a CSR copy of alpha,
//            plus the same-batch events found through a per-node lane mask.
//            It writes lambda_i / per-segment float64 partials and, for the
//            gradient, per-event coefficients for the dense kernel.
//   dense    dense dL/dalpha (first term of eq. 9): block (64 rows x 64
//            columns x event range) per wave; column state K in registers,
//            anchored per 64-event batch so that each event costs one
//            multiply-add per column; rows accumulate in float64 LDS.
#include "hk_device.h"
#include "hk_large.h"

namespace hk {

// ------------------------------------------------------------------ setup
__global__ void fill_d(double* p, int64_t n, double v) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

// colsum[q] = sum_p alpha[p][q]; csr_ptr[p+1] = nnz of row p
__global__ void large_colsum_count(int32_t M, const float* __restrict__ alpha, float* __restrict__ colsum,
                                   int32_t* __restrict__ csr_ptr) {
    const int32_t x = blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= M) return;
    double c = 0.0;
    int32_t cnt = 0;
    for (int32_t p = 0; p < M; ++p) c += (double)alpha[(int64_t)p * M + x];
    for (int32_t q = 0; q < M; ++q) cnt += alpha[(int64_t)x * M + q] != 0.0f;
    colsum[x] = (float)c;
    csr_ptr[x + 1] = cnt;
    if (x == 0) csr_ptr[0] = 0;
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

__global__ void large_csr_fill(int32_t M, const float* __restrict__ alpha, const int32_t* __restrict__ csr_ptr,
                               int32_t* __restrict__ csr_col, float* __restrict__ csr_val) {
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    int32_t o = csr_ptr[p];
    for (int32_t q = 0; q < M; ++q) {
        const float a = alpha[(int64_t)p * M + q];
        if (a != 0.0f) { csr_col[o] = q; csr_val[o] = a; ++o; }
    }
}

// ------------------------------------------------------------------ agg
// one wave per segment; LDS: aggK[M], aggJ[M] (float64)
__global__ __launch_bounds__(64) void large_seg_agg(int64_t c0, int64_t c1, int32_t M, const double* __restrict__ t,
                                                    const int32_t* __restrict__ marks, const float* __restrict__ beta,
                                                    double* __restrict__ agg, double* __restrict__ seg_tend) {
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
    for (int64_t base = a; base < b; base += 64) {
        const int64_t i = base + lane;
        if (i < b) {
            const double d = te - t[i];
            const float e = exp_f64arg(-bet * d);
            const int mi = clamp_mark(marks[i], M);
            atomicAdd(&aK[mi], (double)e);
            atomicAdd(&aJ[mi], d * (double)e);
        }
    }
    __syncthreads();
    double* o = agg + (int64_t)s * 2 * M;
    for (int32_t q = lane; q < M; q += 64) { o[q] = aK[q]; o[M + q] = aJ[q]; }
    if (lane == 0) seg_tend[s] = te;
}

// ------------------------------------------------------------------ scan
// thread per node: chain the segment maps; agg[s] is overwritten by the
// carry-in of segment s (state just after the event preceding the segment).
__global__ void large_seg_scan(int64_t c0, int32_t nseg, int32_t M, const double* __restrict__ t,
                               const float* __restrict__ beta, double* __restrict__ agg,
                               const double* __restrict__ seg_tend, double* __restrict__ carry) {
    const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M) return;
    const double bet = (double)beta[0];
    double K = carry[q], J = carry[M + q];
    double tref = c0 > 0 ? t[c0 - 1] : t[c0];
    for (int32_t s = 0; s < nseg; ++s) {
        double* row = agg + (int64_t)s * 2 * M;
        const double aK = row[q], aJ = row[M + q];
        row[q] = K;
        row[M + q] = J;
        const double te = seg_tend[s];
        const double D = te - tref;
        const double ex = exp(-bet * D);
        const double k0 = K;
        K = __builtin_fma(ex, k0, aK);
        J = __builtin_fma(ex, __builtin_fma(D, k0, J), aJ);
        tref = te;
    }
    carry[q] = K;
    carry[M + q] = J;
}

// ------------------------------------------------------------------ forward
// frame end of the 64-event batch starting at global index g (events [g, min(g+64, c1))):
// its first event time, or its last one when the batch is "wide"
__device__ __forceinline__ double batch_frame_end(const double* __restrict__ t, int64_t g, int64_t c1, double bet,
                                                  bool* wide) {
    const int64_t l = g + 64 < c1 ? g + 63 : c1 - 1;
    const double t0 = t[g], tl = t[l];
    *wide = bet * (tl - t0) > HK_WIDE;
    return *wide ? tl : t0;
}

template <bool GRAD, bool INTENS>
__global__ __launch_bounds__(64) void large_forward(int64_t c0, int64_t c1, int32_t M, double T,
                                                    const double* __restrict__ t, const int32_t* __restrict__ marks,
                                                    const float* __restrict__ mu, const float* __restrict__ beta,
                                                    const int32_t* __restrict__ csr_ptr,
                                                    const int32_t* __restrict__ csr_col,
                                                    const float* __restrict__ csr_val,
                                                    const float* __restrict__ colsum,
                                                    const double* __restrict__ carry_seg,
                                                    double* __restrict__ seg_part,
                                                    int32_t* __restrict__ ev_m, float* __restrict__ ev_c,
                                                    float* __restrict__ ev_b, float* __restrict__ ev_w,
                                                    float* __restrict__ ev_ct, float* __restrict__ batch_rho,
                                                    int32_t* __restrict__ batch_wide,
                                                    float* __restrict__ lambda_out) {
    extern __shared__ double lds[];
    double* rtau = lds;                                   // [M]
    uint64_t* rmask = (uint64_t*)(lds + M);               // [M]
    float* rK = (float*)(lds + 2 * M);                    // [M]
    float* rJ = rK + M;                                   // [M]
    __shared__ double tb[64];
    const int32_t s = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t a = c0 + (int64_t)s * HK_SEG;
    const int64_t b = a + HK_SEG < c1 ? a + HK_SEG : c1;
    const double bet = (double)beta[0];
    const float betf = beta[0];
    const double tref = a > 0 ? t[a - 1] : t[a];
    const double* cs = carry_seg + (int64_t)s * 2 * M;
    for (int32_t q = lane; q < M; q += 64) {
        rtau[q] = tref;
        rK[q] = (float)cs[q];
        rJ[q] = (float)cs[M + q];
        rmask[q] = 0ull;
    }
    __syncthreads();
    double logsum = 0.0, comp = 0.0, Esum = 0.0, gb = 0.0;
    for (int64_t base = a; base < b; base += 64) {
        const int64_t i = base + lane;
        const bool valid = i < b;
        const double ti = valid ? t[i] : 0.0;
        const int mi = valid ? clamp_mark(marks[i], M) : 0;
        tb[lane] = ti;
        if (valid) atomicOr((unsigned long long*)&rmask[mi], 1ull << lane);
        __syncthreads();
        float R = 0.0f, Dd = 0.0f;
        if (valid) {
            const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
            const int32_t k0 = csr_ptr[mi], k1 = csr_ptr[mi + 1];
            for (int32_t k = k0; k < k1; ++k) {
                const int32_t q = csr_col[k];
                const float av = csr_val[k];
                const double d = ti - rtau[q];
                const float e = exp_f64arg(-bet * d);
                const float kq = rK[q];
                float Kv = e * kq;
                float Jv = GRAD ? e * __builtin_fmaf((float)d, kq, rJ[q]) : 0.0f;
                uint64_t bits = rmask[q] & below;
                while (bits) {
                    const int j = __builtin_ctzll(bits);
                    bits &= bits - 1;
                    const double dj = ti - tb[j];
                    const float ej = exp_f64arg(-bet * dj);
                    Kv += ej;
                    if (GRAD) Jv = __builtin_fmaf((float)dj, ej, Jv);
                }
                R = __builtin_fmaf(av, Kv, R);
                if (GRAD) Dd = __builtin_fmaf(av, Jv, Dd);
            }
            const float lam = __builtin_fmaf(betf, R, mu[mi]);
            if (INTENS) lambda_out[i] = lam;
            logsum += (double)__logf(lam);
            const double x = bet * (T - ti);
            const float em1 = -expm1f(-(float)x);   // 1 - e^{-x}
            const float cs_m = colsum[mi];
            comp += (double)cs_m * (double)em1;
            if (GRAD) {
                const float w = 1.0f / lam;
                gb += (double)w * ((double)R - bet * (double)Dd);
                const float ex = exp_f64arg(-x);
                Esum += (double)cs_m * (T - ti) * (double)ex;
                const int64_t ii = i - c0;
                ev_m[ii] = mi;
                ev_w[ii] = w;
                ev_ct[ii] = em1;
            }
        }
        if (GRAD) {
            // dense-kernel coefficients for this batch, anchored at its first event
            const int64_t last = base + 63 < b - 1 ? base + 63 : b - 1;
            const double tau = tb[0];
            const bool wide = bet * (tb[last - base] - tau) > HK_WIDE;
            if (valid) {
                const int64_t ii = i - c0;
                const float w = ev_w[ii];
                if (!wide) {
                    const double xl = bet * (ti - tau);
                    ev_c[ii] = betf * w * exp_f64arg(-xl);
                    ev_b[ii] = exp_f64arg(xl);
                } else {
                    ev_c[ii] = betf * w;
                    ev_b[ii] = lane == 0 ? 1.0f : exp_f64arg(-bet * (ti - tb[lane - 1]));
                }
            }
            if (lane == 0) {
                const int64_t bi = (base - c0) / 64;
                batch_wide[bi] = wide ? 1 : 0;
                float rho = 1.0f;
                if (base - 64 >= c0) {
                    bool pw;
                    const double fe = batch_frame_end(t, base - 64, c1, bet, &pw);
                    rho = exp_f64arg(-bet * (tau - fe));
                }
                batch_rho[bi] = rho;
            }
        }
        __syncthreads();
        // lazy record update, one leader lane per node, events in index order
        if (valid) {
            uint64_t grp = rmask[mi];
            if (__builtin_ctzll(grp) == lane) {
                double tq = rtau[mi];
                float kq = rK[mi], jq = rJ[mi];
                while (grp) {
                    const int j = __builtin_ctzll(grp);
                    grp &= grp - 1;
                    const double d = tb[j] - tq;
                    const float e = exp_f64arg(-bet * d);
                    jq = e * __builtin_fmaf((float)d, kq, jq);
                    kq = __builtin_fmaf(e, kq, 1.0f);
                    tq = tb[j];
                }
                rtau[mi] = tq;
                rK[mi] = kq;
                rJ[mi] = jq;
            }
        }
        __syncthreads();
        if (valid) rmask[mi] = 0ull;
        __syncthreads();
    }
    // deterministic wave reduction of the float64 partials
    for (int off = 32; off > 0; off >>= 1) {
        logsum += __shfl_down(logsum, off, 64);
        comp += __shfl_down(comp, off, 64);
        Esum += __shfl_down(Esum, off, 64);
        gb += __shfl_down(gb, off, 64);
    }
    if (lane == 0) {
        double* o = seg_part + (int64_t)s * 4;
        o[0] = logsum; o[1] = comp; o[2] = Esum; o[3] = gb;
    }
}

// acc[k] += sum over segments of seg_part[s][k], segments in order
__global__ void large_chunk_acc(int32_t nseg, const double* __restrict__ seg_part, double* __restrict__ acc) {
    const int k = threadIdx.x;
    if (k >= 4) return;
    double v = 0.0;
    for (int32_t s = 0; s < nseg; ++s) v += seg_part[(int64_t)s * 4 + k];
    acc[k] += v;
}

// ------------------------------------------------------------------ dense dL/dalpha
// block = (row block rb, column slab sb, event range er); one wave.
// LDS G[64][64] float64 accumulates beta * sum_i w_i K_q(t_i) for rows of the
// block; lane c owns column s0 + c and its anchored state Khat.
__global__ __launch_bounds__(64) void large_dense(int64_t c0, int64_t c1, int32_t M, int32_t NB, int32_t ER,
                                                  int32_t segs_per_range, const double* __restrict__ t,
                                                  const float* __restrict__ beta,
                                                  const double* __restrict__ carry_seg,
                                                  const int32_t* __restrict__ ev_m, const float* __restrict__ ev_c,
                                                  const float* __restrict__ ev_b, const float* __restrict__ ev_w,
                                                  const float* __restrict__ ev_ct, const float* __restrict__ batch_rho,
                                                  const int32_t* __restrict__ batch_wide,
                                                  double* __restrict__ gpart, double* __restrict__ spart,
                                                  double* __restrict__ cpart) {
    __shared__ double G[HK_RB * HK_SLAB];
    const int lane = threadIdx.x;
    const int32_t blk = blockIdx.x;
    const int32_t er = blk % ER;
    const int32_t sb = (blk / ER) % NB;
    const int32_t rb = blk / (ER * NB);
    const int32_t r0 = rb * HK_RB, s0 = sb * HK_SLAB;
    const int64_t a = c0 + (int64_t)er * segs_per_range * HK_SEG;
    if (a >= c1) return;
    const int64_t bnd = a + (int64_t)segs_per_range * HK_SEG;
    const int64_t b = bnd < c1 ? bnd : c1;
    const int32_t col = s0 + lane;
    // load this block's accumulators (accumulated over chunks)
    double* gp = gpart + (int64_t)er * M * M;
    for (int r = 0; r < HK_RB; ++r) {
        const int32_t row = r0 + r;
        G[r * HK_SLAB + lane] = (row < M && col < M) ? gp[(int64_t)row * M + col] : 0.0;
    }
    const double bet = (double)beta[0];
    // carry-in at the event before the range, moved to the first batch frame
    const int32_t seg = (int32_t)((a - c0) / HK_SEG);
    const double tref = a > 0 ? t[a - 1] : t[a];
    double Kh = col < M ? carry_seg[(int64_t)seg * 2 * M + col] : 0.0;
    Kh *= (double)exp_f64arg(-bet * (t[a] - tref));
    double Sacc = 0.0, Cacc = 0.0;
    const bool diag_owner = rb == 0;
    __syncthreads();
    for (int64_t base = a; base < b; base += 64) {
        const int64_t bi = (base - c0) / 64;
        const int nb = (int)(b - base < 64 ? b - base : 64);
        const int64_t ii = base - c0 + lane;
        const int mi = lane < nb ? ev_m[ii] : -1;
        const float ci = lane < nb ? ev_c[ii] : 0.0f;
        const float bi_ = lane < nb ? ev_b[ii] : 0.0f;
        const float wi = lane < nb ? ev_w[ii] : 0.0f;
        const float cti = lane < nb ? ev_ct[ii] : 0.0f;
        const int wide = uniform(batch_wide[bi]);
        if (base != a) Kh *= (double)batch_rho[bi];
        const bool own = mi >= r0 && mi < r0 + HK_RB;
        const bool sl = mi >= s0 && mi < s0 + HK_SLAB;
        if (!wide) {
            uint64_t mo = __ballot(own), ms = __ballot(sl);
            uint64_t all = mo | ms;
            while (all) {
                const int k = __builtin_ctzll(all);
                all &= all - 1;
                const int mk = __shfl(mi, k, 64);
                if ((mo >> k) & 1ull) {
                    const double ck = (double)__shfl(ci, k, 64);
                    atomicAdd(&G[(mk - r0) * HK_SLAB + lane], ck * Kh);
                }
                if ((ms >> k) & 1ull) {
                    const float bk = __shfl(bi_, k, 64);
                    const float wk = __shfl(wi, k, 64);
                    const float ctk = __shfl(cti, k, 64);
                    if (lane == mk - s0) {
                        Kh += (double)bk;
                        Sacc += (double)wk;
                        Cacc += (double)ctk;
                    }
                }
            }
        } else {
            for (int k = 0; k < nb; ++k) {
                const float rk = __shfl(bi_, k, 64);
                if (k > 0) Kh *= (double)rk;
                const int mk = __shfl(mi, k, 64);
                const bool ok = mk >= r0 && mk < r0 + HK_RB;
                const bool sk = mk >= s0 && mk < s0 + HK_SLAB;
                if (ok) {
                    const double ck = (double)__shfl(ci, k, 64);
                    atomicAdd(&G[(mk - r0) * HK_SLAB + lane], ck * Kh);
                }
                const float wk = __shfl(wi, k, 64);
                const float ctk = __shfl(cti, k, 64);
                if (sk && lane == mk - s0) {
                    Kh += 1.0;
                    Sacc += (double)wk;
                    Cacc += (double)ctk;
                }
            }
        }
    }
    __syncthreads();
    for (int r = 0; r < HK_RB; ++r) {
        const int32_t row = r0 + r;
        if (row < M && col < M) gp[(int64_t)row * M + col] = G[r * HK_SLAB + lane];
    }
    if (diag_owner && col < M) {
        spart[(int64_t)er * M + col] += Sacc;
        cpart[(int64_t)er * M + col] += Cacc;
    }
}

// ------------------------------------------------------------------ finalize
__global__ void large_final(int32_t M, int32_t ER, double T, const float* __restrict__ mu,
                            const double* __restrict__ acc, const double* __restrict__ gpart,
                            const double* __restrict__ spart, const double* __restrict__ cpart,
                            double* __restrict__ loglik, double* __restrict__ g_mu, double* __restrict__ g_alpha,
                            double* __restrict__ g_beta, int grad) {
    const int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t MM = (int64_t)M * M;
    if (x == 0) {
        double musum = 0.0;
        for (int32_t p = 0; p < M; ++p) musum += (double)mu[p];
        loglik[0] = acc[0] - T * musum - acc[1];
        if (grad && g_beta) g_beta[0] = acc[3] - acc[2];
    }
    if (!grad) return;
    if (x < MM && g_alpha) {
        const int32_t q = (int32_t)(x % M);
        double g = 0.0, c = 0.0;
        for (int32_t e = 0; e < ER; ++e) {
            g += gpart[(int64_t)e * MM + x];
            c += cpart[(int64_t)e * M + q];
        }
        g_alpha[x] = g - c;
    }
    if (x < M && g_mu) {
        double s = 0.0;
        for (int32_t e = 0; e < ER; ++e) s += spart[(int64_t)e * M + x];
        g_mu[x] = s - T;
    }
}

// ------------------------------------------------------------------ host
size_t large_layout(LargeArgs& A, const hawkes_problem* p, bool grad, void* ws, size_t ws_bytes) {
    A.n = p->n;
    A.M = p->m;
    A.per_target = p->beta_mode == HAWKES_BETA_PER_TARGET;
    A.T = p->T;
    const int lg = p->chunk_log2 ? p->chunk_log2 : 20;
    A.CH = (int64_t)1 << lg;
    A.nchunks = (A.n + A.CH - 1) / A.CH;
    A.nseg = (int32_t)((A.CH + HK_SEG - 1) / HK_SEG);
    A.NB = (A.M + 63) / 64;
    int32_t er = (int32_t)((2048 + A.NB * A.NB - 1) / (A.NB * A.NB));
    if (er < 1) er = 1;
    if (er > A.nseg) er = A.nseg;
    A.ER = er;
    A.grad = grad;
    const int64_t M = A.M, MM = M * M;
    Carve c(ws, ws_bytes);
    A.csr_ptr = c.take<int32_t>(M + 1);
    A.csr_col = c.take<int32_t>(MM);
    A.csr_val = c.take<float>(MM);
    A.colsum = c.take<float>(M);
    A.agg = c.take<double>((size_t)A.nseg * 2 * M);
    A.seg_tend = c.take<double>(A.nseg);
    A.carry = c.take<double>(2 * M);
    A.carry_t = c.take<double>(1);
    A.seg_part = c.take<double>((size_t)A.nseg * 4);
    A.acc = c.take<double>(4);
    A.ll_scratch = c.take<double>(1);
    if (grad) {
        A.ev_m = c.take<int32_t>(A.CH);
        A.ev_c = c.take<float>(A.CH);
        A.ev_b = c.take<float>(A.CH);
        A.ev_w = c.take<float>(A.CH);
        A.ev_ct = c.take<float>(A.CH);
        A.batch_rho = c.take<float>(A.CH / 64 + 1);
        A.batch_wide = c.take<int32_t>(A.CH / 64 + 1);
        A.gpart = c.take<double>((size_t)A.ER * MM);
        A.spart = c.take<double>((size_t)A.ER * M);
        A.cpart_ = c.take<double>((size_t)A.ER * M);
    }
    return c.off + 256;
}

hawkes_status run_large(LargeArgs& A, hipStream_t st) {
    if (A.per_target) return HAWKES_EUNSUPPORTED;
    const int32_t M = A.M;
    const int64_t MM = (int64_t)M * M;
    const unsigned gM = (unsigned)((M + 255) / 256);
    // zero the carried state and accumulators
    hipLaunchKernelGGL(fill_d, dim3(1), dim3(256), 0, st, A.carry, (int64_t)2 * M, 0.0);
    hipLaunchKernelGGL(fill_d, dim3(1), dim3(64), 0, st, A.acc, (int64_t)4, 0.0);
    if (A.grad) {
        const int64_t ng = (int64_t)A.ER * MM;
        hipLaunchKernelGGL(fill_d, dim3((unsigned)((ng + 255) / 256 < 65535 ? (ng + 255) / 256 : 65535)),
                           dim3(256), 0, st, A.gpart, ng, 0.0);
        hipLaunchKernelGGL(fill_d, dim3(64), dim3(256), 0, st, A.spart, (int64_t)A.ER * M, 0.0);
        hipLaunchKernelGGL(fill_d, dim3(64), dim3(256), 0, st, A.cpart_, (int64_t)A.ER * M, 0.0);
    }
    hipLaunchKernelGGL(large_colsum_count, dim3(gM), dim3(256), 0, st, M, A.alpha, A.colsum, A.csr_ptr);
    hipLaunchKernelGGL(large_csr_scan, dim3(1), dim3(1024), 0, st, M, A.csr_ptr);
    hipLaunchKernelGGL(large_csr_fill, dim3(gM), dim3(256), 0, st, M, A.alpha, A.csr_ptr, A.csr_col, A.csr_val);
    const size_t lds_agg = (size_t)2 * M * sizeof(double);
    const size_t lds_fwd = (size_t)M * (sizeof(double) + sizeof(uint64_t) + 2 * sizeof(float));
    if (lds_agg > 160 * 1024 || lds_fwd > 150 * 1024) return HAWKES_EUNSUPPORTED;
    for (int64_t ch = 0; ch < A.nchunks; ++ch) {
        const int64_t c0 = ch * A.CH;
        const int64_t c1 = c0 + A.CH < A.n ? c0 + A.CH : A.n;
        const int32_t nseg = (int32_t)((c1 - c0 + HK_SEG - 1) / HK_SEG);
        {
            TimedScope ts(2, st);
            hipLaunchKernelGGL(large_seg_agg, dim3(nseg), dim3(64), lds_agg, st, c0, c1, M, A.t, A.marks, A.beta,
                               A.agg, A.seg_tend);
        }
        {
            TimedScope ts(3, st);
            hipLaunchKernelGGL(large_seg_scan, dim3(gM), dim3(256), 0, st, c0, nseg, M, A.t, A.beta, A.agg,
                               A.seg_tend, A.carry);
        }
        TimedScope* tf = new TimedScope(1, st);
        if (A.grad)
            hipLaunchKernelGGL((large_forward<true, false>), dim3(nseg), dim3(64), lds_fwd, st, c0, c1, M, A.T,
                               A.t, A.marks, A.mu, A.beta, A.csr_ptr, A.csr_col, A.csr_val, A.colsum, A.agg,
                               A.seg_part, A.ev_m, A.ev_c, A.ev_b, A.ev_w, A.ev_ct, A.batch_rho, A.batch_wide,
                               (float*)nullptr);
        else if (A.lambda_out)
            hipLaunchKernelGGL((large_forward<false, true>), dim3(nseg), dim3(64), lds_fwd, st, c0, c1, M, A.T,
                               A.t, A.marks, A.mu, A.beta, A.csr_ptr, A.csr_col, A.csr_val, A.colsum, A.agg,
                               A.seg_part, A.ev_m, A.ev_c, A.ev_b, A.ev_w, A.ev_ct, A.batch_rho, A.batch_wide,
                               A.lambda_out);
        else
            hipLaunchKernelGGL((large_forward<false, false>), dim3(nseg), dim3(64), lds_fwd, st, c0, c1, M, A.T,
                               A.t, A.marks, A.mu, A.beta, A.csr_ptr, A.csr_col, A.csr_val, A.colsum, A.agg,
                               A.seg_part, A.ev_m, A.ev_c, A.ev_b, A.ev_w, A.ev_ct, A.batch_rho, A.batch_wide,
                               (float*)nullptr);
        delete tf;
        hipLaunchKernelGGL(large_chunk_acc, dim3(1), dim3(64), 0, st, nseg, A.seg_part, A.acc);
        if (A.grad) {
            int32_t spr = (nseg + A.ER - 1) / A.ER;
            const unsigned nblk = (unsigned)(A.NB * A.NB * A.ER);
            TimedScope ts(0, st);
            hipLaunchKernelGGL(large_dense, dim3(nblk), dim3(64), 0, st, c0, c1, M, A.NB, A.ER, spr, A.t, A.beta,
                               A.agg, A.ev_m, A.ev_c, A.ev_b, A.ev_w, A.ev_ct, A.batch_rho, A.batch_wide,
                               A.gpart, A.spart, A.cpart_);
        }
    }
    const int64_t nfin = A.grad ? (MM > M ? MM : M) : 1;
    hipLaunchKernelGGL(large_final, dim3((unsigned)((nfin + 255) / 256)), dim3(256), 0, st, M, A.ER, A.T, A.mu,
                       A.acc, A.gpart, A.spart, A.cpart_, A.loglik, A.g_mu, A.g_alpha, A.g_beta, A.grad ? 1 : 0);
    return hipGetLastError() == hipSuccess ? HAWKES_OK : HAWKES_EDEVICE;
}

}  // namespace hk
