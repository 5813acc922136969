// Sequential baseline and device-side input validation.
#include "hk_device.h"
#include "hk_large.h"

namespace hk {

// ------------------------------------------------------------------ sequential baseline
// The recurrence of eq. 4 (and eqs. 11-12 for the gradient) taken event by
// event in index order by one workgroup: thread x owns nodes x, x+1024, ...
// of the source-indexed states K_q, J_q (float64).  Each event costs a
// block-wide dot product with alpha's row m_i and a row update of the float64
// gradient accumulator in global memory.  No parallelism over events.
#define SEQ_NT 1024
#define SEQ_NQ 4   // nodes per thread: M <= 4096

__global__ __launch_bounds__(SEQ_NT) void seq_kernel(int64_t n, int32_t M, double T, const double* __restrict__ t,
                                                     const int32_t* __restrict__ marks, const float* __restrict__ mu,
                                                     const float* __restrict__ alpha, const float* __restrict__ beta,
                                                     double* __restrict__ gacc, double* __restrict__ loglik,
                                                     double* __restrict__ g_mu, double* __restrict__ g_alpha,
                                                     double* __restrict__ g_beta) {
    __shared__ double red[2][SEQ_NT / 64];
    __shared__ float colsum_s[SEQ_NT * SEQ_NQ];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wid = tid >> 6;
    const double bet = (double)beta[0];
    double K[SEQ_NQ], J[SEQ_NQ], S[SEQ_NQ], C[SEQ_NQ];
    for (int k = 0; k < SEQ_NQ; ++k) {
        K[k] = 0.0; J[k] = 0.0; S[k] = 0.0; C[k] = 0.0;
        const int32_t q = tid + k * SEQ_NT;
        if (q < M) {
            double c = 0.0;
            for (int32_t p = 0; p < M; ++p) c += (double)alpha[(int64_t)p * M + q];
            colsum_s[q] = (float)c;
            for (int32_t r = 0; r < M; ++r) gacc[(int64_t)r * M + q] = 0.0;
        }
    }
    __syncthreads();
    double logsum = 0.0, comp = 0.0, Esum = 0.0, gb = 0.0;
    int mprev = -1;
    double tprev = n > 0 ? t[0] : 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double ti = t[i];
        const double d = ti - tprev;
        const double s = exp(-bet * d);
        const int p = clamp_mark(marks[i], M);
        double r = 0.0, dd = 0.0;
        for (int k = 0; k < SEQ_NQ; ++k) {
            const int32_t q = tid + k * SEQ_NT;
            if (q < M) {
                K[k] = s * (K[k] + (q == mprev ? 1.0 : 0.0));
                J[k] = __builtin_fma(s, J[k], d * K[k]);
                const double a = (double)alpha[(int64_t)p * M + q];
                r = __builtin_fma(a, K[k], r);
                dd = __builtin_fma(a, J[k], dd);
            }
        }
        for (int off = 32; off > 0; off >>= 1) {
            r += __shfl_down(r, off, 64);
            dd += __shfl_down(dd, off, 64);
        }
        if (lane == 0) { red[0][wid] = r; red[1][wid] = dd; }
        __syncthreads();
        double R = 0.0, D = 0.0;
        for (int w = 0; w < SEQ_NT / 64; ++w) { R += red[0][w]; D += red[1][w]; }
        __syncthreads();
        const double lam = (double)mu[p] + bet * R;
        const double w = 1.0 / lam;
        const double x = bet * (T - ti);
        const double ex = exp(-x);
        for (int k = 0; k < SEQ_NQ; ++k) {
            const int32_t q = tid + k * SEQ_NT;
            if (q < M) {
                gacc[(int64_t)p * M + q] += bet * w * K[k];
                if (q == p) { S[k] += w; C[k] += 1.0 - ex; }
            }
        }
        if (tid == 0) {
            logsum += log(lam);
            comp += (double)colsum_s[p] * (1.0 - ex);
            Esum += (double)colsum_s[p] * (T - ti) * ex;
            gb += w * (R - bet * D);
        }
        mprev = p;
        tprev = ti;
    }
    __syncthreads();
    if (tid == 0) {
        double musum = 0.0;
        for (int32_t q = 0; q < M; ++q) musum += (double)mu[q];
        loglik[0] = logsum - T * musum - comp;
        if (g_beta) g_beta[0] = gb - Esum;
    }
    for (int k = 0; k < SEQ_NQ; ++k) {
        const int32_t q = tid + k * SEQ_NT;
        if (q < M) {
            if (g_mu) g_mu[q] = S[k] - T;
            if (g_alpha)
                for (int32_t r = 0; r < M; ++r) g_alpha[(int64_t)r * M + q] = gacc[(int64_t)r * M + q] - C[k];
        }
    }
}

size_t seq_workspace_bytes(const hawkes_problem* p) {
    return (size_t)p->m * p->m * sizeof(double) + 512;
}

hawkes_status run_sequential(const hawkes_problem* p, const double* t, const int32_t* marks, const float* mu,
                             const float* alpha, const float* beta, double* loglik, double* g_mu,
                             double* g_alpha, double* g_beta, void* ws, hipStream_t st) {
    if (p->m > SEQ_NT * SEQ_NQ) return HAWKES_EUNSUPPORTED;
    hipLaunchKernelGGL(seq_kernel, dim3(1), dim3(SEQ_NT), 0, st, p->n, p->m, p->T, t, marks, mu, alpha, beta,
                       (double*)ws, loglik, g_mu, g_alpha, g_beta);
    return hipGetLastError() == hipSuccess ? HAWKES_OK : HAWKES_EDEVICE;
}

// ------------------------------------------------------------------ input checks
__global__ void check_zero(int32_t* s) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *s = 0;
}

__global__ void check_events(int64_t n, int32_t M, double T, const double* __restrict__ t,
                             const int32_t* __restrict__ marks, int32_t* status) {
    int32_t bad = 0;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double ti = t[i];
        if (i > 0 && !(ti >= t[i - 1])) bad |= 1;
        const int32_t m = marks[i];
        if (m < 0 || m >= M) bad |= 2;
        if (!(ti >= 0.0) || !(ti <= T)) bad |= 4;
    }
    if (bad) atomicOr(status, bad);
}

__global__ void check_params(int32_t M, int32_t K, int32_t nbeta, const float* __restrict__ mu,
                             const float* __restrict__ alpha, const float* __restrict__ beta, int32_t* status) {
    int32_t bad = 0;
    const int64_t MM = (int64_t)K * M * M;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < MM; i += (int64_t)gridDim.x * blockDim.x) {
        const float a = alpha[i];
        if (!(a >= 0.0f) || !isfinite(a)) bad |= 16;
        if (i < M) {
            const float m = mu[i];
            if (!(m > 0.0f) || !isfinite(m)) bad |= 8;
        }
        if (i < nbeta) {
            const float b = beta[i];
            if (!(b > 0.0f) || !isfinite(b)) bad |= 32;
        }
    }
    if (bad) atomicOr(status, bad);
}

hawkes_status run_check_inputs(const hawkes_problem* p, const double* t, const int32_t* marks, const float* mu,
                               const float* alpha, const float* beta, int32_t* status_out, hipStream_t st) {
    hipLaunchKernelGGL(check_zero, dim3(1), dim3(64), 0, st, status_out);
    if (p->n > 0)
        hipLaunchKernelGGL(check_events, dim3(1024), dim3(256), 0, st, p->n, p->m, p->T, t, marks, status_out);
    const int32_t nb = p->beta_mode == HAWKES_BETA_PER_TARGET ? p->m : p->k;
    hipLaunchKernelGGL(check_params, dim3(256), dim3(256), 0, st, p->m, p->k, nb, mu, alpha, beta, status_out);
    return hipGetLastError() == hipSuccess ? HAWKES_OK : HAWKES_EDEVICE;
}

}  // namespace hk
