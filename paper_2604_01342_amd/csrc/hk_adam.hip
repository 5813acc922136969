// Projected Adam step on the training objective of section "Background" (the
// per-event negative log-likelihood plus the hinge-l1 penalty on alpha's
// off-diagonal entries below h), fused after a log-likelihood + gradient
// evaluation: the maximum-likelihood loop the paper trains with (Algorithm 1:
// forward pass, backward pass, optimizer step).  Everything is stream-ordered and reads no
// device memory from the host, so a whole step can be captured in a HIP graph
// and replayed: the step counter used for the bias corrections lives in the
// device state and is advanced by a kernel.
#include <hip/hip_runtime.h>
#include <math.h>
#include "hk_internal.h"
#include "../../include/hawkes.h"

namespace hk {

// state layout (float64 header, then float32 moments):
//   [0] step count, [1..31] unused, then m and v for mu[M], alpha[K*M*M], beta[nb]
struct AdamLayout {
    int64_t M, MM, nb, np;   // MM: alpha entries over all K kernels
    size_t bytes;
};

static AdamLayout adam_layout(const hawkes_problem* p) {
    AdamLayout L;
    L.M = p->m;
    L.MM = (int64_t)p->k * p->m * p->m;
    L.nb = p->beta_mode == HAWKES_BETA_PER_TARGET ? p->m : p->k;
    L.np = L.M + L.MM + L.nb;
    L.bytes = 256 + (size_t)L.np * 2 * sizeof(float);
    return L;
}

__global__ void adam_zero(float* s, int64_t n, double* head) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        s[i] = 0.0f;
    if (blockIdx.x == 0 && threadIdx.x < 32) head[threadIdx.x] = 0.0;
}

__global__ void adam_tick(double* head) {
    if (threadIdx.x == 0 && blockIdx.x == 0) head[0] += 1.0;
}

// one thread per parameter; index space [mu | alpha | beta]
__global__ void adam_update(int64_t M, int64_t MM, int64_t nb, double scale, hawkes_adam cfg,
                            const double* __restrict__ head, float* __restrict__ mom, float* __restrict__ mu,
                            float* __restrict__ alpha, float* __restrict__ beta, const double* __restrict__ g_mu,
                            const double* __restrict__ g_alpha, const double* __restrict__ g_beta) {
    const int64_t np = M + MM + nb;
    const double step = head[0];
    const double c1 = 1.0 - pow((double)cfg.beta1, step);
    const double c2 = 1.0 - pow((double)cfg.beta2, step);
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
        float* x;
        double g, lo;
        bool lg;   // step on log x
        if (i < M) {
            x = mu + i; g = g_mu[i]; lo = cfg.floor_mu; lg = (cfg.flags & HAWKES_ADAM_LOG_MU) != 0;
        } else if (i < M + MM) {
            x = alpha + (i - M); g = g_alpha[i - M]; lo = 0.0; lg = (cfg.flags & HAWKES_ADAM_LOG_ALPHA) != 0;
        } else {
            x = beta + (i - M - MM); g = g_beta[i - M - MM]; lo = cfg.floor_beta;
            lg = (cfg.flags & HAWKES_ADAM_LOG_BETA) != 0;
        }
        // gradient of the loss -L / scale, plus the penalty's lambda1 on the
        // off-diagonal alpha entries below the hinge point (float32 compare)
        double gl = -g / scale;
        if (i >= M && i < M + MM) {
            const int64_t a = (i - M) % (M * M);   // entry within its kernel's matrix
            if (a / M != a % M && *x < cfg.h) gl += (double)cfg.lambda1;
        }
        const double x0 = (double)*x;
        if (lg) gl *= x0;   // d loss / d log x
        float* m = mom + i;
        float* v = mom + np + i;
        const double mn = cfg.beta1 * (double)*m + (1.0 - cfg.beta1) * gl;
        const double vn = cfg.beta2 * (double)*v + (1.0 - cfg.beta2) * gl * gl;
        *m = (float)mn;
        *v = (float)vn;
        const double stp = cfg.lr * (mn / c1) / (sqrt(vn / c2) + cfg.eps);
        double xn = lg ? x0 * exp(-stp) : x0 - stp;
        if (xn < lo) xn = lo;
        *x = (float)xn;
    }
}

}  // namespace hk

using namespace hk;

extern "C" {

size_t hawkes_adam_state_bytes(const hawkes_problem* p) {
    if (!p || p->m < 1 || p->k < 1 || p->k > HAWKES_MAX_KERNELS) return 0;
    return adam_layout(p).bytes;
}

hawkes_status hawkes_adam_init(const hawkes_problem* p, void* state, size_t state_bytes, hipStream_t stream) {
    if (!p || p->m < 1 || p->k < 1 || p->k > HAWKES_MAX_KERNELS || !state) return HAWKES_EINVAL;
    const AdamLayout L = adam_layout(p);
    if (state_bytes < L.bytes) return HAWKES_EWORKSPACE;
    float* mom = (float*)((char*)state + 256);
    hipLaunchKernelGGL(adam_zero, dim3(256), dim3(256), 0, stream, mom, L.np * 2, (double*)state);
    return hipGetLastError() == hipSuccess ? HAWKES_OK : HAWKES_EDEVICE;
}

hawkes_status hawkes_adam_step(const hawkes_problem* p, const double* t, const int32_t* marks, float* mu,
                               float* alpha, float* beta, const hawkes_adam* cfg, void* state, size_t state_bytes,
                               double* loglik, double* g_mu, double* g_alpha, double* g_beta, void* workspace,
                               size_t workspace_bytes, hipStream_t stream) {
    if (!p || !cfg || !state || !mu || !alpha || !beta || !loglik || !g_mu || !g_alpha || !g_beta)
        return HAWKES_EINVAL;
    if (!(cfg->lr > 0.0f) || !(cfg->beta1 >= 0.0f && cfg->beta1 < 1.0f) ||
        !(cfg->beta2 >= 0.0f && cfg->beta2 < 1.0f) || !(cfg->eps > 0.0f) || !(cfg->floor_mu >= 0.0f) ||
        !(cfg->floor_beta > 0.0f) || !(cfg->lambda1 >= 0.0f) || (cfg->lambda1 > 0.0f && !(cfg->h > 0.0f)) ||
        (cfg->flags & ~(HAWKES_ADAM_LOG_MU | HAWKES_ADAM_LOG_BETA | HAWKES_ADAM_LOG_ALPHA)) != 0)
        return HAWKES_EINVAL;
    const AdamLayout L = adam_layout(p);
    if (state_bytes < L.bytes) return HAWKES_EWORKSPACE;
    hawkes_status s = hawkes_loglik_grad(p, t, marks, mu, alpha, beta, loglik, g_mu, g_alpha, g_beta, workspace,
                                         workspace_bytes, stream);
    if (s != HAWKES_OK) return s;
    double* head = (double*)state;
    float* mom = (float*)((char*)state + 256);
    hipLaunchKernelGGL(adam_tick, dim3(1), dim3(64), 0, stream, head);
    const int64_t nblk = (L.np + 255) / 256;
    hipLaunchKernelGGL(adam_update, dim3((unsigned)(nblk < 4096 ? nblk : 4096)), dim3(256), 0, stream, L.M, L.MM,
                       L.nb, (double)(p->n > 0 ? p->n : 1), *cfg, head, mom, mu, alpha, beta, g_mu, g_alpha, g_beta);
    return hipGetLastError() == hipSuccess ? HAWKES_OK : HAWKES_EDEVICE;
}

}  // extern "C"
