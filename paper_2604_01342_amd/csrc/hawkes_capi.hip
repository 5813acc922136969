// C ABI of the library: argument checks, workspace carving, engine dispatch.
// Every entry point returns a hawkes_status and never throws.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>
#include <mutex>
#include <vector>
#include "hk_device.h"
#include "hk_internal.h"
#include "hk_large.h"

using namespace hk;

namespace hk {

static std::mutex g_tuning_mu;
static hawkes_tuning g_tuning = {0, 0, 0, 0};

hawkes_tuning tuning_snapshot() {
    std::lock_guard<std::mutex> g(g_tuning_mu);
    return g_tuning;
}

static int32_t pow2_at_least(int32_t m) {
    int32_t p = 1;
    while (p < m) p <<= 1;
    return p;
}

// single-sequence descriptor written on the device so calls stay graph-capturable
__global__ void write_single_desc(int64_t n, int32_t m, double T, int64_t* ev_off, int32_t* m_s,
                                  double* T_s) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        ev_off[0] = 0;
        ev_off[1] = n;
        m_s[0] = m;
        T_s[0] = T;
    }
}

size_t small_layout(SmallArgs& A, int32_t S, int64_t n_total, int32_t max_m, bool grad, void* ws,
                    size_t ws_bytes, bool single) {
    A.S = S;
    A.MP = pow2_at_least(max_m < 1 ? 1 : max_m);
    // events per item: at least 16; for long inputs grow it so the item count
    // (and so the workspace) stays bounded: the workspace does not grow with n
    // beyond 64Ki items per sequence block.
    int64_t L = 16;
    const int64_t target_items = single ? 65536 : 262144;
    while (L < 4096 && n_total / L > target_items) L <<= 1;
    if (n_total / L > target_items) L = (n_total + target_items - 1) / target_items;
    // a tuned item length replaces this one unless it breaks the item bound
    const hawkes_tuning tu = tuning_snapshot();
    if (tu.item_log2 > 0) {
        const int64_t Lt = (int64_t)1 << tu.item_log2;
        if (Lt >= L || n_total / Lt <= target_items) L = Lt;
    }
    A.L = (int32_t)L;
    A.n_total = n_total;
    A.n_items_cap = n_total / L + S + 1;
    A.n_chunks_cap = A.n_items_cap / HK_RCH + S + 1;
    A.grad = grad;
    const int64_t tiles = (A.n_items_cap + 63) / 64;
    const int32_t PW = grad ? 4 + 2 * A.MP + A.MP * A.MP : 2;
    Carve c(ws, ws_bytes);
    if (single) {
        A.ev_off = c.take<int64_t>(2);
        A.m_s = c.take<int32_t>(1);
        A.T_s = c.take<double>(1);
    }
    A.item_off = c.take<int64_t>(S + 1);
    A.chunk_off = c.take<int64_t>(S + 1);
    A.mu_off = c.take<int64_t>(S + 1);
    A.a_off = c.take<int64_t>(S + 1);
    A.item_pref = c.take<double>((size_t)A.n_items_cap * (2 + 2 * A.MP));
    A.tile_agg = c.take<double>((size_t)tiles * (2 + 2 * A.MP));
    A.tile_carry = c.take<double>((size_t)tiles * 2 * A.MP);
    A.part = c.take<double>((size_t)A.n_items_cap * PW);
    A.cpart = c.take<double>((size_t)A.n_chunks_cap * PW);
    A.ll_scratch = c.take<double>(1);
    return c.off + 256;
}

}  // namespace hk

static bool problem_ok(const hawkes_problem* p) {
    if (!p) return false;
    if (p->n < 0 || p->m < 1 || p->k < 1 || p->k > HAWKES_MAX_KERNELS) return false;
    if (p->beta_mode != HAWKES_BETA_SHARED && p->beta_mode != HAWKES_BETA_PER_TARGET) return false;
    // a decay per target node is one kernel (beta[m])
    if (p->beta_mode == HAWKES_BETA_PER_TARGET && p->k != 1) return false;
    if (!(p->T >= 0.0) || !isfinite(p->T)) return false;
    if (p->chunk_log2 != 0 && (p->chunk_log2 < 12 || p->chunk_log2 > 26)) return false;
    if ((int64_t)p->m * p->m > ((int64_t)1 << 31)) return false;
    return true;
}

// ---------------------------------------------------------------- fixed scratch
// The workspace of hawkes_loglik_grad_noalloc: one array per device, part of
// the library's code object, held until the process ends.  Host code never
// passes `scratch` itself to a kernel (on the host the name is only a
// stand-in, not a device address); it uses the address that
// hipGetSymbolAddress returns for the current device, resolved once per device
// at the entry point's first call there.
static __device__ __align__(256) unsigned char scratch[HAWKES_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[HK_MAX_DEVICES];

static hawkes_status scratch_address(void** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return HAWKES_EDEVICE;
    }
    if (dev < 0 || dev >= HK_MAX_DEVICES) return HAWKES_EDEVICE;
    std::lock_guard<std::mutex> g(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return HAWKES_EDEVICE;
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return HAWKES_OK;
}

static bool use_small(const hawkes_problem* p) {
    return p->beta_mode == HAWKES_BETA_SHARED && p->m <= 8 && p->k == 1;
}

extern "C" {

const char* hawkes_status_string(hawkes_status s) {
    switch (s) {
        case HAWKES_OK: return "ok";
        case HAWKES_EINVAL: return "invalid argument";
        case HAWKES_EWORKSPACE: return "workspace missing or too small";
        case HAWKES_EDEVICE: return "device error (HIP call or kernel launch failed)";
        case HAWKES_EUNSUPPORTED: return "unsupported request";
        default: return "unknown status";
    }
}

int hawkes_version(void) { return HAWKES_ABI_VERSION; }

hawkes_status hawkes_set_tuning(const hawkes_tuning* t) {
    hawkes_tuning v = {0, 0, 0, 0};
    if (t) {
        v = *t;
        const bool cols_ok = v.dense_cols == 0 || v.dense_cols == 64 || v.dense_cols == 128 || v.dense_cols == 256;
        const bool er_ok = v.dense_ranges == 0 ||
                           (v.dense_ranges >= 1 && v.dense_ranges <= 4096 && (v.dense_ranges & (v.dense_ranges - 1)) == 0);
        const bool item_ok = v.item_log2 == 0 || (v.item_log2 >= 4 && v.item_log2 <= 16);
        const bool rows_ok = v.dense_rows == 0 || v.dense_rows == 16 || v.dense_rows == 32;
        if (!cols_ok || !er_ok || !item_ok || !rows_ok) return HAWKES_EINVAL;
    }
    std::lock_guard<std::mutex> g(g_tuning_mu);
    g_tuning = v;
    return HAWKES_OK;
}

hawkes_status hawkes_get_tuning(hawkes_tuning* t) {
    if (!t) return HAWKES_EINVAL;
    *t = tuning_snapshot();
    return HAWKES_OK;
}

size_t hawkes_workspace_bytes(const hawkes_problem* p, int with_grad) {
    if (!problem_ok(p)) return 0;
    if (use_small(p)) {
        SmallArgs A;
        memset(&A, 0, sizeof(A));
        return small_layout(A, 1, p->n, p->m, with_grad != 0, nullptr, 0, true);
    }
    LargeArgs A;
    memset(&A, 0, sizeof(A));
    return large_layout(A, p, with_grad != 0, nullptr, 0);
}

// support-restricted gradient on the engines that form the dense one: zero
// dL/dalpha where alpha is zero
__global__ void mask_to_support(int64_t n, const float* __restrict__ alpha, double* __restrict__ g_alpha) {
    for (int64_t x = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; x < n; x += (int64_t)gridDim.x * blockDim.x)
        if (alpha[x] == 0.0f) g_alpha[x] = 0.0;
}

static hawkes_status mask_support(const hawkes_problem* p, const float* alpha, double* g_alpha, hipStream_t st) {
    if (!g_alpha) return HAWKES_OK;
    const int64_t n = (int64_t)p->k * p->m * p->m;
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(mask_to_support, dim3((unsigned)(nb < 4096 ? nb : 4096)), dim3(256), 0, st, n, alpha,
                       g_alpha);
    return hipGetLastError() == hipSuccess ? HAWKES_OK : HAWKES_EDEVICE;
}

static hawkes_status run_single(const hawkes_problem* p, const double* t, const int32_t* marks, const float* mu,
                                const float* alpha, const float* beta, double* loglik, double* g_mu,
                                double* g_alpha, double* g_beta, float* lambda_out, bool grad, void* ws,
                                size_t ws_bytes, hipStream_t stream, bool support = false) {
    if (!problem_ok(p) || !mu || !alpha || !beta) return HAWKES_EINVAL;
    if (!loglik && !lambda_out) return HAWKES_EINVAL;
    if (p->n > 0 && (!t || !marks)) return HAWKES_EINVAL;
    if (!ws) return HAWKES_EWORKSPACE;
    if (use_small(p)) {
        SmallArgs A;
        memset(&A, 0, sizeof(A));
        const size_t need = small_layout(A, 1, p->n, p->m, grad, ws, ws_bytes, true);
        if (ws_bytes < need) return HAWKES_EWORKSPACE;
        if (((uintptr_t)ws & 255) != 0) return HAWKES_EWORKSPACE;
        hipLaunchKernelGGL(write_single_desc, dim3(1), dim3(64), 0, stream, p->n, p->m, p->T,
                           (int64_t*)A.ev_off, (int32_t*)A.m_s, (double*)A.T_s);
        A.t = t; A.marks = marks; A.mu = mu; A.alpha = alpha; A.beta = beta;
        A.loglik = loglik ? loglik : A.ll_scratch;
        A.g_mu = g_mu; A.g_alpha = g_alpha; A.g_beta = g_beta;
        A.lambda_out = lambda_out;
        const hawkes_status st = run_small(A, stream);
        return st == HAWKES_OK && support ? mask_support(p, alpha, g_alpha, stream) : st;
    }
    LargeArgs A;
    memset(&A, 0, sizeof(A));
    const size_t need = large_layout(A, p, grad, ws, ws_bytes);
    if (ws_bytes < need) return HAWKES_EWORKSPACE;
    if (((uintptr_t)ws & 255) != 0) return HAWKES_EWORKSPACE;
    A.t = t; A.marks = marks; A.mu = mu; A.alpha = alpha; A.beta = beta;
    A.loglik = loglik ? loglik : A.ll_scratch;
    A.g_mu = g_mu; A.g_alpha = g_alpha; A.g_beta = g_beta;
    A.lambda_out = lambda_out;
    // one shared decay: the first term only on the support (forward pass);
    // per target or several kernels: the dense gradient, masked
    A.support = support && !A.per_target && A.K == 1;
    const hawkes_status st = run_large(A, stream);
    return st == HAWKES_OK && support && !A.support ? mask_support(p, alpha, g_alpha, stream) : st;
}

hawkes_status hawkes_loglik(const hawkes_problem* p, const double* t, const int32_t* marks, const float* mu,
                            const float* alpha, const float* beta, double* loglik, void* workspace,
                            size_t workspace_bytes, hipStream_t stream) {
    return run_single(p, t, marks, mu, alpha, beta, loglik, nullptr, nullptr, nullptr, nullptr, false,
                      workspace, workspace_bytes, stream);
}

hawkes_status hawkes_loglik_grad(const hawkes_problem* p, const double* t, const int32_t* marks, const float* mu,
                                 const float* alpha, const float* beta, double* loglik, double* g_mu,
                                 double* g_alpha, double* g_beta, void* workspace, size_t workspace_bytes,
                                 hipStream_t stream) {
    return run_single(p, t, marks, mu, alpha, beta, loglik, g_mu, g_alpha, g_beta, nullptr, true, workspace,
                      workspace_bytes, stream);
}

hawkes_status hawkes_loglik_grad_noalloc(const hawkes_problem* p, const double* t, const int32_t* marks,
                                         const float* mu, const float* alpha, const float* beta, double* loglik,
                                         double* g_mu, double* g_alpha, double* g_beta, hipStream_t stream) {
    // every host check of hawkes_loglik_grad first, so that a bad argument
    // gives the same status; then the problem's workspace must fit the
    // fixed scratch
    if (!problem_ok(p) || !mu || !alpha || !beta || !loglik) return HAWKES_EINVAL;
    if (p->n > 0 && (!t || !marks)) return HAWKES_EINVAL;
    const size_t need = hawkes_workspace_bytes(p, 1);
    if (need == 0) return HAWKES_EUNSUPPORTED;
    if (need > (size_t)HAWKES_NOALLOC_SCRATCH_BYTES) return HAWKES_EWORKSPACE;
    void* ws = nullptr;
    const hawkes_status st = scratch_address(&ws);
    if (st != HAWKES_OK) return st;
    return run_single(p, t, marks, mu, alpha, beta, loglik, g_mu, g_alpha, g_beta, nullptr, true, ws,
                      (size_t)HAWKES_NOALLOC_SCRATCH_BYTES, stream);
}

hawkes_status hawkes_loglik_grad_support(const hawkes_problem* p, const double* t, const int32_t* marks,
                                         const float* mu, const float* alpha, const float* beta, double* loglik,
                                         double* g_mu, double* g_alpha, double* g_beta, void* workspace,
                                         size_t workspace_bytes, hipStream_t stream) {
    return run_single(p, t, marks, mu, alpha, beta, loglik, g_mu, g_alpha, g_beta, nullptr, true, workspace,
                      workspace_bytes, stream, true);
}

hawkes_status hawkes_intensity(const hawkes_problem* p, const double* t, const int32_t* marks, const float* mu,
                               const float* alpha, const float* beta, float* lambda_out, void* workspace,
                               size_t workspace_bytes, hipStream_t stream) {
    if (!lambda_out) return HAWKES_EINVAL;
    // the log-likelihood computed alongside goes to a workspace slot
    return run_single(p, t, marks, mu, alpha, beta, nullptr, nullptr, nullptr, nullptr, lambda_out, false,
                      workspace, workspace_bytes, stream);
}

// Batches with more than 8 nodes in some sequence: the small-M engine's
// workspace for the whole batch (at 8 nodes), then the large-M engine's for
// one sequence of up to n_total events and max_m nodes (constant beyond one
// chunk), 256-byte aligned after it.
static size_t batched_large_bytes(int64_t n_total, int32_t max_m, bool grad) {
    hawkes_problem p;
    memset(&p, 0, sizeof(p));
    p.n = n_total;
    p.m = max_m;
    p.k = 1;
    p.beta_mode = HAWKES_BETA_SHARED;
    p.T = 1.0;
    LargeArgs A;
    memset(&A, 0, sizeof(A));
    return large_layout(A, &p, grad, nullptr, 0);
}

size_t hawkes_batched_workspace_bytes(int32_t S, int64_t n_total, int32_t max_m, int with_grad) {
    if (S < 1 || n_total < 0 || max_m < 1) return 0;
    if ((int64_t)max_m * max_m > ((int64_t)1 << 31)) return 0;
    SmallArgs A;
    memset(&A, 0, sizeof(A));
    const size_t small = small_layout(A, S, n_total, max_m < 8 ? max_m : 8, with_grad != 0, nullptr, 0, false);
    if (max_m <= 8) return small;
    return ((small + 255) & ~(size_t)255) + batched_large_bytes(n_total, max_m, with_grad != 0);
}

static hawkes_status run_batched(int32_t S, int64_t n_total, int32_t max_m, const int64_t* ev_off,
                                 const int32_t* m_s, const double* T_s, const double* t, const int32_t* marks,
                                 const float* mu, const float* alpha, const float* beta, double* loglik,
                                 double* g_mu, double* g_alpha, double* g_beta, bool grad, void* ws,
                                 size_t ws_bytes, hipStream_t stream) {
    if (S < 1 || n_total < 0 || max_m < 1) return HAWKES_EINVAL;
    if ((int64_t)max_m * max_m > ((int64_t)1 << 31)) return HAWKES_EINVAL;
    if (!ev_off || !m_s || !T_s || !mu || !alpha || !beta || !loglik) return HAWKES_EINVAL;
    if (n_total > 0 && (!t || !marks)) return HAWKES_EINVAL;
    if (!ws) return HAWKES_EWORKSPACE;
    const size_t need = hawkes_batched_workspace_bytes(S, n_total, max_m, grad ? 1 : 0);
    if (need == 0) return HAWKES_EINVAL;
    if (ws_bytes < need || ((uintptr_t)ws & 255) != 0) return HAWKES_EWORKSPACE;
    SmallArgs A;
    memset(&A, 0, sizeof(A));
    const size_t small = small_layout(A, S, n_total, max_m < 8 ? max_m : 8, grad, ws, ws_bytes, false);
    A.ev_off = ev_off; A.m_s = m_s; A.T_s = T_s;
    A.t = t; A.marks = marks; A.mu = mu; A.alpha = alpha; A.beta = beta;
    A.loglik = loglik; A.g_mu = g_mu; A.g_alpha = g_alpha; A.g_beta = g_beta;
    A.lambda_out = nullptr;
    if (max_m <= 8) return run_small(A, stream);
    // Sequences with more than 8 nodes: the offsets, node counts and window
    // ends come to the host (the call synchronises the stream), the small-M
    // engine evaluates the whole batch (its results for the larger
    // sequences, computed on their first 8 nodes, are then overwritten), and
    // the large-M engine evaluates each larger sequence in turn on the same
    // stream, in the workspace after the small engine's.
    std::vector<int64_t> off((size_t)S + 1);
    std::vector<int32_t> ms((size_t)S);
    std::vector<double> Ts((size_t)S);
    if (hipMemcpyAsync(off.data(), ev_off, sizeof(int64_t) * (S + 1), hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(ms.data(), m_s, sizeof(int32_t) * S, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipMemcpyAsync(Ts.data(), T_s, sizeof(double) * S, hipMemcpyDeviceToHost, stream) != hipSuccess ||
        hipStreamSynchronize(stream) != hipSuccess) {
        (void)hipGetLastError();
        return HAWKES_EDEVICE;
    }
    bool any_small = false;
    for (int32_t q = 0; q < S; ++q) {
        if (ms[q] < 1 || ms[q] > max_m || off[q] < 0 || off[q + 1] < off[q] || off[q + 1] > n_total)
            return HAWKES_EINVAL;
        any_small = any_small || ms[q] <= 8;
    }
    hawkes_status st = any_small ? run_small(A, stream) : HAWKES_OK;
    char* lws = (char*)ws + ((small + 255) & ~(size_t)255);
    const size_t lbytes = ws_bytes - ((small + 255) & ~(size_t)255);
    int64_t mu_o = 0, a_o = 0;
    for (int32_t q = 0; q < S && st == HAWKES_OK; ++q) {
        const int64_t mq = ms[q];
        if (mq > 8) {
            hawkes_problem p;
            memset(&p, 0, sizeof(p));
            p.n = off[q + 1] - off[q];
            p.m = (int32_t)mq;
            p.k = 1;
            p.beta_mode = HAWKES_BETA_SHARED;
            p.T = Ts[q];
            const int64_t e0 = off[q];
            st = run_single(&p, t ? t + e0 : nullptr, marks ? marks + e0 : nullptr, mu + mu_o, alpha + a_o,
                            beta + q, loglik + q, g_mu ? g_mu + mu_o : nullptr, g_alpha ? g_alpha + a_o : nullptr,
                            g_beta ? g_beta + q : nullptr, nullptr, grad, lws, lbytes, stream);
        }
        mu_o += mq;
        a_o += mq * mq;
    }
    return st;
}

hawkes_status hawkes_loglik_batched(int32_t S, int64_t n_total, int32_t max_m, const int64_t* ev_off,
                                    const int32_t* m_s, const double* T_s, const double* t, const int32_t* marks,
                                    const float* mu, const float* alpha, const float* beta, double* loglik,
                                    void* workspace, size_t workspace_bytes, hipStream_t stream) {
    return run_batched(S, n_total, max_m, ev_off, m_s, T_s, t, marks, mu, alpha, beta, loglik, nullptr, nullptr,
                       nullptr, false, workspace, workspace_bytes, stream);
}

hawkes_status hawkes_loglik_grad_batched(int32_t S, int64_t n_total, int32_t max_m, const int64_t* ev_off,
                                         const int32_t* m_s, const double* T_s, const double* t,
                                         const int32_t* marks, const float* mu, const float* alpha,
                                         const float* beta, double* loglik, double* g_mu, double* g_alpha,
                                         double* g_beta, void* workspace, size_t workspace_bytes,
                                         hipStream_t stream) {
    return run_batched(S, n_total, max_m, ev_off, m_s, T_s, t, marks, mu, alpha, beta, loglik, g_mu, g_alpha,
                       g_beta, true, workspace, workspace_bytes, stream);
}

hawkes_status hawkes_sequential_loglik_grad(const hawkes_problem* p, const double* t, const int32_t* marks,
                                            const float* mu, const float* alpha, const float* beta,
                                            double* loglik, double* g_mu, double* g_alpha, double* g_beta,
                                            void* workspace, size_t workspace_bytes, hipStream_t stream) {
    if (!problem_ok(p) || !mu || !alpha || !beta || !loglik) return HAWKES_EINVAL;
    if (p->k != 1 || p->beta_mode != HAWKES_BETA_SHARED) return HAWKES_EUNSUPPORTED;
    if (p->n > 0 && (!t || !marks)) return HAWKES_EINVAL;
    if (!workspace) return HAWKES_EWORKSPACE;
    const size_t need = seq_workspace_bytes(p);
    if (workspace_bytes < need || ((uintptr_t)workspace & 255) != 0) return HAWKES_EWORKSPACE;
    return run_sequential(p, t, marks, mu, alpha, beta, loglik, g_mu, g_alpha, g_beta, workspace, stream);
}

hawkes_status hawkes_check_inputs(const hawkes_problem* p, const double* t, const int32_t* marks, const float* mu,
                                  const float* alpha, const float* beta, int32_t* status_out,
                                  hipStream_t stream) {
    if (!problem_ok(p) || !mu || !alpha || !beta || !status_out) return HAWKES_EINVAL;
    if (p->n > 0 && (!t || !marks)) return HAWKES_EINVAL;
    return run_check_inputs(p, t, marks, mu, alpha, beta, status_out, stream);
}

}  // extern "C"
