/*
 * FP64 CPU oracle for the exact log-likelihood of the multivariate linear
 * exponential Hawkes process and its gradient.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
 * call this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code, header, table or constant with the
 * HIP library.
 *
 * Paper: "Massively Parallel Exact Inference for Hawkes Processes"
 * (arXiv 2604.01342).  Notation follows the paper:
 *   lambda_p(t) = mu_p + sum_{j: t_j < t} sum_k alpha_{p,m_j,k} gamma_k
 *                 exp(-gamma_k (t - t_j))                    (Background, eq. 1)
 *   L = sum_i log lambda_{m_i}(t_i) - sum_m int_0^T lambda_m(t) dt   (eq. 2)
 * The decay rate gamma_k is called beta here.  alpha is stored
 * alpha[k][p][q] with p the target (the intensity being computed) and q the
 * source node, as in eq. 1.  Events with equal time stamps follow index order
 * (event j excites event i iff j < i), which is what the recurrence of eq. 4
 * computes.  All arithmetic is double precision.
 *
 * Three routines:
 *   oracle_brute      the definition itself: eq. 1 and eq. 2 as O(N^2) double
 *                     sums, with the gradient of eqs. 8-10 as double sums.
 *                     The decay may differ per (kernel, target): beta[k][p].
 *   oracle_forward    the sequential recurrence of Background section "Sequential
 *                     Recurrence" (eq. 4) in its source-indexed form K (the
 *                     gradient state of eq. 11) plus a time-weighted state J,
 *                     one pass in index order.  Shared decay per kernel.
 *   oracle_adjoint    a reverse-mode (adjoint) pass for one kernel whose decay
 *                     differs per target node, beta[p].
 * The two recurrences are exact rewritings of the double sums (equal up to
 * rounding order); the tests pin them to oracle_brute, to central finite
 * differences, to the Poisson closed form and to a hand-derived closed form.
 *
 * Return value: 0 on success, -1 on invalid arguments.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------------
 * Definition (eqs. 1, 2, 8, 9, 10) as O(N^2) sums.
 * beta is [K][M]: decay of kernel k for target p.  A decay shared by all
 * targets (the paper's gamma_k) is beta[k][p] = gamma_k for every p, and its
 * gradient is the sum over p of g_beta[k][p].
 * Outputs may be NULL (except loglik).
 * ------------------------------------------------------------------------- */
int oracle_brute(int64_t n, int32_t M, int32_t K, double T,
                 const double* t, const int32_t* m,
                 const double* mu, const double* alpha, const double* beta,
                 double* loglik, double* g_mu, double* g_alpha, double* g_beta)
{
    if (n < 0 || M < 1 || K < 1 || !loglik || (n > 0 && (!t || !m)) || !mu || !alpha || !beta)
        return -1;
    const int64_t MM = (int64_t)M * M;
    double* lam = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!lam) return -1;

    /* eq. 1 at every event: lambda_{m_i}(t_i), sum over j < i */
    for (int64_t i = 0; i < n; ++i) {
        const int p = m[i];
        double l = mu[p];
        for (int64_t j = 0; j < i; ++j)
            for (int k = 0; k < K; ++k) {
                const double b = beta[(int64_t)k * M + p];
                l += alpha[k * MM + (int64_t)p * M + m[j]] * b * exp(-b * (t[i] - t[j]));
            }
        lam[i] = l;
    }

    /* eq. 2: log-sum minus the integral; the integral of eq. 1 over [0,T] is
       mu_p T + sum_j sum_k alpha_{p,m_j,k} (1 - exp(-beta (T - t_j))). */
    double L = 0.0;
    for (int64_t i = 0; i < n; ++i) L += log(lam[i]);
    for (int p = 0; p < M; ++p) {
        double comp = mu[p] * T;
        for (int64_t j = 0; j < n; ++j)
            for (int k = 0; k < K; ++k) {
                const double b = beta[(int64_t)k * M + p];
                comp += alpha[k * MM + (int64_t)p * M + m[j]] * (1.0 - exp(-b * (T - t[j])));
            }
        L -= comp;
    }
    *loglik = L;

    /* eq. 8: dL/dmu_p = sum_{i: m_i = p} 1/lambda_i - T */
    if (g_mu) {
        for (int p = 0; p < M; ++p) g_mu[p] = -T;
        for (int64_t i = 0; i < n; ++i) g_mu[m[i]] += 1.0 / lam[i];
    }
    /* eq. 9: dL/dalpha_{p,q,k} = sum_{i: m_i=p} beta sum_{j<i, m_j=q} e^{-beta(t_i-t_j)} / lambda_i
                                 - sum_{j: m_j = q} (1 - e^{-beta (T - t_j)}) */
    if (g_alpha) {
        for (int64_t x = 0; x < (int64_t)K * MM; ++x) g_alpha[x] = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            const int p = m[i];
            for (int64_t j = 0; j < i; ++j)
                for (int k = 0; k < K; ++k) {
                    const double b = beta[(int64_t)k * M + p];
                    g_alpha[k * MM + (int64_t)p * M + m[j]] += b * exp(-b * (t[i] - t[j])) / lam[i];
                }
        }
        for (int k = 0; k < K; ++k)
            for (int p = 0; p < M; ++p)
                for (int64_t j = 0; j < n; ++j) {
                    const double b = beta[(int64_t)k * M + p];
                    g_alpha[k * MM + (int64_t)p * M + m[j]] -= 1.0 - exp(-b * (T - t[j]));
                }
    }
    /* eq. 10 (per target): d lambda_i / d beta = sum_{j<i} alpha (1 - beta (t_i - t_j)) e^{-beta (t_i - t_j)};
       d integral / d beta = sum_j alpha (T - t_j) e^{-beta (T - t_j)}.  The paper's form
       (1 - gamma t_i) R + gamma L equals this with L the t_j-weighted state. */
    if (g_beta) {
        for (int64_t x = 0; x < (int64_t)K * M; ++x) g_beta[x] = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            const int p = m[i];
            for (int64_t j = 0; j < i; ++j)
                for (int k = 0; k < K; ++k) {
                    const double b = beta[(int64_t)k * M + p];
                    const double a = alpha[k * MM + (int64_t)p * M + m[j]];
                    const double dt = t[i] - t[j];
                    g_beta[(int64_t)k * M + p] += a * (1.0 - b * dt) * exp(-b * dt) / lam[i];
                }
        }
        for (int k = 0; k < K; ++k)
            for (int p = 0; p < M; ++p)
                for (int64_t j = 0; j < n; ++j) {
                    const double b = beta[(int64_t)k * M + p];
                    const double a = alpha[k * MM + (int64_t)p * M + m[j]];
                    g_beta[(int64_t)k * M + p] -= a * (T - t[j]) * exp(-b * (T - t[j]));
                }
    }
    free(lam);
    return 0;
}

/* Intensity at selected events by the definition (eq. 1), each an O(i) sum.
 * beta is [K][M] as in oracle_brute.  lam_out[s] = lambda_{m_i}(t_i), i = idx[s]. */
int oracle_intensity_at(int64_t n, int32_t M, int32_t K,
                        const double* t, const int32_t* m,
                        const double* mu, const double* alpha, const double* beta,
                        int64_t ns, const int64_t* idx, double* lam_out)
{
    if (n < 0 || M < 1 || K < 1 || ns < 0 || !t || !m || !mu || !alpha || !beta || !idx || !lam_out)
        return -1;
    const int64_t MM = (int64_t)M * M;
    for (int64_t s = 0; s < ns; ++s) {
        const int64_t i = idx[s];
        if (i < 0 || i >= n) return -1;
        const int p = m[i];
        double l = mu[p];
        for (int64_t j = 0; j < i; ++j)
            for (int k = 0; k < K; ++k) {
                const double b = beta[(int64_t)k * M + p];
                l += alpha[k * MM + (int64_t)p * M + m[j]] * b * exp(-b * (t[i] - t[j]));
            }
        lam_out[s] = l;
    }
    return 0;
}

/* ---------------------------------------------------------------------------
 * Sequential recurrence, forward mode, decay beta[k] shared by all targets.
 *
 * State per kernel k, in index order (the paper's eq. 11 and its companion):
 *   K_q(t_i) = sum_{j<i, m_j=q} e^{-beta (t_i - t_j)}
 *   J_q(t_i) = sum_{j<i, m_j=q} (t_i - t_j) e^{-beta (t_i - t_j)}
 * With d = t_i - t_{i-1} and s = e^{-beta d}:
 *   K(t_i) = s (K(t_{i-1}) + e_{m_{i-1}})
 *   J(t_i) = s J(t_{i-1}) + d K(t_i)
 * J uses time relative to the current event; it equals t K - L with the
 * paper's L state (eq. 12) but does not cancel catastrophically.
 * Then R = alpha_{p,:} . K is the state of eq. 3 for target p, and
 *   lambda_i = mu_p + sum_k beta_k R_k,     p = m_i
 *   dL/dalpha_{p,q,k} += beta_k K_q / lambda_i     (first term of eq. 9)
 *   dL/dbeta_k        += (R_k - beta_k alpha_{p,:} . J) / lambda_i   (eq. 10)
 * followed by the compensator terms (second terms of eqs. 2, 9, 10).
 * O(N M) time per kernel; dense alpha.  Outputs other than loglik may be NULL.
 * ------------------------------------------------------------------------- */
int oracle_forward(int64_t n, int32_t M, int32_t K, double T,
                   const double* t, const int32_t* m,
                   const double* mu, const double* alpha, const double* beta,
                   double* loglik, double* g_mu, double* g_alpha, double* g_beta)
{
    if (n < 0 || M < 1 || K < 1 || !loglik || (n > 0 && (!t || !m)) || !mu || !alpha || !beta)
        return -1;
    const int64_t MM = (int64_t)M * M;
    double* Ks = (double*)calloc((size_t)K * M, sizeof(double));
    double* Js = (double*)calloc((size_t)K * M, sizeof(double));
    double* S = (double*)calloc((size_t)M, sizeof(double));
    double* GA = (double*)calloc((size_t)(K * MM), sizeof(double));
    double* GB = (double*)calloc((size_t)K, sizeof(double));
    double* R = (double*)calloc((size_t)K, sizeof(double));
    double* D = (double*)calloc((size_t)K, sizeof(double));
    if (!Ks || !Js || !S || !GA || !GB || !R || !D) {
        free(Ks); free(Js); free(S); free(GA); free(GB); free(R); free(D);
        return -1;
    }
    double logsum = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (i > 0) {
            const double d = t[i] - t[i - 1];
            const int q = m[i - 1];
            for (int k = 0; k < K; ++k) {
                const double s = exp(-beta[k] * d);
                double* Kk = Ks + (int64_t)k * M;
                double* Jk = Js + (int64_t)k * M;
                Kk[q] += 1.0;
                for (int r = 0; r < M; ++r) {
                    Kk[r] *= s;
                    Jk[r] = s * Jk[r] + d * Kk[r];
                }
            }
        }
        const int p = m[i];
        double lam = mu[p];
        for (int k = 0; k < K; ++k) {
            const double* arow = alpha + k * MM + (int64_t)p * M;
            const double* Kk = Ks + (int64_t)k * M;
            const double* Jk = Js + (int64_t)k * M;
            double r = 0.0, dd = 0.0;
            for (int q = 0; q < M; ++q) { r += arow[q] * Kk[q]; dd += arow[q] * Jk[q]; }
            R[k] = r; D[k] = dd;
            lam += beta[k] * r;
        }
        const double w = 1.0 / lam;
        logsum += log(lam);
        S[p] += w;
        for (int k = 0; k < K; ++k) {
            double* grow = GA + k * MM + (int64_t)p * M;
            const double* Kk = Ks + (int64_t)k * M;
            const double bw = beta[k] * w;
            for (int q = 0; q < M; ++q) grow[q] += bw * Kk[q];
            GB[k] += w * (R[k] - beta[k] * D[k]);
        }
    }
    /* Compensator: int_0^T lambda_p = mu_p T + sum_k sum_j alpha_{p,m_j,k} (1 - e^{-beta_k (T - t_j)}).
       Summed over p it needs only colsum_k[q] = sum_p alpha_{p,q,k}. */
    double comp = 0.0;
    for (int p = 0; p < M; ++p) comp += mu[p] * T;
    for (int k = 0; k < K; ++k) {
        double* C = (double*)calloc((size_t)M, sizeof(double));
        double* colsum = (double*)calloc((size_t)M, sizeof(double));
        if (!C || !colsum) { free(C); free(colsum); comp = NAN; continue; }
        for (int p = 0; p < M; ++p)
            for (int q = 0; q < M; ++q) colsum[q] += alpha[k * MM + (int64_t)p * M + q];
        double E = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            const double x = beta[k] * (T - t[j]);
            C[m[j]] += -expm1(-x);                       /* 1 - e^{-x} */
            E += colsum[m[j]] * (T - t[j]) * exp(-x);    /* d/dbeta of the integral */
        }
        for (int q = 0; q < M; ++q) comp += colsum[q] * C[q];
        if (g_alpha)
            for (int p = 0; p < M; ++p)
                for (int q = 0; q < M; ++q)
                    g_alpha[k * MM + (int64_t)p * M + q] = GA[k * MM + (int64_t)p * M + q] - C[q];
        if (g_beta) g_beta[k] = GB[k] - E;
        free(C); free(colsum);
    }
    *loglik = logsum - comp;
    if (g_mu)
        for (int p = 0; p < M; ++p) g_mu[p] = S[p] - T;
    free(Ks); free(Js); free(S); free(GA); free(GB); free(R); free(D);
    return 0;
}

/* ---------------------------------------------------------------------------
 * Reverse mode for one kernel whose decay depends on the target: beta[p].
 *   lambda_p(t) = mu_p + beta_p sum_{j: t_j<t} alpha_{p,m_j} e^{-beta_p (t - t_j)}
 * Forward pass: R_p(t_i) = sum_{j<i} alpha_{p,m_j} e^{-beta_p (t_i - t_j)} by the
 * affine recurrence of eq. 4 with an element-wise decay; w_i = 1/lambda_i.
 * Reverse pass, j = n-1 .. 0, with adjoint states
 *   A_p(t) = sum_{i: t_i>t, m_i=p} w_i e^{-beta_p (t_i - t)} + e^{-beta_p (T - t)} / beta_p
 *   B_p(t) = sum_{i: t_i>t, m_i=p} w_i (t_i - t) e^{-beta_p (t_i - t)}
 *            + (T - t) e^{-beta_p (T - t)} / beta_p
 * (the second terms fold the compensator into the adjoint).  Then
 *   dL/dalpha_{p,q} = sum_{j: m_j=q} beta_p A_p(t_j) - N_q
 *   dL/dbeta_p      = (N_p - mu_p S_p) / beta_p - beta_p sum_j alpha_{p,m_j} B_p(t_j)
 * with S_p = sum_{i: m_i=p} w_i and N_q the number of q-events.
 * ------------------------------------------------------------------------- */
int oracle_adjoint(int64_t n, int32_t M, double T,
                   const double* t, const int32_t* m,
                   const double* mu, const double* alpha, const double* beta,
                   double* loglik, double* g_mu, double* g_alpha, double* g_beta)
{
    if (n < 0 || M < 1 || !loglik || (n > 0 && (!t || !m)) || !mu || !alpha || !beta)
        return -1;
    double* R = (double*)calloc((size_t)M, sizeof(double));
    double* A = (double*)malloc(sizeof(double) * (size_t)M);
    double* B = (double*)calloc((size_t)M, sizeof(double));
    double* H = (double*)calloc((size_t)M, sizeof(double));
    double* S = (double*)calloc((size_t)M, sizeof(double));
    double* Nq = (double*)calloc((size_t)M, sizeof(double));
    double* GA = (double*)calloc((size_t)M * M, sizeof(double));
    double* w = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!R || !A || !B || !H || !S || !Nq || !GA || !w) {
        free(R); free(A); free(B); free(H); free(S); free(Nq); free(GA); free(w);
        return -1;
    }
    /* forward */
    double logsum = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (i > 0) {
            const double d = t[i] - t[i - 1];
            const int q = m[i - 1];
            for (int p = 0; p < M; ++p)
                R[p] = exp(-beta[p] * d) * (R[p] + alpha[(int64_t)p * M + q]);
        }
        const int p = m[i];
        const double lam = mu[p] + beta[p] * R[p];
        w[i] = 1.0 / lam;
        logsum += log(lam);
        S[p] += w[i];
        Nq[p] += 1.0;
    }
    /* compensator (eq. 2 integral) with per-target decay */
    double comp = 0.0;
    for (int p = 0; p < M; ++p) comp += mu[p] * T;
    for (int64_t j = 0; j < n; ++j)
        for (int p = 0; p < M; ++p)
            comp += alpha[(int64_t)p * M + m[j]] * (-expm1(-beta[p] * (T - t[j])));
    *loglik = logsum - comp;

    /* reverse */
    for (int p = 0; p < M; ++p) A[p] = 1.0 / beta[p];
    double tnext = T;
    for (int64_t j = n - 1; j >= 0; --j) {
        const double d = tnext - t[j];
        const int q = m[j];
        for (int p = 0; p < M; ++p) {
            const double s = exp(-beta[p] * d);
            B[p] = s * (B[p] + d * A[p]);
            A[p] = s * A[p];
            GA[(int64_t)p * M + q] += beta[p] * A[p];
            H[p] += alpha[(int64_t)p * M + q] * beta[p] * B[p];
        }
        A[q] += w[j];
        tnext = t[j];
    }
    if (g_alpha)
        for (int p = 0; p < M; ++p)
            for (int q = 0; q < M; ++q)
                g_alpha[(int64_t)p * M + q] = GA[(int64_t)p * M + q] - Nq[q];
    if (g_beta)
        for (int p = 0; p < M; ++p)
            g_beta[p] = (Nq[p] - mu[p] * S[p]) / beta[p] - H[p];
    if (g_mu)
        for (int p = 0; p < M; ++p) g_mu[p] = S[p] - T;
    free(R); free(A); free(B); free(H); free(S); free(Nq); free(GA); free(w);
    return 0;
}
