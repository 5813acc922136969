// Large-M engine (M > 8, or a decay per target node): internals.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "hk_internal.h"

#define HK_SEG 2048        // events per forward segment (one wave)
#define HK_RB 64           // rows per dense-gradient block
#define HK_SLAB 64         // columns per dense-gradient block (one per lane)
#define HK_WIDE 60.0       // anchored-exponent limit inside one 64-event batch

namespace hk {

struct LargeArgs {
    int64_t n;
    int32_t M;
    int32_t per_target;   // beta[M] instead of beta[1]
    double T;
    int64_t CH;           // events per chunk
    int64_t nchunks;
    int32_t nseg;         // segments per chunk
    int32_t ER;           // event ranges of the dense kernel per chunk
    int32_t NB;           // node blocks of 64 (rows and columns)
    bool grad;
    const double* t;
    const int32_t* marks;
    const float *mu, *alpha, *beta;
    // workspace
    int32_t *csr_ptr, *csr_col;
    float *csr_val, *colsum;
    double* agg;          // [nseg][2M] segment maps (K_run, J_run)
    double* seg_span;     // [nseg] time from the event before the segment to its last event
    double* seg_dec;      // [nseg] e^{-beta (span of the segment from the preceding event)}
    double* carry_seg;    // [nseg][2M] state just after the event preceding segment s
    int32_t ngr;          // scan groups per chunk
    double *gagg, *gcarry, *gspan, *gdec;   // group maps, carries, spans, decays
    int4* node_info;      // [M] (csr begin, csr end, mu, colsum)
    double* carry;        // [2M] chunk carry (K, J) at carry_t
    double* carry_t;      // [1] time of the carry (last event before the chunk)
    double* seg_part;     // [nseg][4]
    double* acc;          // [4] call-level sums: logsum, comp, E, gbeta
    double* ll_scratch;   // [1] log-likelihood slot when the caller wants intensities only
    int4* ev_rec;         // [CH] per-event (mark, c, b, w) for the dense kernel
    float* ev_ct;         // [CH] 1 - e^{-beta (T - t_i)} for the dense kernel's row-block 0
    int2* batch_info;     // [CH/64 + 1] per 64-event batch: (rescale factor bits, wide flag)
    double *gpart, *spart, *cpart_;  // [ER][M][M], [ER][M], [ER][M]
    // outputs
    double *loglik, *g_mu, *g_alpha, *g_beta;
    float* lambda_out;
};

size_t large_layout(LargeArgs& A, const hawkes_problem* p, bool grad, void* ws, size_t ws_bytes);
hawkes_status run_large(LargeArgs& A, hipStream_t st);

size_t seq_workspace_bytes(const hawkes_problem* p);
hawkes_status run_sequential(const hawkes_problem* p, const double* t, const int32_t* marks, const float* mu,
                             const float* alpha, const float* beta, double* loglik, double* g_mu,
                             double* g_alpha, double* g_beta, void* ws, hipStream_t st);
hawkes_status run_check_inputs(const hawkes_problem* p, const double* t, const int32_t* marks, const float* mu,
                               const float* alpha, const float* beta, int32_t* status_out, hipStream_t st);

}  // namespace hk
