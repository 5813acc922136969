// Large-M engine (M > 8, or a decay per target node): internals.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "hk_internal.h"

#ifndef HK_SEG
#define HK_SEG 1024        // events per forward segment (one wave)
#endif
#define HK_RB 64           // targets per block of the per-target (adjoint) dense kernel
#define HK_SLAB 64         // columns per dense-gradient block (one per lane)
#ifndef HK_DW
#define HK_DW 2            // waves per workgroup of the shared-decay dense kernel
#endif
#ifndef HK_CKR
#define HK_CKR 4           // segments per checkpoint run of the shared-decay dense gradient
#endif
#define HK_WIDE 60.0       // anchored-exponent limit inside one window of the dense kernel
#ifndef HK_DWF
#define HK_DWF 4           // waves per workgroup of the float32-accumulator dense kernel (32-row tiles)
#endif
#ifndef HK_F32_MIN_M
#define HK_F32_MIN_M 384   // nodes from which the 32-row float32-accumulator tiles are the rule
#endif
// float64 words of a dense-gradient checkpoint slot: state, header, and
// per record (64 NGW of them) its time, key and factor
#define HK_SLOT_WORDS(CPL, NGW) (64 * (CPL) + 8 + 128 * (NGW))

namespace hk {

#define HK_KMAX 8          // decay kernels per problem (shared decay per kernel)

struct LargeArgs {
    int64_t n;
    int32_t M;
    int32_t K;            // decay kernels (shared decay): alpha[K][M][M], beta[K]
    int32_t per_target;   // beta[M] instead of beta[1]
    double T;
    int64_t CH;           // events per chunk
    int64_t nchunks;
    int32_t nseg;         // segments per chunk
    int32_t ER;           // event ranges of the dense kernel per chunk
    int32_t NB;           // node blocks of 64 (bucketing; columns of the dense kernels)
    int32_t NBR;          // row blocks of the dense kernel (DR rows shared decay, HK_RB per target)
    int32_t CPL;          // columns per lane of the shared-decay dense kernel (1, 2, 4 or 8)
    int32_t DRB;          // log2 of DR, the rows per block of the shared-decay dense kernel
    int32_t NGW;          // groups of 64 column records per window of the shared-decay dense kernel (1, 2)
    int32_t NBC;          // column blocks of the dense kernel (64 CPL columns each)
    int32_t CKR;          // segments per checkpoint run (shared decay)
    int32_t NRUN;         // checkpoint runs per chunk (nseg / CKR)
    bool grad;
    bool support;         // dL/dalpha only at alpha's nonzeros (zero elsewhere), shared decay
    const double* t;
    const int32_t* marks;
    const float *mu, *alpha, *beta;
    // workspace (with K > 1 the per-kernel arrays below are K consecutive
    // copies: csr_*, colsum, node_info, carry, carry_seg, gpart, spart, cpart_)
    int32_t* csr_ptr;
    int2* csr_cv;         // nonzeros of alpha by row: (column, float bits of the value)
    float* colsum;
    double *rk, *dk;      // K > 1: [K][CH] per event of the chunk, R_k and D_k (alpha row . K and . J)
    double* agg;          // [nseg][2M] segment maps (K_run, J_run)
    double* seg_span;     // [nseg] time from the event before the segment to its last event
    double* seg_dec;      // [nseg] e^{-beta (span of the segment from the preceding event)}
    double* seg_off;      // [nseg] time from the event before the segment's scan group to the event before it
    double* seg_offdec;   // [nseg] e^{-beta seg_off} (shared decay)
    double* carry_seg;    // [nseg][2M] state just after the event preceding segment s
    int32_t ngr;          // scan groups per chunk
    double *gagg, *gcarry, *gspan, *gdec;   // group maps, carries, spans, decays
    int4* node_info;      // [M] (csr begin, csr end, mu, colsum)
    double* carry;        // [2M] chunk carry (K, J) just after the chunk's last event
    float* pt_flags;      // [2] per-target engine: beta_min, and (int) whether a chunk is near T
    double* seg_part;     // [nseg][2 + 2K]
    double* acc;          // [2 + 2K] call-level sums: logsum, comp, E[K], gbeta[K]
    double* ll_scratch;   // [1] log-likelihood slot when the caller wants intensities only
    bool carry_prefix;    // carry_seg holds in-group prefixes (the scan's apply pass left out)
    double *gpart, *spart, *cpart_;  // [ER][M][M]; [ER][M] per target, [NRUN][M] shared decay
    double* gsup;         // [min(8, ER)][M*M] support-restricted first term of eq. 9 in CSR order (the
                          //   first nnz(alpha) entries of each copy; shares gpart's space)
    int64_t nslot;        // checkpoint slots
    double* kck;          // [nslot][HK_SLOT_WORDS(CPL, NGW)] state checkpoints of the dense gradient (shared
                          //   decay) with their groups' records
    int4* runinfo;        // [NBC][NRUN] per checkpoint run: first slot, groups, P0, P1
    // per-target decays (R-form forward, reverse adjoint for the gradient)
    int32_t* csc_ptr;   // alpha by column: targets p of source q
    int2* csc_cv;       // (target, float bits of the value)
    float* wv;            // [CH] w_i = 1/lambda_i of the chunk's events
    double* pt_ck;        // [2 HK_PTCK][2M] chunk-start states (R, D): level-1 slots, then level-2 slots
    int64_t pt_ckr;       // chunks per level-1 slot
    double* ebseg;        // [nseg][M] per segment: sum_j alpha_{p,m_j} (T - t_j) e^{-beta_p (T - t_j)}
                          //   minus sum_{i: m_i = p} w_i (R_i - beta_p D_i)
    double* ebacc;        // [M] the same over the whole sequence (= -dL/dbeta_p)
    double* aggA;         // [nseg][M] reverse segment aggregates of the adjoint state
    double* rcarry_seg;   // [nseg][M] adjoint state at each segment's first event (events from there on)
    double *rgagg, *rgcarry;  // [ngr][M] reverse group aggregates and carries
    double* achunk;       // [M] adjoint state entering the current chunk from the right
    // events of the chunk partitioned by node block (64 nodes), in event order
    // (per-target decays)
    int32_t* bk_cnt;      // [NB][nseg] events per (block, segment)
    int32_t* bk_off;      // [NB][nseg + 1] start of each (block, segment) run within the block
    int32_t* bk_base;     // [NB] start of each block in the records
    uint32_t* bk_key;     // [CH] (index in chunk) << bs | mark mod 2^bs (blocks of 2^bs nodes)
    double* bk_t;         // [CH] event time
    float* bk_w;          // [CH] 1 / lambda
    float* wchunk;        // [CH] 1 / lambda of the chunk's events (shared decay)
    // the same events partitioned by blocks of DR nodes (the row blocks of
    // the shared-decay dense kernel): its own-event streams
    int32_t NBO;          // row blocks (ceil(M / DR))
    int32_t *bo_cnt, *bo_off, *bo_base;
    uint32_t* bo_key;     // [CH] (index in chunk) << DRB | mark mod DR
    double* bo_t;
    float* bo_w;
    // outputs
    double *loglik, *g_mu, *g_alpha, *g_beta;
    float* lambda_out;
};

#define HK_SG 32           // segments per scan group
#define HK_NBO_MAX 256     // node blocks the forward pass can count for the partition

// optional parts of the shared-decay forward pass (see large_forward)
struct FwdExtra {
    double* rtau;         // [nseg][2M] scratch (the segment maps' buffer, consumed by the scan):
                          // the first M doubles of segment s hold its lazy records' times
    const double* gcarry;
    const double* seg_off;
    const double* seg_offdec;
    int32_t* bcnt;
    int32_t bs, nbo;
};
#define HK_PTCK 64         // checkpoint slots per level of the per-target gradient (at most 64^2 chunks)

size_t large_layout(LargeArgs& A, const hawkes_problem* p, bool grad, void* ws, size_t ws_bytes);
hawkes_status run_large(LargeArgs& A, hipStream_t st);
hawkes_status run_large_pt(LargeArgs& A, hipStream_t st);
// helpers shared by the two large-M paths (host side)
size_t lds_limit();
hawkes_status allow_lds(const void* kernel, size_t bytes, bool with_static = false);
// grants the float32-accumulator dense kernel its LDS tile (when the layout selects it)
hawkes_status dense_allow_lds(const LargeArgs& A);
void large_build_index(int32_t M, const float* alpha, int trans, int32_t* ptr, int2* cv, hipStream_t st);
// entries between consecutive kernels' packed rows of alpha: even (each
// kernel's array starts 16-byte aligned for the forward pass's pair loads)
// and at least one spare entry past the M^2 a dense alpha fills
inline int64_t cv_stride(int64_t MM) { return (MM + 2) & ~(int64_t)1; }
// apply = false leaves carry_seg as in-group prefixes (the forward pass and
// the checkpoint kernel then add the group carries themselves)
void large_scan(LargeArgs& A, int32_t nseg, const float* beta_pt, hipStream_t st, bool apply = true);
void large_chunk_acc_launch(int32_t nseg, int32_t width, const double* seg_part, double* acc, hipStream_t st);
void bucket_chunk(LargeArgs& A, int64_t c0, int64_t c1, int32_t nseg, const float* wchunk, int bs, hipStream_t st);
// counted: cnt already holds the counts (the forward pass made them)
void bucket_chunk_into(const LargeArgs& A, int64_t c0, int64_t c1, int32_t nseg, const float* wchunk, int bs,
                       int32_t* cnt, int32_t* off, int32_t* base, uint32_t* key, double* tt, float* ww,
                       hipStream_t st, bool counted = false);
// ck_only: the checkpoint kernel alone (its per-column sums of dL/dmu and
// the compensator), for the support-restricted gradient
void large_dense_launch(LargeArgs& A, int64_t c0, int64_t c1, int32_t nseg, hipStream_t st, bool ck_only);

size_t seq_workspace_bytes(const hawkes_problem* p);
hawkes_status run_sequential(const hawkes_problem* p, const double* t, const int32_t* marks, const float* mu,
                             const float* alpha, const float* beta, double* loglik, double* g_mu,
                             double* g_alpha, double* g_beta, void* ws, hipStream_t st);
hawkes_status run_check_inputs(const hawkes_problem* p, const double* t, const int32_t* marks, const float* mu,
                               const float* alpha, const float* beta, int32_t* status_out, hipStream_t st);

}  // namespace hk
