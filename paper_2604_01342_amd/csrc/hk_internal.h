// Host-side internals of the GPU library (not part of the public ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>
#include "../../include/hawkes.h"

#define HK_RCH 256          // items per first-level reduction chunk (small engine)
#define HK_MAX_DEVICES 64   // devices with a resolved fixed-scratch address

namespace hk {

// bump allocator over the caller's workspace (256-byte aligned slices)
struct Carve {
    char* base;
    size_t off;
    size_t cap;
    explicit Carve(void* b = nullptr, size_t c = 0) : base((char*)b), off(0), cap(c) {}
    template <typename T>
    T* take(size_t count) {
        off = (off + 255) & ~(size_t)255;
        T* p = base ? (T*)(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
    bool fits() const { return off <= cap; }
};

struct SmallArgs {
    int32_t S;
    int32_t MP;          // padded node count: 1, 2, 4 or 8
    int32_t L;           // events per item
    int64_t n_total;
    int64_t n_items_cap, n_chunks_cap;
    bool grad;
    const int64_t* ev_off;
    const int32_t* m_s;
    const double* T_s;
    const double* t;
    const int32_t* marks;
    const float *mu, *alpha, *beta;
    // workspace
    int64_t *item_off, *chunk_off, *mu_off, *a_off;
    double *item_pref, *tile_agg, *tile_carry, *part, *cpart;
    double* ll_scratch;  // log-likelihood slot when the caller wants intensities only
    // outputs
    double *loglik, *g_mu, *g_alpha, *g_beta;
    float* lambda_out;
};

hawkes_status run_small(const SmallArgs& A, hipStream_t st);

// optional per-kernel event timing (hawkes_timing_*)
void* timing_begin(int id, hipStream_t st);
void timing_end(void* h, hipStream_t st);
struct TimedScope {
    void* h;
    hipStream_t st;
    TimedScope(int id, hipStream_t s) : h(timing_begin(id, s)), st(s) {}
    ~TimedScope() { timing_end(h, st); }
};

// the process-wide launch tuning (hawkes_set_tuning), copied under a lock
hawkes_tuning tuning_snapshot();

// carve the small-engine workspace; returns bytes needed (A gets pointers when ws != nullptr)
size_t small_layout(SmallArgs& A, int32_t S, int64_t n_total, int32_t max_m, bool grad, void* ws,
                    size_t ws_bytes, bool single);

}  // namespace hk
