// Register window onto a list of bucketed event records (one node block's
// events of a range, in event order), used by the dense-gradient kernels.
// Internal to the GPU library.
#pragma once
#include "hk_device.h"

namespace hk {

__device__ __forceinline__ int rl_i(int v, int k) { return __builtin_amdgcn_readlane(v, k); }
__device__ __forceinline__ float rl_f(float v, int k) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), k));
}
__device__ __forceinline__ double rl_d(double v, int k) {
    const int64_t b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffff), k);
    const int hi = __builtin_amdgcn_readlane((int)(b >> 32), k);
    return __longlong_as_double(((int64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Records [lo, hi) of the arrays (key, t, w), read in order (REV = false: from
// lo upward; REV = true: from hi downward).  Lane l of cur holds the record l
// places ahead of the read position, lane l of nxt the record 64 + l places
// ahead.  consume(n) moves the position by n (0 < n <= 64): both halves shift
// by n lanes (ds_bpermute), and the lanes of nxt that run past the old window
// are refilled by loads issued now and merged at the next consume, so their
// latency hides behind one window of work.  Positions past the list hold a
// clamped (valid, unused) record.
template <bool REV>
struct RecStream {
    const uint32_t* K;
    const double* Tm;
    const float* W;
    int64_t lo, hi, pos;
    uint32_t ck, nk, pk;
    double ct, nt, pt;
    float cw, nw, pw;
    int split;   // lanes >= split of nxt are still in (pk, pt, pw)

    __device__ __forceinline__ int64_t at(int64_t ahead) const {
        int64_t e = REV ? pos - 1 - ahead : pos + ahead;
        if (hi <= lo) return 0;
        e = e < lo ? lo : e;
        e = e >= hi ? hi - 1 : e;
        return e;
    }
    __device__ __forceinline__ void init(const uint32_t* K_, const double* T_, const float* W_, int64_t lo_,
                                         int64_t hi_) {
        K = K_;
        Tm = T_;
        W = W_;
        lo = lo_;
        hi = hi_;
        pos = REV ? hi : lo;
        const int lane = threadIdx.x & 63;
        const int64_t a = at(lane), b = at(64 + lane);
        ck = K[a];
        ct = Tm[a];
        cw = W[a];
        nk = K[b];
        nt = Tm[b];
        nw = W[b];
        split = 64;
    }
    __device__ __forceinline__ int64_t avail() const { return REV ? pos - lo : hi - pos; }
    __device__ __forceinline__ void consume(int n) {
        if (n <= 0) return;
        const int lane = threadIdx.x & 63;
        if (lane >= split) {
            nk = pk;
            nt = pt;
            nw = pw;
        }
        const int src = (lane + n) & 63;
        const bool from_cur = lane + n < 64;
        const uint32_t sck = (uint32_t)__shfl((int)ck, src, 64), snk = (uint32_t)__shfl((int)nk, src, 64);
        const double sct = __shfl(ct, src, 64), snt = __shfl(nt, src, 64);
        const float scw = __shfl(cw, src, 64), snw = __shfl(nw, src, 64);
        ck = from_cur ? sck : snk;
        ct = from_cur ? sct : snt;
        cw = from_cur ? scw : snw;
        nk = snk;
        nt = snt;
        nw = snw;
        pos = REV ? pos - n : pos + n;
        if (!from_cur) {
            const int64_t e = at(64 + lane);
            pk = K[e];
            pt = Tm[e];
            pw = W[e];
        }
        split = 64 - n;
    }
};

}  // namespace hk
