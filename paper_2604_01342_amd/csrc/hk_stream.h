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
// places ahead of the read position; the pending registers hold, once their
// loads land, the record 64 + l places ahead.  A window move is split in two:
// shift(n) (0 <= n <= 64) moves the position by n, taking the records that
// enter cur from the pending ones by one ds_bpermute per word, and refill()
// issues the loads of the next pending records.  A kernel with several
// streams shifts all of them before it refills any, so that no shift waits
// on a load issued in the same window: every load has one window of work to
// land.  Every lane reloads (the lanes whose record did not change hit the
// cache), so the count of loads in flight is the same on every path.
// Positions past the list hold a clamped (valid, unused) record.
template <bool REV>
struct RecStream {
    const uint32_t* K;
    const double* Tm;
    const float* W;
    int64_t lo, hi, pos;
    uint32_t ck, pk;
    double ct, pt;
    float cw, pw;

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
        const int64_t a = at(threadIdx.x & 63);
        ck = K[a];
        ct = Tm[a];
        cw = W[a];
        refill();
    }
    // Called once after every stream of the kernel is set up: the initial
    // loads of cur land here.  Otherwise they would still be in flight on the
    // path into the window loop, and the wait the compiler places at the
    // loop's head (merged over the paths into it) would make every window
    // wait on the refill loads issued just before it.
    __device__ __forceinline__ void settle() { asm volatile("" : "+v"(ck), "+v"(ct), "+v"(cw)); }
    __device__ __forceinline__ int64_t avail() const { return REV ? pos - lo : hi - pos; }
    __device__ __forceinline__ void shift(int n) {
        if (n <= 0) return;
        const int lane = threadIdx.x & 63;
        const int src = (lane + n) & 63;
        const bool from_cur = lane + n < 64;
        const uint32_t sck = (uint32_t)__shfl((int)ck, src, 64), spk = (uint32_t)__shfl((int)pk, src, 64);
        const double sct = __shfl(ct, src, 64), spt = __shfl(pt, src, 64);
        const float scw = __shfl(cw, src, 64), spw = __shfl(pw, src, 64);
        ck = from_cur ? sck : spk;
        ct = from_cur ? sct : spt;
        cw = from_cur ? scw : spw;
        pos = REV ? pos - n : pos + n;
    }
    __device__ __forceinline__ void refill() {
        const int64_t e = at(64 + (threadIdx.x & 63));
        pk = K[e];
        pt = Tm[e];
        pw = W[e];
    }
};

}  // namespace hk
