// Per-chunk partition of the events by node block (16, 64 or 128 nodes per block),
// stable in event order: a counting sort in three steps.
//   count    one wave per segment: events per (block, segment)
//   scan     one workgroup per block: start of every (block, segment) run
//            within the block, boff[block][segment] ([block][nseg] = the
//            block's size)
//   scatter  one workgroup per segment, each wave a quarter of its events:
//            the blocks' starts in the block-major output (bbase[block],
//            stored by segment 0), each event's rank among the events of its
//            block in the same 64-event batch from bit-sliced ballots (one
//            ballot per bit of the block number), plus the block's running
//            count in LDS
// Records: key = (event index in the chunk) << bs | (mark mod 2^bs) for blocks
// of 2^bs nodes (bs = 4, 6 or 7), t (float64),
// w = 1 / lambda (float32).  The dense-gradient kernels stream the records of
// two blocks (the block of their rows and the block of their columns)
// instead of filtering every event of the chunk.
#include "hk_device.h"
#include "hk_large.h"

namespace hk {

__global__ __launch_bounds__(64) void bucket_count(int64_t c0, int64_t c1, int32_t M, int32_t NB, int32_t bs,
                                                   const int32_t* __restrict__ marks, int32_t nseg,
                                                   int32_t* __restrict__ cnt) {
    extern __shared__ int32_t lc[];
    const int32_t s = blockIdx.x;
    const int lane = threadIdx.x;
    for (int32_t k = lane; k < NB; k += 64) lc[k] = 0;
    __syncthreads();
    const int64_t a = c0 + (int64_t)s * HK_SEG;
    const int64_t b = a + HK_SEG < c1 ? a + HK_SEG : c1;
    constexpr int NBT = HK_SEG / 64;
    int mks[NBT];   // all loads up front (past the end: a valid index, not counted)
#pragma unroll
    for (int u = 0; u < NBT; ++u) {
        const int64_t i = a + 64 * u + lane;
        mks[u] = marks[i < b ? i : b - 1];
    }
#pragma unroll
    for (int u = 0; u < NBT; ++u)
        if (a + 64 * u + lane < b) atomicAdd(&lc[clamp_mark(mks[u], M) >> bs], 1);
    __syncthreads();
    for (int32_t k = lane; k < NB; k += 64) cnt[(int64_t)k * nseg + s] = lc[k];
}

// inclusive sum of v over the lanes up to this one
__device__ __forceinline__ int32_t wave_incl_scan(int32_t v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t u = __shfl_up(v, d, 64);
        if (lane >= d) v += u;
    }
    return v;
}

// one workgroup of 1024 threads per block: exclusive scan of its counts
// over the segments (1024 at a time: lane scans, then the waves' totals),
// boff[block][segment] relative to the block's start, boff[block][nseg] =
// its total
__global__ __launch_bounds__(1024) void bucket_scan(int32_t nseg, const int32_t* __restrict__ cnt,
                                                    int32_t* __restrict__ boff) {
    __shared__ int32_t wt[16];
    const int32_t k = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    int32_t carry = 0;
    for (int32_t base = 0; base < nseg; base += 1024) {
        const int32_t s = base + tid;
        const int32_t v = s < nseg ? cnt[(int64_t)k * nseg + s] : 0;
        const int32_t incl = wave_incl_scan(v, lane);
        if (lane == 63) wt[wid] = incl;
        __syncthreads();
        int32_t before = 0, tot = 0;
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int32_t y = wt[u];
            before += u < wid ? y : 0;
            tot += y;
        }
        if (s < nseg) boff[(int64_t)k * (nseg + 1) + s] = carry + before + incl - v;
        carry += tot;
        __syncthreads();   // wt is reused
    }
    if (tid == 0) boff[(int64_t)k * (nseg + 1) + nseg] = carry;
}

// HK_BSW waves per segment, each with a contiguous quarter of its batches:
// (0) the first wave forms every block's start in the block-major output
// for this segment (the totals of the blocks before it, an exclusive scan
// of boff[.][nseg], plus boff[block][segment]); segment 0 also stores the
// blocks' bases in bbase for the dense-gradient kernels, (1) each wave
// counts its batches' events per block, (2) the counts become each wave's
// starting position per block (the block's start plus the counts of the
// waves before it), (3) each wave places its batches in order, an event's
// rank among its block's events in the batch from bit-sliced ballots.
#ifndef HK_BSW
#define HK_BSW 4
#endif
__global__ __launch_bounds__(64 * HK_BSW) void bucket_scatter(int64_t c0, int64_t c1, int32_t M, int32_t NB,
                                                              int32_t nbits, int32_t bs,
                                                              const double* __restrict__ t,
                                                              const int32_t* __restrict__ marks,
                                                              const float* __restrict__ wchunk, int32_t nseg,
                                                              const int32_t* __restrict__ boff,
                                                              int32_t* __restrict__ bbase,
                                                              uint32_t* __restrict__ bk_key, double* __restrict__ bk_t,
                                                              float* __restrict__ bk_w) {
    extern __shared__ int32_t cw[];   // [HK_BSW][NB]: counts, then running positions; then [NB] starts
    int32_t* lb = cw + HK_BSW * NB;
    const int32_t s = blockIdx.x;
    const int tid = threadIdx.x, lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int32_t k = tid; k < HK_BSW * NB; k += 64 * HK_BSW) cw[k] = 0;
    __syncthreads();
    const int64_t a = c0 + (int64_t)s * HK_SEG;
    const int64_t b = a + HK_SEG < c1 ? a + HK_SEG : c1;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    // this wave's marks, times and weights, all loads issued up front
    constexpr int NBT = HK_SEG / 64 / HK_BSW;
    static_assert(NBT * 64 * HK_BSW == HK_SEG, "whole batches per wave");
    const int64_t aw = a + (int64_t)wv * NBT * 64;
    int mks[NBT];
    double ts[NBT];
    float ws[NBT];
#pragma unroll
    for (int u = 0; u < NBT; ++u) {
        const int64_t i = aw + 64 * u + lane;
        const int64_t ic = i < b ? i : b - 1;
        mks[u] = clamp_mark(marks[ic], M);
        ts[u] = t[ic];
        ws[u] = wchunk[ic - c0];
    }
    if (wv == 0) {
        int32_t carry = 0;
        for (int32_t k0 = 0; k0 < NB; k0 += 64) {
            const int32_t k = k0 + lane;
            const int32_t tot = k < NB ? boff[(int64_t)k * (nseg + 1) + nseg] : 0;
            const int32_t off = k < NB ? boff[(int64_t)k * (nseg + 1) + s] : 0;
            const int32_t incl = wave_incl_scan(tot, lane);
            if (k < NB) {
                lb[k] = carry + incl - tot + off;
                if (s == 0) bbase[k] = carry + incl - tot;
            }
            carry += __shfl(incl, 63, 64);
        }
    }
    int32_t* run = cw + wv * NB;
#pragma unroll
    for (int u = 0; u < NBT; ++u)
        if (aw + 64 * u + lane < b) atomicAdd(&run[mks[u] >> bs], 1);
    __syncthreads();
    for (int32_t k = tid; k < NB; k += 64 * HK_BSW) {
        int32_t p = lb[k];
#pragma unroll
        for (int v = 0; v < HK_BSW; ++v) {
            const int32_t x = cw[v * NB + k];
            cw[v * NB + k] = p;
            p += x;
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < NBT; ++u) {
        const int64_t base = aw + 64 * u;
        if (base >= b) break;
        const int64_t i = base + lane;
        const bool v = i < b;
        const int mk = mks[u];
        const int blk = mk >> bs;
        // lanes with the same block: agree on every bit of the block number
        uint64_t same = __ballot(v);
        for (int bit = 0; bit < nbits; ++bit) {
            const uint64_t on = __ballot((blk >> bit) & 1);
            same &= ((blk >> bit) & 1) ? on : ~on;
        }
        const int rank = __builtin_popcountll(same & lt);
        const int32_t before = run[blk];
        if (v) {
            const int64_t pos = (int64_t)before + rank;
            bk_key[pos] = ((uint32_t)(i - c0) << bs) | (uint32_t)(mk & ((1 << bs) - 1));
            bk_t[pos] = ts[u];
            bk_w[pos] = ws[u];
        }
        lds_wait();   // every lane's read of the rank before the update
        if (v && (same & lt) == 0) run[blk] = before + __builtin_popcountll(same);
        lds_wait();   // the update before the next batch's reads
    }
}

// bs: log2 of the block width (4: 16 nodes, 6: 64, 7: 128; keys need
// (events per chunk) << bs < 2^32); records go to the given arrays
void bucket_chunk_into(const LargeArgs& A, int64_t c0, int64_t c1, int32_t nseg, const float* wchunk, int bs,
                       int32_t* cnt, int32_t* off, int32_t* base, uint32_t* key, double* tt, float* ww,
                       hipStream_t st, bool counted) {
    const int32_t nb = (A.M + (1 << bs) - 1) >> bs;
    int nbits = 0;
    while ((1 << nbits) < nb) ++nbits;
    const size_t lds = (size_t)nb * sizeof(int32_t);
    if (!counted)
        hipLaunchKernelGGL(bucket_count, dim3(nseg), dim3(64), lds, st, c0, c1, A.M, nb, bs, A.marks, nseg, cnt);
    hipLaunchKernelGGL(bucket_scan, dim3(nb), dim3(1024), 0, st, nseg, cnt, off);
    hipLaunchKernelGGL(bucket_scatter, dim3(nseg), dim3(64 * HK_BSW), lds * (HK_BSW + 1), st, c0, c1, A.M, nb, nbits,
                       bs, A.t, A.marks, wchunk, nseg, off, base, key, tt, ww);
}

void bucket_chunk(LargeArgs& A, int64_t c0, int64_t c1, int32_t nseg, const float* wchunk, int bs, hipStream_t st) {
    bucket_chunk_into(A, c0, c1, nseg, wchunk, bs, A.bk_cnt, A.bk_off, A.bk_base, A.bk_key, A.bk_t, A.bk_w, st);
}

}  // namespace hk
