// Per-chunk partition of the events by node block (16, 64 or 128 nodes per block),
// stable in event order: a counting sort in three steps.
//   count    one wave per segment: events per (block, segment)
//   scan     one workgroup per block: start of every (block, segment) run
//            within the block, boff[block][segment] ([block][nseg] = the
//            block's size), then bbase[block], the block's start in the
//            block-major output
//   scatter  one wave per segment: each event's rank among the events of its
//            block in the same 64-event batch comes from bit-sliced ballots
//            (one ballot per bit of the block number), plus the block's
//            running count in LDS
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

// one workgroup per block: exclusive scan of its counts over the segments,
// boff[block][segment] relative to the block's start, boff[block][nseg] = its
// total
__global__ __launch_bounds__(256) void bucket_scan(int32_t nseg, const int32_t* __restrict__ cnt,
                                                   int32_t* __restrict__ boff, int32_t* __restrict__ done,
                                                   int32_t* __restrict__ bbase) {
    __shared__ int32_t sh[256];
    const int32_t k = blockIdx.x;
    const int tid = threadIdx.x;
    int32_t carry = 0;
    for (int32_t base = 0; base < nseg; base += 256) {
        const int32_t s = base + tid;
        const int32_t v = s < nseg ? cnt[(int64_t)k * nseg + s] : 0;
        sh[tid] = v;
        __syncthreads();
        for (int d = 1; d < 256; d <<= 1) {
            const int32_t u = tid >= d ? sh[tid - d] : 0;
            __syncthreads();
            sh[tid] += u;
            __syncthreads();
        }
        if (s < nseg) boff[(int64_t)k * (nseg + 1) + s] = carry + sh[tid] - v;
        carry += sh[255];
        __syncthreads();
    }
    if (tid == 0) boff[(int64_t)k * (nseg + 1) + nseg] = carry;
    if (!done) return;
    // the last block to finish forms the blocks' bases (exclusive scan of
    // their totals), instead of a launch of bucket_base
    __shared__ int last;
    __threadfence();
    if (tid == 0) last = atomicAdd(done, 1) == (int)gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    const volatile int32_t* bo = boff;
    const int32_t NB = (int32_t)gridDim.x;
    int32_t run = 0;
    for (int32_t base = 0; base < NB; base += 256) {
        const int32_t b = base + tid;
        const int32_t v = b < NB ? bo[(int64_t)b * (nseg + 1) + nseg] : 0;
        sh[tid] = v;
        __syncthreads();
        for (int d = 1; d < 256; d <<= 1) {
            const int32_t u = tid >= d ? sh[tid - d] : 0;
            __syncthreads();
            sh[tid] += u;
            __syncthreads();
        }
        if (b < NB) bbase[b] = run + sh[tid] - v;
        run += sh[255];
        __syncthreads();
    }
    if (tid == 0) *done = 0;
}

// bbase[block] = number of records of the blocks before it (one workgroup,
// exclusive scan of the blocks' totals 256 at a time)
__global__ __launch_bounds__(256) void bucket_base(int32_t NB, int32_t nseg, const int32_t* __restrict__ boff,
                                                   int32_t* __restrict__ bbase) {
    __shared__ int32_t sh[256];
    const int tid = threadIdx.x;
    int32_t carry = 0;
    for (int32_t base = 0; base < NB; base += 256) {
        const int32_t k = base + tid;
        const int32_t v = k < NB ? boff[(int64_t)k * (nseg + 1) + nseg] : 0;
        sh[tid] = v;
        __syncthreads();
        for (int d = 1; d < 256; d <<= 1) {
            const int32_t u = tid >= d ? sh[tid - d] : 0;
            __syncthreads();
            sh[tid] += u;
            __syncthreads();
        }
        if (k < NB) bbase[k] = carry + sh[tid] - v;
        carry += sh[255];
        __syncthreads();
    }
}

__global__ __launch_bounds__(64) void bucket_scatter(int64_t c0, int64_t c1, int32_t M, int32_t NB, int32_t nbits,
                                                     int32_t bs,
                                                     const double* __restrict__ t,
                                                     const int32_t* __restrict__ marks,
                                                     const float* __restrict__ wchunk, int32_t nseg,
                                                     const int32_t* __restrict__ boff,
                                                     const int32_t* __restrict__ bbase,
                                                     uint32_t* __restrict__ bk_key, double* __restrict__ bk_t,
                                                     float* __restrict__ bk_w) {
    extern __shared__ int32_t run[];
    const int32_t s = blockIdx.x;
    const int lane = threadIdx.x;
    for (int32_t k = lane; k < NB; k += 64) run[k] = 0;
    __syncthreads();
    const int64_t a = c0 + (int64_t)s * HK_SEG;
    const int64_t b = a + HK_SEG < c1 ? a + HK_SEG : c1;
    const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
    // the segment's marks, times and weights, all loads issued up front
    constexpr int NBT = HK_SEG / 64;
    int mks[NBT];
    double ts[NBT];
    float ws[NBT];
#pragma unroll
    for (int u = 0; u < NBT; ++u) {
        const int64_t i = a + 64 * u + lane;
        const int64_t ic = i < b ? i : b - 1;
        mks[u] = marks[ic];
        ts[u] = t[ic];
        ws[u] = wchunk[ic - c0];
    }
#pragma unroll
    for (int u = 0; u < NBT; ++u) {
        const int64_t base = a + 64 * u;
        if (base >= b) break;
        const int64_t i = base + lane;
        const bool v = i < b;
        const int mk = clamp_mark(mks[u], M);
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
            const int64_t pos = (int64_t)bbase[blk] + boff[(int64_t)blk * (nseg + 1) + s] + before + rank;
            bk_key[pos] = ((uint32_t)(i - c0) << bs) | (uint32_t)(mk & ((1 << bs) - 1));
            bk_t[pos] = ts[u];
            bk_w[pos] = ws[u];
        }
        __syncthreads();
        if (v && (same & lt) == 0) run[blk] = before + __builtin_popcountll(same);
        __syncthreads();
    }
}

// bs: log2 of the block width (4: 16 nodes, 6: 64, 7: 128; keys need
// (events per chunk) << bs < 2^32); records go to the given arrays
void bucket_chunk_into(const LargeArgs& A, int64_t c0, int64_t c1, int32_t nseg, const float* wchunk, int bs,
                       int32_t* cnt, int32_t* off, int32_t* base, uint32_t* key, double* tt, float* ww,
                       hipStream_t st, bool counted, int32_t* done) {
    const int32_t nb = (A.M + (1 << bs) - 1) >> bs;
    int nbits = 0;
    while ((1 << nbits) < nb) ++nbits;
    const size_t lds = (size_t)nb * sizeof(int32_t);
    if (!counted)
        hipLaunchKernelGGL(bucket_count, dim3(nseg), dim3(64), lds, st, c0, c1, A.M, nb, bs, A.marks, nseg, cnt);
    hipLaunchKernelGGL(bucket_scan, dim3(nb), dim3(256), 0, st, nseg, cnt, off, done, base);
    if (!done) hipLaunchKernelGGL(bucket_base, dim3(1), dim3(256), 0, st, nb, nseg, off, base);
    hipLaunchKernelGGL(bucket_scatter, dim3(nseg), dim3(64), lds, st, c0, c1, A.M, nb, nbits, bs, A.t, A.marks, wchunk,
                       nseg, off, base, key, tt, ww);
}

void bucket_chunk(LargeArgs& A, int64_t c0, int64_t c1, int32_t nseg, const float* wchunk, int bs, hipStream_t st) {
    bucket_chunk_into(A, c0, c1, nseg, wchunk, bs, A.bk_cnt, A.bk_off, A.bk_base, A.bk_key, A.bk_t, A.bk_w, st);
}

}  // namespace hk
