// Simulation of event sequences on the GPU: the branching (cluster)
// representation of the linear exponential Hawkes process (the construction
// behind the paper's synthetic studies, section "Results").  Input side of
// the evaluation path; nothing here is used by the likelihood kernels.
//
// On [0, T0]:
//   immigrants  node p's events of the baseline rate mu_p form a Poisson
//               process: [0, T0] is cut into cells of expected count <= 2, each
//               cell's count is Poisson, its events uniform in the cell;
//   children    an event of node q has Poisson(sum_{k,p} alpha[k][p][q])
//               children; a child is of (kernel k, node p) with probability
//               alpha[k][p][q] / that sum and follows its parent after an
//               Exp(beta) delay (beta_k with a decay per kernel, beta_p with
//               a decay per target node); children after T0 are dropped;
//   generations repeat until one has no children, then all events are
//   sorted by time (LSD radix sort of the float64 bit patterns, stable).
// Every random number comes from Philox4x64-10 (Salmon, Moraes, Dror and Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC 2011) keyed by the seed,
// with a counter naming what it is for (a cell, an event's child count, a
// child), so the output depends only on the seed and the parameters, never
// on the launch shape, and counts can be drawn twice (a sizing pass, then a
// writing pass) with the same result.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>
#include <vector>
#include "hk_device.h"
#include "hk_internal.h"
#include "../../include/hawkes.h"

namespace hk {

// ---------------------------------------------------------------- Philox4x64-10
struct U64x4 {
    uint64_t v[4];
};

// 64 x 64 -> 128-bit product from 32-bit halves (the same code on host and device)
__host__ __device__ inline void mulhilo64(uint64_t a, uint64_t b, uint64_t* hi, uint64_t* lo) {
    const uint64_t al = (uint32_t)a, ah = a >> 32, bl = (uint32_t)b, bh = b >> 32;
    const uint64_t p0 = al * bl, p1 = al * bh, p2 = ah * bl, p3 = ah * bh;
    const uint64_t mid = (p0 >> 32) + (uint32_t)p1 + (uint32_t)p2;
    *hi = p3 + (p1 >> 32) + (p2 >> 32) + (mid >> 32);
    *lo = a * b;
}

// ten rounds of the Philox S-box on a 4 x 64-bit counter under a 2 x 64-bit key
__host__ __device__ inline U64x4 philox4x64_10(U64x4 c, uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
    for (int r = 0; r < 10; ++r) {
        uint64_t hi0, lo0, hi1, lo1;
        mulhilo64(M0, c.v[0], &hi0, &lo0);
        mulhilo64(M1, c.v[2], &hi1, &lo1);
        U64x4 n;
        n.v[0] = hi1 ^ c.v[1] ^ k0;
        n.v[1] = lo1;
        n.v[2] = hi0 ^ c.v[3] ^ k1;
        n.v[3] = lo0;
        c = n;
        k0 += W0;
        k1 += W1;
    }
    return c;
}

// uniform in (0, 1) from the top 53 bits
__device__ __forceinline__ double unit_open(uint64_t x) {
    return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

// counter purposes
enum : uint64_t { SIM_CELL = 1, SIM_IMM = 2, SIM_NCHILD = 3, SIM_CHILD = 4 };

__device__ __forceinline__ U64x4 draw(uint64_t seed, uint64_t a, uint64_t b, uint64_t purpose, uint64_t salt) {
    U64x4 c;
    c.v[0] = a;
    c.v[1] = b;
    c.v[2] = purpose;
    c.v[3] = salt;
    return philox4x64_10(c, seed, 0x5851F42D4C957F2Dull);
}

// Poisson(lam) by inversion of its distribution function, one uniform per
// part of at most 16 in the mean (a Poisson sum of parts is Poisson)
__device__ int64_t poisson(double lam, uint64_t seed, uint64_t a, uint64_t b, uint64_t purpose) {
    int64_t total = 0;
    uint64_t part = 0;
    while (lam > 0.0) {
        const double l = lam < 16.0 ? lam : 16.0;
        lam -= l;
        const U64x4 r = draw(seed, a, b, purpose, part++);
        const double u = unit_open(r.v[0]);
        double p = exp(-l), F = p;
        int64_t k = 0;
        while (u > F && k < 1000) {
            ++k;
            p *= l / (double)k;
            F += p;
        }
        total += k;
    }
    return total;
}

// ---------------------------------------------------------------- setup
// cells of node p: ceil(mu_p T0 / 2) cells of equal width (expected count <= 2)
__global__ void sim_cells(int32_t M, double T0, const float* __restrict__ mu, int64_t* __restrict__ ncell) {
    const int32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= M) return;
    const double lam = (double)mu[p] * T0;
    ncell[p] = lam > 0.0 ? (int64_t)ceil(lam / 2.0) : 0;
}

// Compressed columns of the K M x M interaction matrices stacked as K M rows:
// for source q, the rows r = k M + p with alpha[k][p][q] != 0 and the running
// sums of those entries (the child-type distribution of a q event).
__global__ __launch_bounds__(64) void sim_col_count(int32_t M, int32_t K, const float* __restrict__ alpha,
                                                    int64_t* __restrict__ cnt) {
    const int32_t q = blockIdx.x;
    int64_t c = 0;
    for (int64_t r = threadIdx.x; r < (int64_t)K * M; r += 64) c += alpha[r * M + q] != 0.0f;
    for (int off = 32; off > 0; off >>= 1) c += __shfl_down(c, off, 64);
    if (threadIdx.x == 0) cnt[q] = c;
}

__global__ __launch_bounds__(64) void sim_col_fill(int32_t M, int32_t K, const float* __restrict__ alpha,
                                                   const int64_t* __restrict__ col_off, int32_t* __restrict__ rows,
                                                   double* __restrict__ cum, double* __restrict__ colsum) {
    const int32_t q = blockIdx.x;
    const int lane = threadIdx.x;
    int64_t o = col_off[q];
    double run = 0.0;
    for (int64_t r0 = 0; r0 < (int64_t)K * M; r0 += 64) {
        const int64_t r = r0 + lane;
        const float a = r < (int64_t)K * M ? alpha[r * M + q] : 0.0f;
        const uint64_t nz = __ballot(a != 0.0f);
        // running sum in row order: an inclusive scan of the wave's entries
        double v = (double)a;
        for (int d = 1; d < 64; d <<= 1) {
            const double u = __shfl_up(v, d, 64);
            if (lane >= d) v += u;
        }
        if (a != 0.0f) {
            const int32_t k = (int32_t)__builtin_popcountll(nz & (lane ? (~0ull >> (64 - lane)) : 0ull));
            rows[o + k] = (int32_t)r;
            cum[o + k] = run + v;
        }
        run += __shfl(v, 63, 64);
        o += __builtin_popcountll(nz);
    }
    if (lane == 0) colsum[q] = run;
}

// ---------------------------------------------------------------- scans
// exclusive scan of n int64 counts into off[0..n] (off[n] = total), in
// tiles of 1024: per-tile sums, a scan of the tile sums, the tiles' scans
__global__ __launch_bounds__(256) void sim_tile_sum(int64_t n, const int64_t* __restrict__ c,
                                                    int64_t* __restrict__ tsum) {
    __shared__ int64_t sh[256];
    const int64_t base = (int64_t)blockIdx.x * 1024;
    int64_t v = 0;
    for (int j = 0; j < 4; ++j) {
        const int64_t i = base + j * 256 + threadIdx.x;
        if (i < n) v += c[i];
    }
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) tsum[blockIdx.x] = sh[0];
}

// one workgroup: exclusive scan of the tile sums in place, total at [nt]
__global__ __launch_bounds__(1024) void sim_scan_tiles(int64_t nt, int64_t* __restrict__ tsum) {
    __shared__ int64_t sh[1024];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t b = 0; b < nt; b += 1024) {
        const int64_t i = b + threadIdx.x;
        const int64_t v = i < nt ? tsum[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int d = 1; d < 1024; d <<= 1) {
            const int64_t a = (int)threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
            __syncthreads();
            sh[threadIdx.x] += a;
            __syncthreads();
        }
        if (i < nt) tsum[i] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += sh[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) tsum[nt] = carry;
}

__global__ __launch_bounds__(256) void sim_tile_scan(int64_t n, const int64_t* __restrict__ c,
                                                     const int64_t* __restrict__ tsum, int64_t* __restrict__ off) {
    __shared__ int64_t sh[1024];
    const int64_t base = (int64_t)blockIdx.x * 1024;
    for (int j = 0; j < 4; ++j) {
        const int64_t i = base + j * 256 + threadIdx.x;
        sh[j * 256 + threadIdx.x] = i < n ? c[i] : 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t run = tsum[blockIdx.x];
        for (int j = 0; j < 1024; ++j) {
            const int64_t v = sh[j];
            sh[j] = run;
            run += v;
        }
    }
    __syncthreads();
    for (int j = 0; j < 4; ++j) {
        const int64_t i = base + j * 256 + threadIdx.x;
        if (i < n) off[i] = sh[j * 256 + threadIdx.x];
    }
    if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) off[n] = tsum[gridDim.x];
}

// ---------------------------------------------------------------- immigrants
__device__ __forceinline__ int32_t find_node(const int64_t* __restrict__ off, int32_t M, int64_t x) {
    int32_t lo = 0, hi = M - 1;   // largest p with off[p] <= x
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// cell c of node p covers [b w, min((b + 1) w, T0)) with w = T0 / ncell_p
template <bool FILL>
__global__ void sim_imm(int32_t M, double T0, uint64_t seed, const float* __restrict__ mu,
                        const int64_t* __restrict__ cell_off, int64_t* __restrict__ cnt,
                        const int64_t* __restrict__ ev_off, double* __restrict__ t_out,
                        int32_t* __restrict__ m_out) {
    const int64_t ncell = cell_off[M];
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncell;
         c += (int64_t)gridDim.x * blockDim.x) {
        const int32_t p = find_node(cell_off, M, c);
        const int64_t nc = cell_off[p + 1] - cell_off[p];
        const int64_t b = c - cell_off[p];
        const double w = T0 / (double)nc;
        const double lo = (double)b * w;
        const double hi = b + 1 == nc ? T0 : (double)(b + 1) * w;
        const int64_t k = poisson((double)mu[p] * (hi - lo), seed, (uint64_t)c, 0, SIM_CELL);
        if (!FILL) {
            cnt[c] = k;
            continue;
        }
        const int64_t o = ev_off[c];
        for (int64_t j = 0; j < k; ++j) {
            const U64x4 r = draw(seed, (uint64_t)c, (uint64_t)j, SIM_IMM, 0);
            double x = lo + unit_open(r.v[0]) * (hi - lo);
            x = x < hi ? x : lo;   // rounding at the cell's end stays inside
            t_out[o + j] = x;
            m_out[o + j] = p;
        }
    }
}

// ---------------------------------------------------------------- generations
// Parent i (index in the unsorted event array, parents [s, e)): its
// children, in order, each with its (kernel, node) and delay; kept if before
// T0.  COUNT writes the kept count, FILL writes the kept children at ev_off.
template <bool FILL>
__global__ void sim_children(int64_t s, int64_t e, int32_t M, double T0, uint64_t seed, int per_target,
                             const float* __restrict__ beta, const int64_t* __restrict__ col_off,
                             const int32_t* __restrict__ rows, const double* __restrict__ cum,
                             const double* __restrict__ colsum, int64_t* __restrict__ cnt,
                             const int64_t* __restrict__ ev_off, int64_t out0, double* __restrict__ t_ev,
                             int32_t* __restrict__ m_ev) {
    for (int64_t i = s + blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < e;
         i += (int64_t)gridDim.x * blockDim.x) {
        const double ti = t_ev[i];
        const int32_t q = clamp_mark(m_ev[i], M);
        const int64_t nch = poisson(colsum[q], seed, (uint64_t)i, 0, SIM_NCHILD);
        const int64_t a = col_off[q], b = col_off[q + 1];
        int64_t kept = 0;
        int64_t o = FILL ? out0 + ev_off[i - s] : 0;
        for (int64_t j = 0; j < nch && b > a; ++j) {
            const U64x4 r = draw(seed, (uint64_t)i, (uint64_t)j, SIM_CHILD, 0);
            // (kernel, node) by the running sums of column q
            const double u = unit_open(r.v[0]) * colsum[q];
            int64_t lo = a, hi = b - 1;   // first entry with cum > u
            while (lo < hi) {
                const int64_t mid = (lo + hi) >> 1;
                if (cum[mid] > u) hi = mid; else lo = mid + 1;
            }
            const int32_t row = rows[lo];
            const int32_t k = row / M, p = row - k * M;
            const double rate = (double)beta[per_target ? p : k];
            const double tc = ti - log(unit_open(r.v[1])) / rate;
            if (tc <= T0) {
                if (FILL) {
                    t_ev[o] = tc;
                    m_ev[o] = p;
                    ++o;
                }
                ++kept;
            }
        }
        if (!FILL) cnt[i - s] = kept;
    }
}

// ---------------------------------------------------------------- radix sort
// LSD radix sort of (time bits, mark) by 8-bit digits, stable: per tile of
// 4096 keys a digit histogram, one exclusive scan over (digit, tile), then
// each tile scatters its keys in order (ranks among equal digits from
// bit-sliced ballots within a wave, wave counts and running digit bases in LDS).
#define SIM_TILE 4096

__global__ __launch_bounds__(256) void sim_rs_hist(int64_t n, int shift, const uint64_t* __restrict__ key,
                                                   int64_t ntile, int64_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * SIM_TILE;
    for (int j = 0; j < SIM_TILE / 256; ++j) {
        const int64_t i = base + j * 256 + threadIdx.x;
        if (i < n) atomicAdd(&h[(key[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntile + blockIdx.x] = h[threadIdx.x];
}

__global__ __launch_bounds__(256) void sim_rs_scatter(int64_t n, int shift, const uint64_t* __restrict__ key,
                                                      const int32_t* __restrict__ val, int64_t ntile,
                                                      const int64_t* __restrict__ hoff, uint64_t* __restrict__ key2,
                                                      int32_t* __restrict__ val2) {
    __shared__ int64_t dbase[256];
    __shared__ uint32_t wcnt[4][256];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    dbase[threadIdx.x] = hoff[(int64_t)threadIdx.x * ntile + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * SIM_TILE;
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    for (int j = 0; j < SIM_TILE / 256; ++j) {
        for (int w = 0; w < 4; ++w) wcnt[w][threadIdx.x] = 0;
        __syncthreads();
        const int64_t i = base + j * 256 + threadIdx.x;
        const bool v = i < n;
        const uint64_t kk = v ? key[i] : 0;
        const int32_t vv = v ? val[i] : 0;
        const uint32_t d = (uint32_t)(kk >> shift) & 255u;
        // lanes of this wave with the same digit
        uint64_t eq = __ballot(v);
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bb = __ballot(v && ((d >> bit) & 1u));
            eq &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__builtin_popcountll(eq & below);
        if (v && rank == 0) wcnt[wv][d] = (uint32_t)__builtin_popcountll(eq);
        __syncthreads();
        if (v) {
            int64_t pos = dbase[d] + rank;
            for (int w = 0; w < wv; ++w) pos += wcnt[w][d];
            key2[pos] = kk;
            val2[pos] = vv;
        }
        __syncthreads();
        dbase[threadIdx.x] += wcnt[0][threadIdx.x] + wcnt[1][threadIdx.x] + wcnt[2][threadIdx.x] +
                              wcnt[3][threadIdx.x];
        __syncthreads();
    }
}

// ---------------------------------------------------------------- host
struct SimLayout {
    int64_t *ncell, *cell_off, *col_cnt, *col_off, *cnt, *off, *tsum, *hist, *hoff, *htsum;
    int32_t* rows;
    double *cum, *colsum;
    uint64_t* key2;
    int32_t* val2;
};

static int64_t tiles_of(int64_t n, int64_t t) { return (n + t - 1) / t; }

static size_t sim_layout(SimLayout& L, int32_t M, int32_t K, int64_t cap, void* ws) {
    Carve c(ws, 0);
    const int64_t ntile = tiles_of(cap, SIM_TILE);
    const int64_t nh = 256 * ntile;
    L.ncell = c.take<int64_t>(M);
    L.cell_off = c.take<int64_t>(M + 1);
    L.col_cnt = c.take<int64_t>(M);
    L.col_off = c.take<int64_t>(M + 1);
    L.rows = c.take<int32_t>((size_t)K * M * M);
    L.cum = c.take<double>((size_t)K * M * M);
    L.colsum = c.take<double>(M);
    L.cnt = c.take<int64_t>(cap + 1);
    L.off = c.take<int64_t>(cap + 2);
    L.tsum = c.take<int64_t>(tiles_of((cap > M ? cap : M) + 1, 1024) + 2);
    L.hist = c.take<int64_t>(nh);
    L.hoff = c.take<int64_t>(nh + 1);
    L.htsum = c.take<int64_t>(tiles_of(nh, 1024) + 2);
    L.key2 = c.take<uint64_t>(cap);
    L.val2 = c.take<int32_t>(cap);
    return c.off + 256;
}

static void scan_launch(int64_t n, const int64_t* cnt, int64_t* tsum, int64_t* off, hipStream_t st) {
    const int64_t nt = tiles_of(n, 1024) > 0 ? tiles_of(n, 1024) : 1;
    hipLaunchKernelGGL(sim_tile_sum, dim3((unsigned)nt), dim3(256), 0, st, n, cnt, tsum);
    hipLaunchKernelGGL(sim_scan_tiles, dim3(1), dim3(1024), 0, st, nt, tsum);
    hipLaunchKernelGGL(sim_tile_scan, dim3((unsigned)nt), dim3(256), 0, st, n, cnt, tsum, off);
}

static unsigned grid_for(int64_t n, int bs) {
    const int64_t g = (n + bs - 1) / bs;
    return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace hk

using namespace hk;

extern "C" {

void hawkes_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
    U64x4 c;
    for (int i = 0; i < 4; ++i) c.v[i] = ctr[i];
    const U64x4 r = philox4x64_10(c, key[0], key[1]);
    for (int i = 0; i < 4; ++i) out[i] = r.v[i];
}

size_t hawkes_simulate_workspace_bytes(int32_t m, int32_t k, int64_t capacity) {
    if (m < 1 || k < 1 || k > HAWKES_MAX_KERNELS || capacity < 1 || capacity > ((int64_t)1 << 40)) return 0;
    SimLayout L;
    return sim_layout(L, m, k, capacity, nullptr);
}

hawkes_status hawkes_simulate(int32_t m, int32_t k, int32_t beta_mode, const float* mu, const float* alpha,
                              const float* beta, double T0, uint64_t seed, int64_t capacity, double* t_out,
                              int32_t* marks_out, int64_t* n_out, void* workspace, size_t workspace_bytes,
                              hipStream_t stream) {
    if (m < 1 || k < 1 || k > HAWKES_MAX_KERNELS || !mu || !alpha || !beta || !t_out || !marks_out || !n_out)
        return HAWKES_EINVAL;
    if (beta_mode != HAWKES_BETA_SHARED && beta_mode != HAWKES_BETA_PER_TARGET) return HAWKES_EINVAL;
    if (beta_mode == HAWKES_BETA_PER_TARGET && k != 1) return HAWKES_EINVAL;
    if (!(T0 >= 0.0) || !isfinite(T0) || capacity < 1) return HAWKES_EINVAL;
    if ((int64_t)k * m * m > ((int64_t)1 << 31)) return HAWKES_EINVAL;
    const size_t need = hawkes_simulate_workspace_bytes(m, k, capacity);
    if (!workspace || need == 0 || workspace_bytes < need || ((uintptr_t)workspace & 255) != 0)
        return HAWKES_EWORKSPACE;
    SimLayout L;
    sim_layout(L, m, k, capacity, workspace);
    const hipStream_t st = stream;
    auto d2h = [&](int64_t* dst, const int64_t* src) -> bool {
        if (hipMemcpyAsync(dst, src, sizeof(int64_t), hipMemcpyDeviceToHost, st) != hipSuccess) return false;
        return hipStreamSynchronize(st) == hipSuccess;
    };
    // child-type distributions per source, cells of the baseline rates
    hipLaunchKernelGGL(sim_col_count, dim3((unsigned)m), dim3(64), 0, st, m, k, alpha, L.col_cnt);
    scan_launch(m, L.col_cnt, L.tsum, L.col_off, st);
    hipLaunchKernelGGL(sim_col_fill, dim3((unsigned)m), dim3(64), 0, st, m, k, alpha, L.col_off, L.rows, L.cum,
                       L.colsum);
    hipLaunchKernelGGL(sim_cells, dim3(grid_for(m, 256)), dim3(256), 0, st, m, T0, mu, L.ncell);
    scan_launch(m, L.ncell, L.tsum, L.cell_off, st);
    int64_t ncell = 0;
    if (!d2h(&ncell, L.cell_off + m)) return HAWKES_EDEVICE;
    // immigrants: counts, offsets, events
    int64_t n = 0;
    if (ncell > 0) {
        if (ncell > capacity) {
            // the cell counts need as many slots as cells
            *n_out = ncell;
            return HAWKES_EWORKSPACE;
        }
        hipLaunchKernelGGL((sim_imm<false>), dim3(grid_for(ncell, 256)), dim3(256), 0, st, m, T0, seed, mu,
                           L.cell_off, L.cnt, (const int64_t*)nullptr, (double*)nullptr, (int32_t*)nullptr);
        scan_launch(ncell, L.cnt, L.tsum, L.off, st);
        if (!d2h(&n, L.off + ncell)) return HAWKES_EDEVICE;
        if (n > capacity) {
            *n_out = n;
            return HAWKES_EWORKSPACE;
        }
        hipLaunchKernelGGL((sim_imm<true>), dim3(grid_for(ncell, 256)), dim3(256), 0, st, m, T0, seed, mu,
                           L.cell_off, L.cnt, L.off, t_out, marks_out);
    }
    // generations: the children of events [s, e) go to [e, e + kids)
    int64_t s = 0, e = n;
    while (e > s) {
        const int64_t np = e - s;
        hipLaunchKernelGGL((sim_children<false>), dim3(grid_for(np, 256)), dim3(256), 0, st, s, e, m, T0, seed,
                           beta_mode == HAWKES_BETA_PER_TARGET ? 1 : 0, beta, L.col_off, L.rows, L.cum, L.colsum,
                           L.cnt, (const int64_t*)nullptr, (int64_t)0, t_out, marks_out);
        scan_launch(np, L.cnt, L.tsum, L.off, st);
        int64_t kids = 0;
        if (!d2h(&kids, L.off + np)) return HAWKES_EDEVICE;
        if (e + kids > capacity) {
            *n_out = e + kids;
            return HAWKES_EWORKSPACE;
        }
        if (kids > 0)
            hipLaunchKernelGGL((sim_children<true>), dim3(grid_for(np, 256)), dim3(256), 0, st, s, e, m, T0, seed,
                               beta_mode == HAWKES_BETA_PER_TARGET ? 1 : 0, beta, L.col_off, L.rows, L.cum,
                               L.colsum, L.cnt, L.off, e, t_out, marks_out);
        s = e;
        e += kids;
    }
    n = e;
    // sort by time: 8 passes of 8 bits over the float64 bit patterns (times
    // are >= 0, so their bit patterns order like the values); the even pass
    // count leaves the result in t_out / marks_out
    if (n > 1) {
        const int64_t ntile = tiles_of(n, SIM_TILE);
        const int64_t nh = 256 * ntile;
        uint64_t* ka = reinterpret_cast<uint64_t*>(t_out);
        int32_t* va = marks_out;
        uint64_t* kb = L.key2;
        int32_t* vb = L.val2;
        for (int pass = 0; pass < 8; ++pass) {
            const int shift = 8 * pass;
            hipLaunchKernelGGL(sim_rs_hist, dim3((unsigned)ntile), dim3(256), 0, st, n, shift, ka, ntile, L.hist);
            scan_launch(nh, L.hist, L.htsum, L.hoff, st);
            hipLaunchKernelGGL(sim_rs_scatter, dim3((unsigned)ntile), dim3(256), 0, st, n, shift, ka, va, ntile,
                               L.hoff, kb, vb);
            uint64_t* tk = ka;
            ka = kb;
            kb = tk;
            int32_t* tv = va;
            va = vb;
            vb = tv;
        }
    }
    if (hipGetLastError() != hipSuccess) return HAWKES_EDEVICE;
    if (hipStreamSynchronize(st) != hipSuccess) return HAWKES_EDEVICE;
    *n_out = n;
    return HAWKES_OK;
}

}  // extern "C"
