// support.hip -- particle bookkeeping and snapshot conversion kernels:
//   * wavefront compaction of the active-particle list (ballot + mbcnt prefix,
//     one atomic per wave);
//   * a counting sort of the active particles by grid tile (and level in 3D),
//     which also drops particles that are no longer active;
//   * conversion of float32 / float64 snapshots into the interleaved node layout
//     of a device slot, including bfloat16 (round to nearest even) and float16
//     with a power-of-two scale per (level, variable).
#include "lp_internal.h"

namespace lp {

namespace {

__global__ void k_fill_u32(uint32_t *p, uint32_t v, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void k_iota(uint32_t *p, size_t n)
{
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = (uint32_t)i;
}

uint32_t grid_blocks(size_t n, uint32_t threads, uint32_t cap = 1u << 16)
{
    size_t b = (n + threads - 1) / threads;
    if (b == 0)
        b = 1;
    return (uint32_t)(b > cap ? cap : b);
}

// Keep the ids whose status is still 0.  Each wave finds its survivors with a
// ballot and ranks them with mbcnt; the waves of a block add up their counts in LDS
// and the block reserves room in the output with a single atomic.  A thread takes
// kCompactItems entries, kCompactThreads apart, so that a block covers 4096 entries
// per atomic: atomics on the one counter serialise (about 12 ns each here), and with
// one per 1024 entries they were most of the kernel's time.  Survivors keep their
// order within a block (entry, then wave, then lane).
constexpr int kCompactThreads = 1024, kCompactItems = 4;

__global__ __launch_bounds__(kCompactThreads) void k_compact(const uint32_t *order_in,
                                                             const uint32_t *n_in,
                                                             const uint8_t *status,
                                                             uint32_t *order_out,
                                                             uint32_t *n_out)
{
    constexpr int W = kCompactThreads / 64;
    __shared__ uint32_t wcount[kCompactItems * W];
    __shared__ uint32_t block_base;
    const uint32_t n = *n_in;
    const size_t base = (size_t)blockIdx.x * kCompactThreads * kCompactItems;
    const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63;
    uint32_t id[kCompactItems], rank[kCompactItems];
    bool keep[kCompactItems];
#pragma unroll
    for (int j = 0; j < kCompactItems; ++j) {
        const size_t k = base + (size_t)j * kCompactThreads + threadIdx.x;
        id[j] = 0;
        keep[j] = false;
        if (k < n) {
            id[j] = order_in[k];
            keep[j] = status[id[j]] == 0;
        }
        const uint64_t mask = __ballot(keep[j]);
        rank[j] = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                            __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
        if (lane == 0)
            wcount[j * W + wid] = (uint32_t)__popcll(mask);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int w = 0; w < kCompactItems * W; ++w) {
            const uint32_t c = wcount[w];
            wcount[w] = tot;
            tot += c;
        }
        block_base = tot ? atomicAdd(n_out, tot) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kCompactItems; ++j)
        if (keep[j])
            order_out[block_base + wcount[j * W + wid] + rank[j]] = id[j];
}

// Runs of equal keys inside a wave (the order is nearly sorted already): each lane
// learns the lane that starts its run and the run length, so one lane per run can
// do the atomic for the whole run.
__device__ inline void wave_runs(uint32_t key, bool valid, int &start, uint32_t &len)
{
    const int lane = threadIdx.x & 63;
    const uint32_t prev = __shfl_up(key, 1, 64);
    const bool prev_valid = __shfl_up(valid ? 1 : 0, 1, 64) != 0;
    const bool is_start = valid && (lane == 0 || !prev_valid || prev != key);
    // lanes that are not valid also end runs
    const uint64_t starts = __ballot(is_start) | __ballot(!valid);
    const uint64_t below = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
    const uint64_t at_or_below = starts & below;
    start = at_or_below ? 63 - __clzll((long long)at_or_below) : lane;
    const uint64_t above = starts & ~below;
    const int next = above ? __ffsll((unsigned long long)above) - 1 : 64;
    len = (uint32_t)(next - lane);  // meaningful on the start lane
}

__device__ inline int cell_of(const AxisDev &a, double x)
{
    int g;
    if (a.uniform) {
        g = (int)((x - a.lo) * a.ginv);
    } else {
        int b = (int)((x - a.lo) * a.ginv);
        b = b < kGuessBins - 1 ? b : kGuessBins - 1;
        b = b < 0 ? 0 : b;
        g = a.guess[b];
    }
    g = g < 0 ? 0 : (g > a.n - 2 ? a.n - 2 : g);
    while (g > 0 && a.c[g] > x)
        --g;
    while (g < a.n - 2 && a.c[g + 1] <= x)
        ++g;
    return g;
}

// Sort key: tile index (16 x 16 cells, row-major over tiles), times the level in
// 3D; with `cells` (2D) the tile index times 256 plus the cell's row-major index in its
// tile, so that a wave's particles share cells, not only a tile.  Inactive particles get
// no key and are dropped by the sort.
__global__ __launch_bounds__(256) void k_sort_keys(GridDev g, const double *x, const double *y,
                                                   const double *z, const uint8_t *status,
                                                   const uint32_t *order, const uint32_t *n_in,
                                                   uint32_t *keys, uint32_t *hist, bool cells)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t n = *n_in;
    uint32_t key = 0xFFFFFFFFu;
    if (k < n) {
        const uint32_t id = order[k];
        if (status[id] == 0) {
            const int i = cell_of(g.ax, x[id]);
            const int j = cell_of(g.ay, y[id]);
            const uint32_t ntx = (uint32_t)(g.ax.n - 2) / kTile + 1;
            key = (uint32_t)(j / kTile) * ntx + (uint32_t)(i / kTile);
            if (cells)
                key = key * (uint32_t)(kTile * kTile) + (uint32_t)((j % kTile) * kTile + i % kTile);
            if (g.az.n) {
                const int kk = cell_of(g.az, z[id]);
                key = key * (uint32_t)(g.az.n - 1) + (uint32_t)kk;
            }
        }
        keys[k] = key;
    }
    const bool valid = key != 0xFFFFFFFFu;
    int start;
    uint32_t len;
    wave_runs(key, valid, start, len);
    if (valid && start == (int)(threadIdx.x & 63))
        atomicAdd(&hist[key], len);
}

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanThreads * kScanItems;

// block-wide exclusive scan of one value per thread; returns the block total
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t &excl)
{
    __shared__ uint32_t wsum[kScanThreads / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t incl = v;
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_up(incl, off, 64);
        if (lane >= off)
            incl += t;
    }
    if (lane == 63)
        wsum[wid] = incl;
    __syncthreads();
    uint32_t wbase = 0, total = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
        if (w < wid)
            wbase += wsum[w];
        total += wsum[w];
    }
    __syncthreads();
    excl = wbase + incl - v;
    return total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_partial(const uint32_t *hist,
                                                               uint32_t nbins,
                                                               uint32_t *blocksums)
{
    const size_t base = (size_t)blockIdx.x * kScanChunk + (size_t)threadIdx.x * kScanItems;
    uint32_t s = 0;
    for (int q = 0; q < kScanItems; ++q)
        if (base + q < nbins)
            s += hist[base + q];
    uint32_t excl;
    const uint32_t tot = block_exclusive_scan(s, excl);
    if (threadIdx.x == 0)
        blocksums[blockIdx.x] = tot;
}

// single block: exclusive scan of the block sums in place; total -> *n_out
__global__ __launch_bounds__(kScanThreads) void k_scan_top(uint32_t *blocksums, uint32_t nblk,
                                                           uint32_t *n_out)
{
    uint32_t carry = 0;
    for (uint32_t base = 0; base < nblk; base += kScanThreads) {
        const uint32_t i = base + threadIdx.x;
        const uint32_t v = i < nblk ? blocksums[i] : 0u;
        uint32_t excl;
        const uint32_t tot = block_exclusive_scan(v, excl);
        if (i < nblk)
            blocksums[i] = carry + excl;
        carry += tot;
    }
    if (threadIdx.x == 0)
        *n_out = carry;
}

// hist -> exclusive offsets (in place)
__global__ __launch_bounds__(kScanThreads) void k_scan_apply(uint32_t *hist, uint32_t nbins,
                                                             const uint32_t *blocksums)
{
    const size_t base = (size_t)blockIdx.x * kScanChunk + (size_t)threadIdx.x * kScanItems;
    uint32_t v[kScanItems];
    uint32_t s = 0;
    for (int q = 0; q < kScanItems; ++q) {
        v[q] = base + q < nbins ? hist[base + q] : 0u;
        s += v[q];
    }
    uint32_t excl;
    block_exclusive_scan(s, excl);
    uint32_t run = blocksums[blockIdx.x] + excl;
    for (int q = 0; q < kScanItems; ++q) {
        if (base + q < nbins)
            hist[base + q] = run;
        run += v[q];
    }
}

__global__ __launch_bounds__(256) void k_sort_scatter(const uint32_t *order_in,
                                                      const uint32_t *n_in, const uint32_t *keys,
                                                      uint32_t *offsets, uint32_t *order_out)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    const uint32_t n = *n_in;
    const uint32_t key = k < n ? keys[k] : 0xFFFFFFFFu;
    const bool valid = key != 0xFFFFFFFFu;
    int start;
    uint32_t len;
    wave_runs(key, valid, start, len);
    const int lane = threadIdx.x & 63;
    uint32_t base = 0;
    if (valid && start == lane)
        base = atomicAdd(&offsets[key], len);
    base = __shfl(base, start, 64);
    if (valid)
        order_out[base + (uint32_t)(lane - start)] = order_in[k];
}

// ---------------------------------------------------------------- snapshot conversion
__device__ inline uint32_t bf16_rne(float f)
{
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu))
        return (b >> 16) | 0x40u;  // quiet NaN
    b += 0x7FFFu + ((b >> 16) & 1u);
    return b >> 16;
}

__device__ inline uint32_t f16_bits(float f)
{
    return (uint32_t)__builtin_bit_cast(uint16_t, (_Float16)f);
}

// Power-of-two scale s = 2^(ceil(log2 m) - 14) for a level whose largest
// magnitude is m (so |F / s| <= 2^14), or 1 when the level is all zeros.
__device__ inline float f16_scale(float m)
{
    if (!(m > 0.f))
        return 1.f;
    int e;
    const float fr = frexpf(m, &e);  // m = fr * 2^e, fr in [0.5, 1)
    const int c = (fr == 0.5f) ? e - 1 : e;
    return ldexpf(1.f, c - 14);
}

__global__ void k_level_absmax(const float *F, size_t plane, float *out)
{
    // one block per level; out[level] = max |F|
    const float *p = F + (size_t)blockIdx.x * plane;
    float m = 0.f;
    for (size_t i = threadIdx.x; i < plane; i += blockDim.x)
        m = fmaxf(m, fabsf(p[i]));
    for (int off = 32; off > 0; off >>= 1)
        m = fmaxf(m, __shfl_xor(m, off, 64));
    __shared__ float wm[16];
    if ((threadIdx.x & 63) == 0)
        wm[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
        float r = 0.f;
        for (unsigned w = 0; w < blockDim.x / 64; ++w)
            r = fmaxf(r, wm[w]);
        out[blockIdx.x] = r;
    }
}

template <int ST, bool IS3D>
__global__ void k_convert(const float *U, const float *V, const float *W, const double *U64,
                          const double *V64, const double *W64, size_t plane, int nzl,
                          void *slot, const float *scales)
{
    const size_t total = plane * (size_t)nzl;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        if constexpr (ST == kF64) {
            const double u = U64 ? U64[i] : (double)U[i];
            const double v = V64 ? V64[i] : (double)V[i];
            if constexpr (IS3D) {
                const double w = W64 ? W64[i] : (double)W[i];
                static_cast<double4 *>(slot)[i] = make_double4(u, v, w, 0.0);
            } else {
                static_cast<double2 *>(slot)[i] = make_double2(u, v);
            }
        } else if constexpr (ST == kF32) {
            if constexpr (IS3D)
                static_cast<float4 *>(slot)[i] = make_float4(U[i], V[i], W[i], 0.f);
            else
                static_cast<float2 *>(slot)[i] = make_float2(U[i], V[i]);
        } else if constexpr (ST == kBF16) {
            const uint32_t a = bf16_rne(U[i]) | (bf16_rne(V[i]) << 16);
            if constexpr (IS3D)
                static_cast<uint2 *>(slot)[i] = make_uint2(a, bf16_rne(W[i]));
            else
                static_cast<uint32_t *>(slot)[i] = a;
        } else {
            const size_t k = i / plane;
            const float *sc = scales + k * 3;
            const uint32_t a = f16_bits(U[i] / sc[0]) | (f16_bits(V[i] / sc[1]) << 16);
            if constexpr (IS3D)
                static_cast<uint2 *>(slot)[i] = make_uint2(a, f16_bits(W[i] / sc[2]));
            else
                static_cast<uint32_t *>(slot)[i] = a;
        }
    }
}

// turn the per-(level, variable) maxima into scales, in place
__global__ void k_scales_from_max(float *s, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        s[i] = f16_scale(s[i]);
}

// gather per-level maxima [var][level] into [level][var]
__global__ void k_interleave_max(const float *m, int nzl, int nvar, float *s)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nzl * 3) {
        const int k = i / 3, v = i % 3;
        s[i] = v < nvar ? m[v * nzl + k] : 0.f;
    }
}

}  // namespace

hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_fill_u32, dim3(grid_blocks(n, 256, 4096)), dim3(256), 0, s, p, v, n);
    return hipGetLastError();
}

hipError_t launch_iota(uint32_t *p, size_t n, hipStream_t s)
{
    hipLaunchKernelGGL(k_iota, dim3(grid_blocks(n, 256, 4096)), dim3(256), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_compact(const uint32_t *order_in, const uint32_t *n_in, const uint8_t *status,
                          uint32_t *order_out, uint32_t *n_out, uint32_t n_launch,
                          hipStream_t s)
{
    hipError_t e = launch_fill_u32(n_out, 0u, 1, s);
    if (e != hipSuccess || n_launch == 0)
        return e;
    constexpr uint32_t kPerBlock = kCompactThreads * kCompactItems;
    hipLaunchKernelGGL(k_compact, dim3((n_launch + kPerBlock - 1) / kPerBlock),
                       dim3(kCompactThreads), 0, s, order_in, n_in, status, order_out, n_out);
    return hipGetLastError();
}

uint32_t sort_bins(const GridDev &g, bool cells)
{
    const uint32_t ntx = (uint32_t)(g.ax.n - 2) / kTile + 1;
    const uint32_t nty = (uint32_t)(g.ay.n - 2) / kTile + 1;
    uint32_t nb = ntx * nty;
    if (g.az.n)
        nb *= (uint32_t)(g.az.n - 1);
    else if (cells)
        nb *= (uint32_t)(kTile * kTile);
    return nb;
}

size_t sort_blocksums(uint32_t nbins) { return (nbins + kScanChunk - 1) / kScanChunk; }

hipError_t launch_sort(const GridDev &g, const double *x, const double *y, const double *z,
                       const uint8_t *status, const uint32_t *order_in, const uint32_t *n_in,
                       uint32_t n_launch, uint32_t *keys, uint32_t *hist, uint32_t nbins,
                       uint32_t *blocksums, uint32_t *order_out, uint32_t *n_out,
                       hipStream_t s, bool cells)
{
    hipError_t e = launch_fill_u32(hist, 0u, nbins, s);
    if (e != hipSuccess)
        return e;
    const uint32_t nb = (n_launch + 255) / 256;
    if (nb)
        hipLaunchKernelGGL(k_sort_keys, dim3(nb), dim3(256), 0, s, g, x, y, z, status, order_in,
                           n_in, keys, hist, cells && !g.az.n);
    const uint32_t nblk = (uint32_t)sort_blocksums(nbins);
    hipLaunchKernelGGL(k_scan_partial, dim3(nblk), dim3(kScanThreads), 0, s, hist, nbins,
                       blocksums);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanThreads), 0, s, blocksums, nblk, n_out);
    hipLaunchKernelGGL(k_scan_apply, dim3(nblk), dim3(kScanThreads), 0, s, hist, nbins,
                       blocksums);
    if (nb)
        hipLaunchKernelGGL(k_sort_scatter, dim3(nb), dim3(256), 0, s, order_in, n_in, keys, hist,
                           order_out);
    return hipGetLastError();
}

hipError_t launch_level_absmax(const float *F, size_t plane, int nzl, float *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_level_absmax, dim3(nzl), dim3(1024), 0, s, F, plane, out);
    return hipGetLastError();
}

hipError_t launch_convert_snapshot(int store, bool is3d, const float *U, const float *V,
                                   const float *W, const double *U64, const double *V64,
                                   const double *W64, size_t plane, int nzl, void *slot,
                                   float *scales, float *tmp, hipStream_t s)
{
    const size_t total = plane * (size_t)nzl;
    const dim3 grid(grid_blocks(total, 256, 1u << 15)), blk(256);
    if (store == kF16S) {
        // scales[level*3 + var] from the per-level maxima of each variable (tmp: 3*nzl)
        float *m = scales;
        hipError_t e = launch_level_absmax(U, plane, nzl, tmp, s);
        if (e == hipSuccess)
            e = launch_level_absmax(V, plane, nzl, tmp + nzl, s);
        if (e == hipSuccess && is3d)
            e = launch_level_absmax(W, plane, nzl, tmp + 2 * nzl, s);
        if (e != hipSuccess)
            return e;
        hipLaunchKernelGGL(k_interleave_max, dim3((nzl * 3 + 255) / 256), dim3(256), 0, s, tmp,
                           nzl, is3d ? 3 : 2, m);
        hipLaunchKernelGGL(k_scales_from_max, dim3((nzl * 3 + 255) / 256), dim3(256), 0, s, m,
                           nzl * 3);
    }
#define LP_CONV(ST, D3)                                                                       \
    hipLaunchKernelGGL((k_convert<ST, D3>), grid, blk, 0, s, U, V, W, U64, V64, W64, plane,   \
                       nzl, slot, scales)
    switch (store) {
    case kF64: if (is3d) LP_CONV(kF64, true); else LP_CONV(kF64, false); break;
    case kF32: if (is3d) LP_CONV(kF32, true); else LP_CONV(kF32, false); break;
    case kBF16: if (is3d) LP_CONV(kBF16, true); else LP_CONV(kBF16, false); break;
    case kF16S: if (is3d) LP_CONV(kF16S, true); else LP_CONV(kF16S, false); break;
    default: return hipErrorInvalidValue;
    }
#undef LP_CONV
    return hipGetLastError();
}

}  // namespace lp
