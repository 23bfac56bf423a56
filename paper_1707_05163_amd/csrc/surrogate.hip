// surrogate.hip -- learned flow map: an MLP that predicts the displacement of a
// particle over one segment of fine RK4 steps, trained on segments that the RK4
// advection itself produces, and used with plain RK4 as the arbiter: a particle whose
// prediction disagrees with a coarse RK4 estimate by more than a threshold (or
// whose predicted end point is outside the grid or on land) is re-integrated with
// the fine RK4 steps.
//
// Network input (64 values, bf16): lon/180, lat/90, sin and cos of the phase of the
// periodic field, the 5 x 5 patch of U and V (m/s) around the nearest node,
// interpolated linearly in time, the particle's offset from that node, U and V at the
// particle and the cell size (see k_features).  Output: the segment displacement in
// metres (east, north) divided by kOutScale.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <random>
#include <vector>

#include "../../include/lp.h"
#include "lp_internal.h"
#include "lp_objects.h"

using lp::GemmArgs;
using lp::TimeEntry;

namespace {

constexpr int kIn = 64, kHid = 256, kOut = 2, kOutPad = 32, kLayers = 5;
constexpr double kOutScale = 7200.0;  // metres: 1 m/s over 2 h
const int kFanIn[kLayers] = {kIn, kHid, kHid, kHid, kHid};
const int kFanOut[kLayers] = {kHid, kHid, kHid, kHid, kOut};
const int kPadOut[kLayers] = {kHid, kHid, kHid, kHid, kOutPad};

#define SCHECK(expr)                                                                          \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) {                                                               \
            char b_[384];                                                                     \
            snprintf(b_, sizeof b_, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                     __LINE__);                                                               \
            lp_set_error(b_);                                                                 \
            return e_ == hipErrorOutOfMemory ? LP_ENOMEM : LP_EDEVICE;                        \
        }                                                                                     \
    } while (0)

template <class T>
hipError_t dmalloc(T **p, size_t n)
{
    *p = nullptr;
    return n ? hipMalloc((void **)p, n * sizeof(T)) : hipSuccess;
}

template <class T>
void dfree(T *&p)
{
    if (p)
        (void)hipFree((void *)p);
    p = nullptr;
}

// ------------------------------------------------------------------ device kernels
__device__ inline uint16_t to_bf16(float f)
{
    uint32_t b = __float_as_uint(f);
    if ((b & 0x7F800000u) == 0x7F800000u && (b & 0x007FFFFFu))
        return (uint16_t)((b >> 16) | 0x40u);
    b += 0x7FFFu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

__device__ inline int nearest_node(const lp::AxisDev &a, double x)
{
    if (!(x >= a.lo))
        return 0;
    if (!(x <= a.hi))
        return a.n - 1;
    int g = a.uniform ? (int)((x - a.lo) * a.ginv) : 0;
    if (!a.uniform) {
        int b = (int)((x - a.lo) * a.ginv);
        b = b < lp::kGuessBins - 1 ? b : lp::kGuessBins - 1;
        g = a.guess[b];
    }
    g = g < 0 ? 0 : (g > a.n - 2 ? a.n - 2 : g);
    while (g > 0 && a.c[g] > x)
        --g;
    while (g < a.n - 2 && a.c[g + 1] <= x)
        ++g;
    return (x - a.c[g]) * a.rw[g] < 0.5 ? g : g + 1;
}

__device__ inline void node_uv(const lp::FieldDev &f, int slot, size_t node, float &u, float &v,
                               int store)
{
    const char *p = static_cast<const char *>(f.slots) + (size_t)slot * f.slot_bytes;
    if (store == lp::kF32) {
        const float2 q = reinterpret_cast<const float2 *>(p)[node];
        u = q.x;
        v = q.y;
    } else if (store == lp::kF64) {
        const double2 q = reinterpret_cast<const double2 *>(p)[node];
        u = (float)q.x;
        v = (float)q.y;
    } else if (store == lp::kBF16) {
        const uint32_t q = reinterpret_cast<const uint32_t *>(p)[node];
        u = __uint_as_float(q << 16);
        v = __uint_as_float(q & 0xFFFF0000u);
    } else {
        const uint32_t q = reinterpret_cast<const uint32_t *>(p)[node];
        const float *sc = f.scales + (size_t)slot * f.nzl * 3;
        u = (float)__builtin_bit_cast(_Float16, (uint16_t)(q & 0xFFFFu)) * sc[0];
        v = (float)__builtin_bit_cast(_Float16, (uint16_t)(q >> 16)) * sc[1];
    }
}

struct FeatArgs {
    lp::GridDev g;
    lp::FieldDev f;
    int32_t store;
    const double *x, *y;      // positions (sample- or id-indexed)
    const uint32_t *sel;      // row r reads sample/id sel[r] (null: r)
    const uint32_t *round;    // per sample round (null: round 0)
    const TimeEntry *tab;     // time bracket per round
    const float *phase;       // sin, cos per round
    const uint32_t *n_dev;    // number of rows with data (device), or null
    int64_t n, npad;          // rows with data (if n_dev is null), padded rows
    uint16_t *X;              // [npad x 64]
    const float *tgt;         // per sample targets (2 floats), or null
    float *T;                 // [npad x 2]
};

__device__ inline int cell_frac(const lp::AxisDev &a, double x, double &f)
{
    double xc = x < a.lo ? a.lo : (x > a.hi ? a.hi : x);
    int g = a.uniform ? (int)((xc - a.lo) * a.ginv) : 0;
    if (!a.uniform) {
        int b = (int)((xc - a.lo) * a.ginv);
        b = b < lp::kGuessBins - 1 ? b : lp::kGuessBins - 1;
        g = a.guess[b];
    }
    g = g < 0 ? 0 : (g > a.n - 2 ? a.n - 2 : g);
    while (g > 0 && a.c[g] > xc)
        --g;
    while (g < a.n - 2 && a.c[g + 1] <= xc)
        ++g;
    f = (xc - a.c[g]) * a.rw[g];
    return g;
}

// Network input row: [0..3] lon/180, lat/90, sin and cos of the phase; [4..53] the
// 5 x 5 patch of (U, V) around the nearest node, linear in time; [54..55] the offset
// of the particle from that node in cell widths; [56..57] U, V interpolated
// bilinearly at the particle; [58..59] the cell width and height in units of 30 km;
// [60..63] zero.
constexpr int kFeatBlock = 128;  // rows (threads) per block of k_features

__device__ inline void feature_row(const FeatArgs &a, int64_t r, uint32_t P[32]);

// Each thread assembles one row as 32 pairs of bfloat16 (feature 2m in the low half);
// the block's 128 rows, 16 KB of consecutive memory, go out through LDS so that each
// store instruction of a wave writes 1 KB of consecutive bytes.
__global__ __launch_bounds__(kFeatBlock) void k_features(FeatArgs a)
{
    static_assert(kIn == 64, "a row is 32 bf16 pairs");
    __shared__ uint4 stage[kFeatBlock * 9];  // 8 chunks per row + 1 of padding (no conflicts)
    const int64_t base = blockIdx.x * (int64_t)kFeatBlock, r = base + threadIdx.x;
    const int64_t n = a.n_dev ? (int64_t)*a.n_dev : a.n;
    uint32_t P[32];
    if (r < a.npad && r < n) {
        feature_row(a, r, P);
    } else {
#pragma unroll
        for (int q = 0; q < 32; ++q)
            P[q] = 0u;
        if (r < a.npad && a.T) {
            a.T[2 * r] = 0.f;
            a.T[2 * r + 1] = 0.f;
        }
    }
#pragma unroll
    for (int q = 0; q < 8; ++q)
        stage[threadIdx.x * 9 + q] = uint4{P[4 * q], P[4 * q + 1], P[4 * q + 2], P[4 * q + 3]};
    __syncthreads();
    for (int c = threadIdx.x; c < kFeatBlock * 8; c += kFeatBlock) {
        const int row = c >> 3, part = c & 7;
        if (base + row < a.npad)
            reinterpret_cast<uint4 *>(a.X + (base + row) * kIn)[part] = stage[row * 9 + part];
    }
}

__device__ inline void feature_row(const FeatArgs &a, int64_t r, uint32_t P[32])
{
    // the hardware's round-to-nearest-even convert, one instruction per pair (the
    // features are finite, so it rounds as to_bf16 does)
    auto pair = [](float lo, float hi) {
        typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));
        typedef float f32x2 __attribute__((ext_vector_type(2)));
        return __builtin_bit_cast(uint32_t, __builtin_convertvector(f32x2{lo, hi}, bf16x2));
    };
    const uint32_t s = a.sel ? a.sel[r] : (uint32_t)r;
    const uint32_t rd = a.round ? a.round[s] : 0u;
    const TimeEntry e = a.tab[rd];
    const double x = a.x[s], y = a.y[s];
    const float t = (float)e.tau;
    P[0] = pair((float)(x / 180.0), (float)(y / 90.0));
    P[1] = pair(a.phase[2 * rd], a.phase[2 * rd + 1]);
    double fx, fy;
    const int ci = cell_frac(a.g.ax, x, fx), cj = cell_frac(a.g.ay, y, fy);
    const int i0 = fx < 0.5 ? ci : ci + 1, j0 = fy < 0.5 ? cj : cj + 1;
    const int nx = a.g.ax.n, ny = a.g.ay.n;
#pragma unroll
    for (int dj = -2; dj <= 2; ++dj) {
        int jj = j0 + dj;
        jj = jj < 0 ? 0 : (jj > ny - 1 ? ny - 1 : jj);
#pragma unroll
        for (int di = -2; di <= 2; ++di) {
            int ii = i0 + di;
            ii = ii < 0 ? 0 : (ii > nx - 1 ? nx - 1 : ii);
            const size_t node = (size_t)jj * nx + ii;
            float ua, va, ub, vb;
            node_uv(a.f, e.sa, node, ua, va, a.store);
            node_uv(a.f, e.sb, node, ub, vb, a.store);
            P[2 + 5 * (dj + 2) + (di + 2)] = pair(ua + t * (ub - ua), va + t * (vb - va));
        }
    }
    P[27] = pair((float)(fx < 0.5 ? fx : fx - 1.0), (float)(fy < 0.5 ? fy : fy - 1.0));
    float up = 0.f, vp = 0.f;
    const float w[4] = {(float)((1 - fx) * (1 - fy)), (float)(fx * (1 - fy)),
                        (float)((1 - fx) * fy), (float)(fx * fy)};
    const size_t c00 = (size_t)cj * nx + ci;
    const size_t cn[4] = {c00, c00 + 1, c00 + nx, c00 + nx + 1};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        float ua, va, ub, vb;
        node_uv(a.f, e.sa, cn[k], ua, va, a.store);
        node_uv(a.f, e.sb, cn[k], ub, vb, a.store);
        up += w[k] * (ua + t * (ub - ua));
        vp += w[k] * (va + t * (vb - va));
    }
    P[28] = pair(up, vp);
    double hx = a.g.ax.c[ci + 1] - a.g.ax.c[ci], hy = a.g.ay.c[cj + 1] - a.g.ay.c[cj];
    if (a.g.spherical) {
        hx *= lp::kMetresPerDegree * cos(y * lp::kDegToRad);
        hy *= lp::kMetresPerDegree;
    }
    P[29] = pair((float)(hx / 30000.0), (float)(hy / 30000.0));
    P[30] = 0u;
    P[31] = 0u;
    if (a.T) {
        a.T[2 * r] = a.tgt[2 * s];
        a.T[2 * r + 1] = a.tgt[2 * s + 1];
    }
}

// Philox4x32-10 (Salmon et al., SC'11), for seeding and batch sampling
__device__ inline void philox(uint32_t c[4], uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        const uint32_t lo0 = 0xD2511F53u * c[0], hi0 = __umulhi(0xD2511F53u, c[0]);
        const uint32_t lo1 = 0xCD9E8D57u * c[2], hi1 = __umulhi(0xCD9E8D57u, c[2]);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

// n start positions uniform inside cells whose four corner nodes are ocean
__global__ void k_seed(lp::GridDev g, const uint8_t *landnode, int64_t n, uint32_t seed,
                       uint32_t round, double *x, double *y)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= n)
        return;
    const int nx = g.ax.n, ny = g.ay.n;
    for (uint32_t attempt = 0; attempt < 256; ++attempt) {
        uint32_t c[4] = {(uint32_t)p, attempt, round, 0x5EEDu};
        philox(c, seed, 0xC0FFEEu);
        const int i = (int)(((uint64_t)c[0] * (uint64_t)(nx - 1)) >> 32);
        const int j = (int)(((uint64_t)c[1] * (uint64_t)(ny - 1)) >> 32);
        const size_t n00 = (size_t)j * nx + i;
        if (landnode && (landnode[n00] || landnode[n00 + 1] || landnode[n00 + nx] ||
                         landnode[n00 + nx + 1]))
            continue;
        const double fx = (double)c[2] * 0x1p-32, fy = (double)c[3] * 0x1p-32;
        x[p] = g.ax.c[i] + fx * (g.ax.c[i + 1] - g.ax.c[i]);
        y[p] = g.ay.c[j] + fy * (g.ay.c[j + 1] - g.ay.c[j]);
        return;
    }
    x[p] = g.ax.c[0] - 1.0;  // no ocean cell found: outside, dropped as OOB
    y[p] = g.ay.c[0];
}

// Training targets from one round: keep the segments that stayed active, append
// (x0, y0, round, displacement in metres / kOutScale) to the data set.
__global__ void k_targets(const double *x0, const double *y0, const double *x1, const double *y1,
                          const uint8_t *st, int64_t n, int spherical, uint32_t round,
                          double *dx0, double *dy0, uint32_t *dround, float *dtgt,
                          unsigned long long *count, int64_t cap)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const bool keep = p < n && st[p] == 0;
    const uint64_t mask = __ballot(keep);
    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    unsigned long long base = 0;
    if (keep && rank == 0)
        base = atomicAdd(count, (unsigned long long)__popcll(mask));
    const int src = mask ? __ffsll((unsigned long long)mask) - 1 : 0;
    base = __shfl(base, src, 64);
    if (!keep)
        return;
    const int64_t o = (int64_t)base + rank;
    if (o >= cap)
        return;
    double ex = x1[p] - x0[p], ey = y1[p] - y0[p];
    if (spherical) {
        ex *= lp::kMetresPerDegree * cos(y0[p] * lp::kDegToRad);
        ey *= lp::kMetresPerDegree;
    }
    dx0[o] = x0[p];
    dy0[o] = y0[p];
    dround[o] = round;
    dtgt[2 * o] = (float)(ex / kOutScale);
    dtgt[2 * o + 1] = (float)(ey / kOutScale);
}

__global__ void k_sample_batch(uint32_t seed, uint32_t iter, int64_t nsamples, int64_t B,
                               uint32_t *idx)
{
    const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (r >= B)
        return;
    uint32_t c[4] = {(uint32_t)r, iter, 0xBA7C4u, 0u};
    philox(c, seed, 0x5A3Bu);
    idx[r] = (uint32_t)((((uint64_t)c[0] << 32 | c[1]) % (uint64_t)nsamples));
}

__device__ inline bool locate_in(const lp::AxisDev &a, double x, int &i)
{
    if (!(x >= a.lo && x <= a.hi))
        return false;
    int g = a.uniform ? (int)((x - a.lo) * a.ginv) : 0;
    if (!a.uniform) {
        int b = (int)((x - a.lo) * a.ginv);
        b = b < lp::kGuessBins - 1 ? b : lp::kGuessBins - 1;
        g = a.guess[b];
    }
    g = g < 0 ? 0 : (g > a.n - 2 ? a.n - 2 : g);
    while (g > 0 && a.c[g] > x)
        --g;
    while (g < a.n - 2 && a.c[g + 1] <= x)
        ++g;
    i = g;
    return true;
}

// Residual check: accept the network's displacement where it agrees with the
// coarse RK4 displacement to within thr metres and ends in an ocean cell inside the
// grid; otherwise queue the particle for the fine RK4 steps.  The queue is appended
// with one atomic per block (block_append): one per wave on the single counter
// serialised and took most of the kernel's time.  Every active
// particle is either accepted or queued, so the accepted count is the active count
// less the queue's length.
constexpr int kCheckThreads = 1024;

// The slot of this thread's item (when `in`) in a list that the block of kCheckThreads
// threads appends to with one atomic on the list's counter: the waves' ballot counts are
// summed in LDS by the first thread.  Every thread of the block calls it; a block's items
// land together, in thread order.
__device__ inline uint32_t block_append(bool in, uint32_t *count)
{
    __shared__ uint32_t wbase[kCheckThreads / 64];
    __shared__ uint32_t block_base;
    const uint64_t mb = __ballot(in);
    const uint32_t rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(mb >> 32),
                                                    __builtin_amdgcn_mbcnt_lo((uint32_t)mb, 0u));
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0)
        wbase[wid] = (uint32_t)__popcll(mb);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (int w = 0; w < kCheckThreads / 64; ++w) {
            const uint32_t c = wbase[w];
            wbase[w] = tot;
            tot += c;
        }
        block_base = tot ? atomicAdd(count, tot) : 0u;
    }
    __syncthreads();
    return block_base + wbase[wid] + rank;
}

__global__ __launch_bounds__(kCheckThreads) void k_check(lp::GridDev g, const uint32_t *order,
                                                         const uint32_t *n_act, double *x,
                                                         double *y, const double *xc,
                                                         const double *yc, const uint8_t *stc,
                                                         const float *Y, double thr,
                                                         uint32_t *fall, uint32_t *nfall)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    bool back = false;
    uint32_t id = 0;
    if (k < *n_act) {
        id = order[k];
        const double x0 = x[id], y0 = y[id];
        const double mx = (double)Y[2 * k] * kOutScale, my = (double)Y[2 * k + 1] * kOutScale;
        double ex = xc[id] - x0, ey = yc[id] - y0, nx1 = x0 + mx, ny1 = y0 + my;
        if (g.spherical) {
            const double m = lp::kMetresPerDegree * cos(y0 * lp::kDegToRad);
            ex *= m;
            ey *= lp::kMetresPerDegree;
            nx1 = x0 + mx / m;
            ny1 = y0 + my / lp::kMetresPerDegree;
        }
        const double r = sqrt((mx - ex) * (mx - ex) + (my - ey) * (my - ey));
        int ci, cj;
        const bool ok = stc[id] == 0 && r <= thr && locate_in(g.ax, nx1, ci) &&
                        locate_in(g.ay, ny1, cj) &&
                        !(g.landcell && g.landcell[(size_t)cj * (g.ax.n - 1) + ci]);
        if (ok) {
            x[id] = nx1;
            y[id] = ny1;
        } else {
            back = true;
        }
    }
    const uint32_t at = block_append(back, nfall);
    if (back)
        fall[at] = id;
}

// The particle state in the order of the sorted active list: perm lists storage
// positions, the sorted active ones first and the inactive ones after them; pid maps a
// storage position to the particle's id.  With the state in this order the kernels of
// a segment read and write it in consecutive runs instead of one 8-byte word per line.
// k_perm_inactive appends the inactive positions after the n_act active ones
// (block_append; their order does not matter).
__global__ __launch_bounds__(kCheckThreads) void k_perm_inactive(const uint8_t *st, uint32_t n,
                                                                 const uint32_t *n_act,
                                                                 uint32_t *perm, uint32_t *cnt)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    const bool in = p < n && st[p] != 0;
    const uint32_t at = *n_act + block_append(in, cnt);
    if (in && at < n)
        perm[at] = p;
}

// The first n_in entries of a list.
__global__ void k_copy_list(const uint32_t *src, const uint32_t *n_in, uint32_t *dst)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < *n_in)
        dst[k] = src[k];
}

__global__ void k_permute(const uint32_t *perm, uint32_t n, const double *x, const double *y,
                          const uint8_t *st, const uint32_t *pid, double *x2, double *y2,
                          uint8_t *st2, uint32_t *pid2)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) {
        const uint32_t q = perm[p];
        x2[p] = x[q];
        y2[p] = y[q];
        st2[p] = st[q];
        pid2[p] = pid[q];
    }
}

// Back to id order.
__global__ void k_unpermute(const uint32_t *pid, uint32_t n, const double *x2, const double *y2,
                            const uint8_t *st2, double *x, double *y, uint8_t *st)
{
    const uint32_t p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p < n) {
        const uint32_t q = pid[p];
        x[q] = x2[p];
        y[q] = y2[p];
        st[q] = st2[p];
    }
}

// A list of storage positions as particle ids.
__global__ void k_map_ids(const uint32_t *pid, const uint32_t *n_in, const uint32_t *order,
                          uint32_t *out)
{
    const uint32_t k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < *n_in)
        out[k] = pid[order[k]];
}

}  // namespace

// ------------------------------------------------------------------ model object
struct lp_model {
    float *W[kLayers] = {}, *b[kLayers] = {};  // FP32 master [fan_in x pad_out], [pad_out]
    float *mW[kLayers] = {}, *vW[kLayers] = {}, *mb[kLayers] = {}, *vb[kLayers] = {};
    float *gW[kLayers] = {}, *gb[kLayers] = {};
    uint16_t *Wb[kLayers] = {}, *WT[kLayers] = {};  // bf16 [fan_in x pad], [pad x fan_in]
    int adam_t = 0;
    // work buffers for `cap` rows
    int64_t cap = 0;
    uint16_t *X = nullptr, *H[kLayers - 1] = {}, *dzq[2] = {}, *pad = nullptr;
    float *Z[kLayers - 1] = {}, *Y = nullptr, *T = nullptr, *dz = nullptr, *dz2 = nullptr;
    float *loss = nullptr;
};

namespace {

int model_alloc(lp_model *m)
{
    for (int l = 0; l < kLayers; ++l) {
        const size_t n = (size_t)kFanIn[l] * kPadOut[l], nb = (size_t)kPadOut[l];
        SCHECK(dmalloc(&m->W[l], n));
        SCHECK(dmalloc(&m->b[l], nb));
        SCHECK(dmalloc(&m->mW[l], n));
        SCHECK(dmalloc(&m->vW[l], n));
        SCHECK(dmalloc(&m->mb[l], nb));
        SCHECK(dmalloc(&m->vb[l], nb));
        SCHECK(dmalloc(&m->gW[l], n));
        SCHECK(dmalloc(&m->gb[l], nb));
        SCHECK(dmalloc(&m->Wb[l], n));
        SCHECK(dmalloc(&m->WT[l], n));
        SCHECK(hipMemset(m->mW[l], 0, n * 4));
        SCHECK(hipMemset(m->vW[l], 0, n * 4));
        SCHECK(hipMemset(m->mb[l], 0, nb * 4));
        SCHECK(hipMemset(m->vb[l], 0, nb * 4));
        SCHECK(hipMemset(m->gW[l], 0, n * 4));
        SCHECK(hipMemset(m->gb[l], 0, nb * 4));
    }
    SCHECK(dmalloc(&m->loss, 1));
    return LP_OK;
}

void model_free_work(lp_model *m)
{
    dfree(m->X);
    dfree(m->pad);
    dfree(m->Y);
    dfree(m->T);
    dfree(m->dz);
    dfree(m->dz2);
    dfree(m->dzq[0]);
    dfree(m->dzq[1]);
    for (int l = 0; l < kLayers - 1; ++l) {
        dfree(m->H[l]);
        dfree(m->Z[l]);
    }
    m->cap = 0;
}

int model_work(lp_model *m, int64_t rows)
{
    if (rows <= m->cap)
        return LP_OK;
    model_free_work(m);
    SCHECK(dmalloc(&m->X, (size_t)rows * kIn));
    for (int l = 0; l < kLayers - 1; ++l) {
        SCHECK(dmalloc(&m->H[l], (size_t)rows * kHid));
        SCHECK(dmalloc(&m->Z[l], (size_t)rows * kHid));
    }
    SCHECK(dmalloc(&m->pad, (size_t)rows * kOutPad));
    SCHECK(dmalloc(&m->dzq[0], (size_t)rows * kHid));
    SCHECK(dmalloc(&m->dzq[1], (size_t)rows * kHid));
    SCHECK(dmalloc(&m->Y, (size_t)rows * kOut));
    SCHECK(dmalloc(&m->T, (size_t)rows * kOut));
    SCHECK(dmalloc(&m->dz, (size_t)rows * kHid));
    SCHECK(dmalloc(&m->dz2, (size_t)rows * kOut));
    m->cap = rows;
    return LP_OK;
}

// bf16 copies of the master weights
int refresh_bf16(lp_model *m, hipStream_t s)
{
    for (int l = 0; l < kLayers; ++l)
        SCHECK(lp::launch_adam(m->W[l], nullptr, nullptr, nullptr, kFanIn[l], kPadOut[l],
                               kFanOut[l], 0.f, 0.9f, 0.999f, 1e-8f, 1, m->Wb[l], m->WT[l], s));
    return LP_OK;
}

// forward over `rows` (multiple of 128) rows of m->X; keeps pre-activations if train.
// Inference runs the fused kernel (activations never leave the chip); training runs
// the layer-by-layer GEMMs, which store what the backward pass needs.
int forward(lp_model *m, int64_t rows, bool train, hipStream_t s)
{
    if (!train) {
        lp::MlpFusedArgs a{};
        a.X = m->X;
        a.rows = rows;
        for (int l = 0; l < kLayers; ++l) {
            a.WT[l] = m->WT[l];
            a.bias[l] = m->b[l];
        }
        a.Y = m->Y;
        SCHECK(lp::launch_mlp_fused(a, s));
        return LP_OK;
    }
    const uint16_t *in = m->X;
    for (int l = 0; l < kLayers; ++l) {
        GemmArgs g{};
        g.A = in;
        g.B = m->WT[l];
        g.M = rows;
        g.N = kPadOut[l];
        g.K = kFanIn[l];
        g.kchunk = g.K;
        g.sai = kFanIn[l];
        g.sak = 1;
        g.sbk = 1;
        g.sbj = kFanIn[l];
        g.bias = m->b[l];
        g.ldc = kPadOut[l];
        if (l < kLayers - 1) {
            g.Z = train ? m->Z[l] : nullptr;
            g.H = m->H[l];
            SCHECK(lp::launch_gemm(lp::kEpiHidden, g, s));
            in = m->H[l];
        } else {
            g.Y = m->Y;
            g.ldy = kOut;
            g.nvalid = kOut;
            SCHECK(lp::launch_gemm(lp::kEpiOut, g, s));
        }
    }
    return LP_OK;
}

__global__ void k_pad_out(const float *dz2, int64_t rows, uint16_t *pad)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= rows * kOutPad)
        return;
    const int64_t r = i / kOutPad;
    const int c = (int)(i % kOutPad);
    pad[i] = c < kOut ? to_bf16(dz2[r * kOut + c]) : (uint16_t)0;
}

int64_t split_of(int64_t rows)
{
    // split the batch dimension of the weight gradients over more blocks
    int64_t c = rows;
    while (c > 512 && c % 2 == 0 && (c / 2) % 16 == 0)
        c /= 2;
    return c;
}

// gradients of L = (1/2B) sum (y - t)^2 for the batch in m->X / m->T (after forward)
int backward(lp_model *m, int64_t rows, hipStream_t s)
{
    SCHECK(lp::launch_fill_f32(m->loss, 0.f, 1, s));
    uint16_t *scratch = m->dzq[0];  // the loss kernel's bf16 output is not used
    SCHECK(lp::launch_loss_grad(m->Y, m->T, rows, kOut, m->dz2, scratch, m->loss, s));
    hipLaunchKernelGGL(k_pad_out, dim3((uint32_t)((rows * kOutPad + 255) / 256)), dim3(256), 0,
                       s, m->dz2, rows, m->pad);
    SCHECK(hipGetLastError());
    int cur = 0;
    for (int l = kLayers - 1; l >= 0; --l) {
        const int K = kFanIn[l], N = kPadOut[l];
        const bool out = l == kLayers - 1;
        const uint16_t *dzq = out ? m->pad : m->dzq[cur];
        const uint16_t *hin = l == 0 ? m->X : m->H[l - 1];
        // gW[l] [K x N] = H_in^T dzq
        SCHECK(lp::launch_fill_f32(m->gW[l], 0.f, (int64_t)K * N, s));
        GemmArgs gw{};
        gw.A = hin;
        gw.B = dzq;
        gw.M = K;
        gw.N = N;
        gw.K = rows;
        gw.kchunk = split_of(rows);
        gw.sai = 1;
        gw.sak = K;
        gw.sbk = N;
        gw.sbj = 1;
        gw.Y = m->gW[l];
        gw.ldy = N;
        SCHECK(lp::launch_gemm(lp::kEpiAccum, gw, s));
        if (out) {
            SCHECK(lp::launch_colsum(m->dz2, rows, kOut, m->gb[l], s));
            SCHECK(lp::launch_fill_f32(m->gb[l] + kOut, 0.f, N - kOut, s));
        } else {
            SCHECK(lp::launch_colsum(m->dz, rows, N, m->gb[l], s));
        }
        if (l > 0) {
            // dH = dzq W_l^T, then dz = dH * gelu'(z_{l-1}) -> m->dz, bf16 -> other buffer
            const int nxt = out ? 0 : 1 - cur;
            GemmArgs g{};
            g.A = dzq;
            g.B = m->Wb[l];
            g.M = rows;
            g.N = K;
            g.K = N;
            g.kchunk = N;
            g.sai = N;
            g.sak = 1;
            g.sbk = 1;
            g.sbj = N;
            g.Zin = m->Z[l - 1];
            g.ldc = K;
            g.dZ = m->dz;
            g.H = m->dzq[nxt];
            SCHECK(lp::launch_gemm(lp::kEpiBackData, g, s));
            cur = nxt;
        }
    }
    return LP_OK;
}

int adam(lp_model *m, float lr, hipStream_t s)
{
    m->adam_t++;
    for (int l = 0; l < kLayers; ++l) {
        SCHECK(lp::launch_adam(m->W[l], m->gW[l], m->mW[l], m->vW[l], kFanIn[l], kPadOut[l],
                               kFanOut[l], lr, 0.9f, 0.999f, 1e-8f, m->adam_t, m->Wb[l], m->WT[l],
                               s));
        SCHECK(lp::launch_adam(m->b[l], m->gb[l], m->mb[l], m->vb[l], 1, kPadOut[l], kFanOut[l],
                               lr, 0.9f, 0.999f, 1e-8f, m->adam_t, nullptr, nullptr, s));
    }
    return LP_OK;
}

// host fp32 rows [B x 64] -> padded bf16 m->X (and targets [B x 2] -> m->T)
int upload_batch(lp_model *m, int64_t B, int64_t rows, const float *X, const float *T,
                 hipStream_t s)
{
    float *tmp = nullptr;
    SCHECK(dmalloc(&tmp, (size_t)rows * kIn));
    hipError_t e = hipMemset(tmp, 0, (size_t)rows * kIn * 4);
    if (e == hipSuccess) e = hipMemcpy(tmp, X, (size_t)B * kIn * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = lp::launch_to_bf16(tmp, rows * kIn, m->X, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e == hipSuccess && T) {
        e = hipMemset(m->T, 0, (size_t)rows * kOut * 4);
        if (e == hipSuccess) e = hipMemcpy(m->T, T, (size_t)B * kOut * 4, hipMemcpyHostToDevice);
    }
    dfree(tmp);
    SCHECK(e);
    return LP_OK;
}

int64_t round128(int64_t n) { return (n + 127) / 128 * 128; }

}  // namespace

// ------------------------------------------------------------------ C ABI
extern "C" int64_t surrogate_param_count(void)
{
    int64_t n = 0;
    for (int l = 0; l < kLayers; ++l)
        n += (int64_t)kFanIn[l] * kFanOut[l] + kFanOut[l];
    return n;
}

extern "C" void surrogate_destroy(lp_model *m)
{
    if (!m)
        return;
    (void)hipDeviceSynchronize();
    for (int l = 0; l < kLayers; ++l) {
        dfree(m->W[l]);
        dfree(m->b[l]);
        dfree(m->mW[l]);
        dfree(m->vW[l]);
        dfree(m->mb[l]);
        dfree(m->vb[l]);
        dfree(m->gW[l]);
        dfree(m->gb[l]);
        dfree(m->Wb[l]);
        dfree(m->WT[l]);
    }
    dfree(m->loss);
    model_free_work(m);
    delete m;
}

extern "C" int surrogate_set_params(lp_model *m, const float *params)
{
    if (!m || !params) {
        lp_set_error("null argument");
        return LP_EINVAL;
    }
    const float *p = params;
    for (int l = 0; l < kLayers; ++l) {
        std::vector<float> w((size_t)kFanIn[l] * kPadOut[l], 0.f), b((size_t)kPadOut[l], 0.f);
        for (int k = 0; k < kFanIn[l]; ++k)
            for (int j = 0; j < kFanOut[l]; ++j)
                w[(size_t)k * kPadOut[l] + j] = *p++;
        for (int j = 0; j < kFanOut[l]; ++j)
            b[j] = *p++;
        SCHECK(hipMemcpy(m->W[l], w.data(), w.size() * 4, hipMemcpyHostToDevice));
        SCHECK(hipMemcpy(m->b[l], b.data(), b.size() * 4, hipMemcpyHostToDevice));
    }
    int rc = refresh_bf16(m, nullptr);
    if (rc)
        return rc;
    SCHECK(hipDeviceSynchronize());
    return LP_OK;
}

static int copy_out(lp_model *m, float *const *W, float *const *b, float *out)
{
    (void)m;
    float *p = out;
    for (int l = 0; l < kLayers; ++l) {
        std::vector<float> w((size_t)kFanIn[l] * kPadOut[l]), bb((size_t)kPadOut[l]);
        SCHECK(hipMemcpy(w.data(), W[l], w.size() * 4, hipMemcpyDeviceToHost));
        SCHECK(hipMemcpy(bb.data(), b[l], bb.size() * 4, hipMemcpyDeviceToHost));
        for (int k = 0; k < kFanIn[l]; ++k)
            for (int j = 0; j < kFanOut[l]; ++j)
                *p++ = w[(size_t)k * kPadOut[l] + j];
        for (int j = 0; j < kFanOut[l]; ++j)
            *p++ = bb[j];
    }
    return LP_OK;
}

extern "C" int surrogate_get_params(lp_model *m, float *params)
{
    if (!m || !params) {
        lp_set_error("null argument");
        return LP_EINVAL;
    }
    SCHECK(hipDeviceSynchronize());
    return copy_out(m, m->W, m->b, params);
}

extern "C" int surrogate_create(uint32_t seed, lp_model **out)
{
    if (!out) {
        lp_set_error("null argument");
        return LP_EINVAL;
    }
    *out = nullptr;
    lp_model *m = new lp_model();
    int rc = model_alloc(m);
    if (rc) {
        surrogate_destroy(m);
        return rc;
    }
    // He-normal initialisation, std sqrt(2 / fan_in), zero biases
    std::mt19937_64 gen(seed);
    std::normal_distribution<double> nd(0.0, 1.0);
    std::vector<float> p((size_t)surrogate_param_count());
    size_t q = 0;
    for (int l = 0; l < kLayers; ++l) {
        const double sd = std::sqrt(2.0 / kFanIn[l]);
        for (int k = 0; k < kFanIn[l] * kFanOut[l]; ++k)
            p[q++] = (float)(nd(gen) * sd);
        for (int j = 0; j < kFanOut[l]; ++j)
            p[q++] = 0.f;
    }
    if ((rc = surrogate_set_params(m, p.data()))) {
        surrogate_destroy(m);
        return rc;
    }
    *out = m;
    return LP_OK;
}

extern "C" int surrogate_forward(lp_model *m, int64_t B, const float *X, float *Y)
{
    if (!m || B < 1 || !X || !Y) {
        lp_set_error("bad arguments");
        return LP_EINVAL;
    }
    const int64_t rows = round128(B);
    int rc;
    if ((rc = model_work(m, rows)) || (rc = upload_batch(m, B, rows, X, nullptr, nullptr)) ||
        (rc = forward(m, rows, false, nullptr)))
        return rc;
    SCHECK(hipDeviceSynchronize());
    SCHECK(hipMemcpy(Y, m->Y, (size_t)B * kOut * 4, hipMemcpyDeviceToHost));
    return LP_OK;
}

extern "C" int surrogate_gradients(lp_model *m, int64_t B, const float *X, const float *T,
                                   float *grads, float *loss)
{
    if (!m || B < 1 || B % 128 || !X || !T || !grads) {
        lp_set_error("bad arguments (B must be a multiple of 128)");
        return LP_EINVAL;
    }
    int rc;
    if ((rc = model_work(m, B)) || (rc = upload_batch(m, B, B, X, T, nullptr)) ||
        (rc = forward(m, B, true, nullptr)) || (rc = backward(m, B, nullptr)))
        return rc;
    SCHECK(hipDeviceSynchronize());
    if (loss)
        SCHECK(hipMemcpy(loss, m->loss, 4, hipMemcpyDeviceToHost));
    return copy_out(m, m->gW, m->gb, grads);
}

extern "C" int surrogate_train_step(lp_model *m, int64_t B, const float *X, const float *T,
                                    double lr, float *loss)
{
    if (!m || B < 1 || B % 128 || !X || !T) {
        lp_set_error("bad arguments (B must be a multiple of 128)");
        return LP_EINVAL;
    }
    int rc;
    if ((rc = model_work(m, B)) || (rc = upload_batch(m, B, B, X, T, nullptr)) ||
        (rc = forward(m, B, true, nullptr)) || (rc = backward(m, B, nullptr)) ||
        (rc = adam(m, (float)lr, nullptr)))
        return rc;
    SCHECK(hipDeviceSynchronize());
    if (loss)
        SCHECK(hipMemcpy(loss, m->loss, 4, hipMemcpyDeviceToHost));
    return LP_OK;
}

// ------------------------------------------------------------------ training
namespace {

struct Timer {
    hipEvent_t a = nullptr, b = nullptr;
    Timer() {
        (void)hipEventCreate(&a);
        (void)hipEventCreate(&b);
    }
    ~Timer() {
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
    }
    void start(hipStream_t s) { (void)hipEventRecord(a, s); }
    double stop_ms(hipStream_t s) {
        (void)hipEventRecord(b, s);
        (void)hipEventSynchronize(b);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, a, b);
        return ms;
    }
};

// The phase boundaries of one inference segment (sort, network, coarse steps, check and
// fine steps) as events, read back only once the stream has passed them anyway.
struct SegmentEvents {
    hipEvent_t e[5] = {};
    bool sorted = false, live = false;
    SegmentEvents() {
        for (auto &x : e)
            (void)hipEventCreate(&x);
    }
    ~SegmentEvents() {
        for (auto &x : e)
            if (x)
                (void)hipEventDestroy(x);
    }
    void account(lp_surrogate_stats *st) {
        if (!live)
            return;
        float ms = 0.f;
        if (sorted && hipEventElapsedTime(&ms, e[0], e[1]) == hipSuccess)
            st->sort_ms += ms;
        if (hipEventElapsedTime(&ms, e[1], e[2]) == hipSuccess)
            st->mlp_ms += ms;
        if (hipEventElapsedTime(&ms, e[2], e[3]) == hipSuccess)
            st->coarse_ms += ms;
        if (hipEventElapsedTime(&ms, e[3], e[4]) == hipSuccess)
            st->fine_ms += ms;
        live = false;
    }
};

struct DeviceBuf {
    std::vector<void *> p;
    ~DeviceBuf() {
        for (void *q : p)
            if (q) (void)hipFree(q);
    }
    template <class T>
    hipError_t get(T **out, size_t n) {
        hipError_t e = dmalloc(out, n);
        if (e == hipSuccess)
            p.push_back((void *)*out);
        return e;
    }
};

double field_period(const lp_fieldset *fs, double &t_lo)
{
    std::vector<double> t;
    for (int s = 0; s < fs->capacity; ++s)
        if (fs->slot_seq[s] >= 0)
            t.push_back(fs->slot_t[s]);
    double lo = t.empty() ? 0.0 : t[0], hi = lo;
    for (double x : t) {
        lo = std::min(lo, x);
        hi = std::max(hi, x);
    }
    t_lo = lo;
    return fs->period > 0.0 ? fs->period : hi - lo;
}

int make_feat(const lp_fieldset *fs, FeatArgs &a)
{
    a.g = fs->g;
    a.f.slots = fs->dslots;
    a.f.slot_bytes = fs->slot_bytes;
    a.f.scales = fs->dscales;
    a.f.nzl = fs->nzl;
    a.f.steady = fs->npushed == 1;
    a.store = fs->dtype;
    return LP_OK;
}

}  // namespace

extern "C" int surrogate_train(lp_fieldset *fs, lp_model *m, const lp_surrogate_cfg *cfg,
                               lp_train_stats *st, void *stream_)
{
    hipStream_t stream = (hipStream_t)stream_;
    if (!fs || !m || !cfg || !st || cfg->n_segments < 1 || cfg->steps_per_segment < 1 ||
        !(cfg->dt > 0.0) || cfg->round_size < 1 || cfg->batch < 128 || cfg->batch % 128 ||
        cfg->iterations < 1 || !(cfg->lr > 0.0)) {
        lp_set_error("bad surrogate training arguments");
        return LP_EINVAL;
    }
    if (fs->is3d) {
        lp_set_error("the surrogate works on 2D field sets");
        return LP_EINVAL;
    }
    *st = lp_train_stats{};
    double t_lo = 0.0;
    const double P = field_period(fs, t_lo);
    const double seg_t = cfg->steps_per_segment * cfg->dt;
    const int64_t nslots = (int64_t)std::floor((fs->period > 0.0 ? P : P - seg_t) / cfg->dt);
    if (nslots < 1) {
        lp_set_error("the resident snapshots do not span one segment");
        return LP_ETIME;
    }
    DeviceBuf mem;
    const int64_t cap = cfg->n_segments, R = cfg->round_size;
    double *dx0, *dy0, *sx, *sy;
    uint32_t *dround, *idx;
    float *dtgt, *loss_hist;
    unsigned long long *count;
    SCHECK(mem.get(&dx0, cap));
    SCHECK(mem.get(&dy0, cap));
    SCHECK(mem.get(&dround, cap));
    SCHECK(mem.get(&dtgt, 2 * cap));
    SCHECK(mem.get(&sx, R));
    SCHECK(mem.get(&sy, R));
    SCHECK(mem.get(&count, 1));
    SCHECK(mem.get(&idx, (size_t)cfg->batch));
    SCHECK(mem.get(&loss_hist, (size_t)cfg->iterations));
    SCHECK(hipMemsetAsync(count, 0, 8, stream));
    // seeds for the work set (overwritten every round)
    hipLaunchKernelGGL(k_seed, dim3((uint32_t)((R + 255) / 256)), dim3(256), 0, stream, fs->g,
                       fs->dlandnode, R, cfg->seed, 0xFFFFFFFFu, sx, sy);
    SCHECK(hipGetLastError());
    lp_pset *ps = nullptr;
    int rc = pset_create_device(fs, R, sx, sy, nullptr, 0.0, 0, stream, &ps);
    if (rc)
        return rc;
    lp_exec_opts o{};
    o.kernel = LP_KERNEL_RK4;
    o.recovery = LP_DELETE;
    o.stencil_cache = 1;
    std::mt19937_64 gen(cfg->seed);
    std::vector<TimeEntry> tabs;
    std::vector<float> phases;
    Timer tg;
    tg.start(stream);
    int64_t kept = 0, generated = 0;
    uint32_t round = 0;
    const int64_t max_rounds = 3 * ((cap + R - 1) / R) + 4;
    while (kept < cap && (int64_t)round < max_rounds) {
        const int64_t slot = (int64_t)(gen() % (uint64_t)nslots);
        const double t0 = t_lo + (double)slot * cfg->dt;
        TimeEntry e{};
        if ((rc = lp_time_entry(fs, t0, &e))) {
            pset_destroy(ps);
            return rc;
        }
        const double ph = 2.0 * M_PI * std::fmod(t0 - t_lo, P) / P;
        tabs.push_back(e);
        phases.push_back((float)std::sin(ph));
        phases.push_back((float)std::cos(ph));
        hipLaunchKernelGGL(k_seed, dim3((uint32_t)((R + 255) / 256)), dim3(256), 0, stream,
                           fs->g, fs->dlandnode, R, cfg->seed, round, sx, sy);
        SCHECK(hipGetLastError());
        if ((rc = lp_pset_reset_device(ps, R, sx, sy, t0, stream)) ||
            (rc = pset_execute(ps, seg_t, cfg->dt, 0.0, &o, stream))) {
            pset_destroy(ps);
            return rc;
        }
        hipLaunchKernelGGL(k_targets, dim3((uint32_t)((R + 255) / 256)), dim3(256), 0, stream,
                           sx, sy, ps->dx, ps->dy, ps->dst, R, fs->g.spherical, round, dx0, dy0,
                           dround, dtgt, count, cap);
        SCHECK(hipGetLastError());
        generated += R;
        ++round;
        if (round % 16 == 0 || generated >= cap) {
            unsigned long long c = 0;
            SCHECK(hipMemcpyAsync(&c, count, 8, hipMemcpyDeviceToHost, stream));
            SCHECK(hipStreamSynchronize(stream));
            kept = (int64_t)std::min<unsigned long long>(c, (unsigned long long)cap);
        }
    }
    pset_destroy(ps);
    {
        unsigned long long c = 0;
        SCHECK(hipMemcpyAsync(&c, count, 8, hipMemcpyDeviceToHost, stream));
        SCHECK(hipStreamSynchronize(stream));
        kept = (int64_t)std::min<unsigned long long>(c, (unsigned long long)cap);
        st->segments_dropped = generated - (int64_t)c;
    }
    st->segments_kept = kept;
    st->gen_ms = tg.stop_ms(stream);
    if (kept < 1) {
        lp_set_error("no segment stayed in the ocean");
        return LP_ESTATE;
    }
    TimeEntry *dtab;
    float *dphase;
    SCHECK(mem.get(&dtab, tabs.size()));
    SCHECK(mem.get(&dphase, phases.size()));
    SCHECK(hipMemcpy(dtab, tabs.data(), tabs.size() * sizeof(TimeEntry), hipMemcpyHostToDevice));
    SCHECK(hipMemcpy(dphase, phases.data(), phases.size() * 4, hipMemcpyHostToDevice));
    const int64_t B = cfg->batch;
    if ((rc = model_work(m, B)))
        return rc;
    FeatArgs fa{};
    make_feat(fs, fa);
    fa.x = dx0;
    fa.y = dy0;
    fa.sel = idx;
    fa.round = dround;
    fa.tab = dtab;
    fa.phase = dphase;
    fa.n = B;
    fa.npad = B;
    fa.X = m->X;
    fa.tgt = dtgt;
    fa.T = m->T;
    Timer tt;
    tt.start(stream);
    for (int64_t it = 0; it < cfg->iterations; ++it) {
        hipLaunchKernelGGL(k_sample_batch, dim3((uint32_t)((B + 255) / 256)), dim3(256), 0,
                           stream, cfg->seed ^ 0xA5A5A5A5u, (uint32_t)it, kept, B, idx);
        hipLaunchKernelGGL(k_features, dim3((uint32_t)((B + kFeatBlock - 1) / kFeatBlock)),
                           dim3(kFeatBlock), 0, stream, fa);
        SCHECK(hipGetLastError());
        const double frac = (double)it / (double)cfg->iterations;
        const double lr = cfg->lr * (0.05 + 0.95 * 0.5 * (1.0 + std::cos(M_PI * frac)));
        if ((rc = forward(m, B, true, stream)) || (rc = backward(m, B, stream)) ||
            (rc = adam(m, (float)lr, stream)))
            return rc;
        SCHECK(hipMemcpyAsync(loss_hist + it, m->loss, 4, hipMemcpyDeviceToDevice, stream));
    }
    st->train_ms = tt.stop_ms(stream);
    std::vector<float> lh((size_t)cfg->iterations);
    SCHECK(hipMemcpy(lh.data(), loss_hist, lh.size() * 4, hipMemcpyDeviceToHost));
    const int64_t w = std::min<int64_t>(100, cfg->iterations);
    double a = 0.0, b = 0.0;
    for (int64_t k = 0; k < w; ++k) {
        a += lh[(size_t)k];
        b += lh[(size_t)(cfg->iterations - 1 - k)];
    }
    st->first_loss = a / w;
    st->final_loss = b / w;
    st->iterations = cfg->iterations;
    return LP_OK;
}

// ------------------------------------------------------------------ the two steps alone
extern "C" int surrogate_features(lp_fieldset *fs, int64_t n, const double *x, const double *y,
                                  double t, float *X)
{
    if (!fs || n < 0 || (n > 0 && (!x || !y || !X))) {
        lp_set_error("bad surrogate_features arguments");
        return LP_EINVAL;
    }
    if (fs->is3d) {
        lp_set_error("the surrogate works on 2D field sets");
        return LP_EINVAL;
    }
    if (n == 0)
        return LP_OK;
    TimeEntry e{};
    int rc = lp_time_entry(fs, t, &e);
    if (rc)
        return rc;
    double t_lo = 0.0;
    const double P = field_period(fs, t_lo);
    const double ph = P > 0.0 ? 2.0 * M_PI * std::fmod(t - t_lo, P) / P : 0.0;
    const float phs[2] = {(float)std::sin(ph), (float)std::cos(ph)};
    DeviceBuf mem;
    double *dx, *dy;
    TimeEntry *dtab;
    float *dphase;
    uint16_t *dX;
    SCHECK(mem.get(&dx, (size_t)n));
    SCHECK(mem.get(&dy, (size_t)n));
    SCHECK(mem.get(&dtab, 1));
    SCHECK(mem.get(&dphase, 2));
    SCHECK(mem.get(&dX, (size_t)n * kIn));
    SCHECK(hipMemcpy(dx, x, (size_t)n * 8, hipMemcpyHostToDevice));
    SCHECK(hipMemcpy(dy, y, (size_t)n * 8, hipMemcpyHostToDevice));
    SCHECK(hipMemcpy(dtab, &e, sizeof e, hipMemcpyHostToDevice));
    SCHECK(hipMemcpy(dphase, phs, 8, hipMemcpyHostToDevice));
    SCHECK(hipStreamSynchronize(fs->up));  // the snapshots the entry names are in place
    FeatArgs fa{};
    make_feat(fs, fa);
    fa.x = dx;
    fa.y = dy;
    fa.tab = dtab;
    fa.phase = dphase;
    fa.n = n;
    fa.npad = n;
    fa.X = dX;
    hipLaunchKernelGGL(k_features, dim3((uint32_t)((n + kFeatBlock - 1) / kFeatBlock)),
                       dim3(kFeatBlock), 0, nullptr, fa);
    SCHECK(hipGetLastError());
    std::vector<uint16_t> h((size_t)n * kIn);
    SCHECK(hipDeviceSynchronize());
    SCHECK(hipMemcpy(h.data(), dX, h.size() * 2, hipMemcpyDeviceToHost));
    for (size_t q = 0; q < h.size(); ++q) {
        const uint32_t b = (uint32_t)h[q] << 16;
        std::memcpy(&X[q], &b, 4);
    }
    return LP_OK;
}

extern "C" int surrogate_check(lp_fieldset *fs, int64_t n, const double *x0, const double *y0,
                               const double *xc, const double *yc, const uint8_t *coarse_status,
                               const float *Y, double residual_m, uint8_t *accept, double *x1,
                               double *y1)
{
    if (!fs || n < 0 || n > 0x7FFFFFFFll ||
        (n > 0 && (!x0 || !y0 || !xc || !yc || !coarse_status || !Y || !accept || !x1 ||
                   !y1)) ||
        !(residual_m >= 0.0)) {
        lp_set_error("bad surrogate_check arguments");
        return LP_EINVAL;
    }
    if (fs->is3d) {
        lp_set_error("the surrogate works on 2D field sets");
        return LP_EINVAL;
    }
    if (n == 0)
        return LP_OK;
    const size_t N = (size_t)n;
    DeviceBuf mem;
    double *dx, *dy, *dxc, *dyc;
    uint8_t *dst;
    float *dY;
    uint32_t *order, *nact, *fall, *nfall;
    SCHECK(mem.get(&dx, N));
    SCHECK(mem.get(&dy, N));
    SCHECK(mem.get(&dxc, N));
    SCHECK(mem.get(&dyc, N));
    SCHECK(mem.get(&dst, N));
    SCHECK(mem.get(&dY, 2 * N));
    SCHECK(mem.get(&order, N));
    SCHECK(mem.get(&nact, 1));
    SCHECK(mem.get(&fall, N));
    SCHECK(mem.get(&nfall, 1));
    SCHECK(hipMemcpy(dx, x0, N * 8, hipMemcpyHostToDevice));
    SCHECK(hipMemcpy(dy, y0, N * 8, hipMemcpyHostToDevice));
    SCHECK(hipMemcpy(dxc, xc, N * 8, hipMemcpyHostToDevice));
    SCHECK(hipMemcpy(dyc, yc, N * 8, hipMemcpyHostToDevice));
    SCHECK(hipMemcpy(dst, coarse_status, N, hipMemcpyHostToDevice));
    SCHECK(hipMemcpy(dY, Y, N * 8, hipMemcpyHostToDevice));
    SCHECK(lp::launch_iota(order, N, nullptr));
    SCHECK(lp::launch_fill_u32(nact, (uint32_t)n, 1, nullptr));
    SCHECK(lp::launch_fill_u32(nfall, 0u, 1, nullptr));
    hipLaunchKernelGGL(k_check, dim3((uint32_t)((N + kCheckThreads - 1) / kCheckThreads)),
                       dim3(kCheckThreads), 0, nullptr, fs->g, order, nact, dx, dy, dxc, dyc,
                       dst, dY, residual_m, fall, nfall);
    SCHECK(hipGetLastError());
    SCHECK(hipDeviceSynchronize());
    uint32_t nf = 0;
    SCHECK(hipMemcpy(&nf, nfall, 4, hipMemcpyDeviceToHost));
    std::vector<uint32_t> hf(nf);
    if (nf)
        SCHECK(hipMemcpy(hf.data(), fall, (size_t)nf * 4, hipMemcpyDeviceToHost));
    SCHECK(hipMemcpy(x1, dx, N * 8, hipMemcpyDeviceToHost));
    SCHECK(hipMemcpy(y1, dy, N * 8, hipMemcpyDeviceToHost));
    std::memset(accept, 1, N);
    for (uint32_t id : hf)
        accept[id] = 0;
    return LP_OK;
}

// ------------------------------------------------------------------ inference
// Segments between two cell sorts of the active list during inference (a day at 24
// steps of 300 s per segment).  At 1 m/s a particle crosses about three 0.25-degree
// cells a day, small beside the 16 x 16-cell tiles of the sort key, so rows that are
// neighbours in the list stay near each other on the grid between sorts.
constexpr int64_t kSortSegments = 12;

extern "C" int pset_execute_surrogate(lp_pset *ps, lp_model *m, double runtime, double dt,
                                      int32_t steps_per_segment, double residual_m,
                                      lp_surrogate_stats *st, void *stream_)
{
    hipStream_t stream = (hipStream_t)stream_;
    if (!ps || !m || !st || !(dt > 0.0) || steps_per_segment < 2 || !(residual_m >= 0.0) ||
        !(runtime >= 0.0)) {
        lp_set_error("bad surrogate execute arguments");
        return LP_EINVAL;
    }
    lp_fieldset *fs = ps->fs;
    if (fs->is3d) {
        lp_set_error("the surrogate works on 2D field sets");
        return LP_EINVAL;
    }
    const double seg_t = steps_per_segment * dt;
    const int64_t nseg = (int64_t)std::llround(runtime / seg_t);
    if (std::fabs((double)nseg * seg_t - runtime) > 1e-9 * std::max(runtime, seg_t)) {
        lp_set_error("runtime must be a whole number of segments");
        return LP_EINVAL;
    }
    *st = lp_surrogate_stats{};
    if (ps->dt != 0.0 && ps->dt != dt) {
        lp_set_error("the particle set already runs with another dt");
        return LP_EINVAL;
    }
    double t_lo = 0.0;
    const double P = field_period(fs, t_lo);
    const int64_t n = ps->n, rows = round128(n);
    DeviceBuf mem;
    uint32_t *fall, *nfall, *saved_count;
    TimeEntry *dtab;
    float *dphase;
    SCHECK(mem.get(&fall, (size_t)n));
    SCHECK(mem.get(&nfall, 1));
    SCHECK(mem.get(&saved_count, 1));
    SCHECK(mem.get(&dtab, 1));
    SCHECK(mem.get(&dphase, 2));
    // the state in sorted order (see k_permute) and its position -> id map
    uint32_t *pid, *pid2, *perm, *pcnt;
    double *tx, *ty;
    uint8_t *tst;
    SCHECK(mem.get(&pid, (size_t)n));
    SCHECK(mem.get(&pid2, (size_t)n));
    SCHECK(mem.get(&perm, (size_t)n));
    SCHECK(mem.get(&pcnt, 1));
    SCHECK(mem.get(&tx, (size_t)n));
    SCHECK(mem.get(&ty, (size_t)n));
    SCHECK(mem.get(&tst, (size_t)n));
    SCHECK(lp::launch_iota(pid, (size_t)n, stream));
    const uint32_t un = (uint32_t)n, nb = std::max(1u, (un + 255) / 256);
    // the sorts order the list by cell within each tile (the set's own sort buffers are
    // sized for tiles)
    const uint32_t cbins = lp::sort_bins(fs->g, true);
    uint32_t *chist, *cblk;
    SCHECK(mem.get(&chist, (size_t)cbins));
    SCHECK(mem.get(&cblk, lp::sort_blocksums(cbins)));
    int rc = model_work(m, rows);
    if (rc)
        return rc;
    // coarse-RK4 twin of the set
    lp_pset *cs = nullptr;
    if ((rc = pset_create_device(fs, n, ps->dx, ps->dy, nullptr, 0.0, 0, stream, &cs)))
        return rc;
    lp_exec_opts o{};
    o.kernel = LP_KERNEL_RK4;
    o.recovery = LP_DELETE;
    o.stencil_cache = 1;
    o.sort_every = 0;
    // The stream is synchronised once a segment, to read the rejected queue's length; the
    // phase times of a segment are read after the next segment's synchronisation (two sets
    // of events) and the active counts once at the end.
    uint32_t *dna;
    SCHECK(mem.get(&dna, (size_t)std::max<int64_t>(nseg, 1)));
    SegmentEvents ev[2];
    uint64_t nf_sum = 0;
    Timer ttot;
    ttot.start(stream);
    for (int64_t q = 0; q < nseg && rc == LP_OK; ++q) {
        const double t = ps->t0 + (double)ps->step * dt;
        TimeEntry e{};
        if ((rc = lp_time_entry(fs, t, &e)))
            break;
        SegmentEvents &E = ev[q & 1];
        E.sorted = q % kSortSegments == 0;
        // the active list in cell order (cells within tiles), so that neighbouring rows
        // gather neighbouring patches (the fine and coarse twins inherit the order), and the
        // state moved into that order, so that the list becomes 0 .. active - 1
        if (E.sorted) {
            SCHECK(hipEventRecord(E.e[0], stream));
            SCHECK(lp::launch_sort(fs->g, ps->dx, ps->dy, ps->dz, ps->dst, ps->dorder[ps->cur],
                                   ps->dcount + ps->cur, ps->n_launch, ps->dkeys, chist, cbins,
                                   cblk, ps->dorder[1 - ps->cur], ps->dcount + (1 - ps->cur),
                                   stream, true));
            ps->cur = 1 - ps->cur;
            SCHECK(lp::launch_iota(perm, (size_t)n, stream));
            hipLaunchKernelGGL(k_copy_list, dim3(nb), dim3(256), 0, stream, ps->dorder[ps->cur],
                               ps->dcount + ps->cur, perm);
            SCHECK(lp::launch_fill_u32(pcnt, 0u, 1, stream));
            const uint32_t nbc = std::max(1u, (un + kCheckThreads - 1) / kCheckThreads);
            hipLaunchKernelGGL(k_perm_inactive, dim3(nbc), dim3(kCheckThreads), 0, stream,
                               ps->dst, un, ps->dcount + ps->cur, perm, pcnt);
            hipLaunchKernelGGL(k_permute, dim3(nb), dim3(256), 0, stream, perm, un, ps->dx,
                               ps->dy, ps->dst, pid, tx, ty, tst, pid2);
            SCHECK(hipGetLastError());
            std::swap(pid, pid2);
            SCHECK(hipMemcpyAsync(ps->dx, tx, (size_t)n * 8, hipMemcpyDeviceToDevice, stream));
            SCHECK(hipMemcpyAsync(ps->dy, ty, (size_t)n * 8, hipMemcpyDeviceToDevice, stream));
            SCHECK(hipMemcpyAsync(ps->dst, tst, (size_t)n, hipMemcpyDeviceToDevice, stream));
            SCHECK(lp::launch_iota(ps->dorder[ps->cur], (size_t)n, stream));
        }
        const double ph = 2.0 * M_PI * std::fmod(t - t_lo, P) / P;
        const float phs[2] = {(float)std::sin(ph), (float)std::cos(ph)};
        SCHECK(hipMemcpyAsync(dtab, &e, sizeof e, hipMemcpyHostToDevice, stream));
        SCHECK(hipMemcpyAsync(dphase, phs, 8, hipMemcpyHostToDevice, stream));
        const int c0 = ps->cur;
        // network on every active particle
        SCHECK(hipEventRecord(E.e[1], stream));
        FeatArgs fa{};
        make_feat(fs, fa);
        fa.x = ps->dx;
        fa.y = ps->dy;
        fa.sel = ps->dorder[c0];
        fa.tab = dtab;
        fa.phase = dphase;
        fa.n_dev = ps->dcount + c0;
        fa.npad = rows;
        fa.X = m->X;
        hipLaunchKernelGGL(k_features, dim3((uint32_t)((rows + kFeatBlock - 1) / kFeatBlock)),
                           dim3(kFeatBlock), 0, stream, fa);
        SCHECK(hipGetLastError());
        if ((rc = forward(m, rows, false, stream)))
            break;
        SCHECK(hipEventRecord(E.e[2], stream));
        // coarse RK4: two steps over the segment from the same state
        SCHECK(hipMemcpyAsync(cs->dx, ps->dx, (size_t)n * 8, hipMemcpyDeviceToDevice, stream));
        SCHECK(hipMemcpyAsync(cs->dy, ps->dy, (size_t)n * 8, hipMemcpyDeviceToDevice, stream));
        SCHECK(hipMemcpyAsync(cs->dst, ps->dst, (size_t)n, hipMemcpyDeviceToDevice, stream));
        SCHECK(hipMemcpyAsync(cs->dorder[0], ps->dorder[c0], (size_t)n * 4,
                              hipMemcpyDeviceToDevice, stream));
        SCHECK(hipMemcpyAsync(cs->dcount, ps->dcount + c0, 4, hipMemcpyDeviceToDevice, stream));
        cs->cur = 0;
        cs->n_launch = ps->n_launch;
        cs->count_pending = false;
        cs->t0 = t;
        cs->dt = 0.0;
        cs->step = 0;
        if ((rc = pset_execute(cs, seg_t, seg_t / 2, 0.0, &o, stream)))
            break;
        SCHECK(hipEventRecord(E.e[3], stream));
        // residual check; the rest goes to the fine RK4 steps
        SCHECK(hipMemsetAsync(nfall, 0, 4, stream));
        hipLaunchKernelGGL(k_check, dim3((ps->n_launch + kCheckThreads - 1) / kCheckThreads),
                           dim3(kCheckThreads), 0, stream,
                           fs->g, ps->dorder[c0], ps->dcount + c0, ps->dx, ps->dy, cs->dx,
                           cs->dy, cs->dst, m->Y, residual_m, fall, nfall);
        SCHECK(hipGetLastError());
        uint32_t *full = ps->dorder[c0];
        SCHECK(hipMemcpyAsync(saved_count, ps->dcount + c0, 4, hipMemcpyDeviceToDevice, stream));
        SCHECK(hipMemcpyAsync(ps->dcount + c0, nfall, 4, hipMemcpyDeviceToDevice, stream));
        ps->dorder[c0] = fall;
        // The fine steps' launch spans the queue's own blocks (read back first): sized for the
        // whole set, its remap onto the XCDs would give the queue, a short prefix of the
        // grid, to the first one or two of them.  One block at least, since the call also
        // advances the set's clock.
        uint32_t nf = 0;
        SCHECK(hipMemcpyAsync(&nf, nfall, 4, hipMemcpyDeviceToHost, stream));
        SCHECK(hipStreamSynchronize(stream));
        ev[(q + 1) & 1].account(st);  // the previous segment's events have all passed
        const uint32_t n_full = ps->n_launch;
        ps->n_launch = std::max(nf, 1u);
        rc = pset_execute(ps, seg_t, dt, 0.0, &o, stream);
        ps->n_launch = n_full;
        ps->dorder[c0] = full;
        ps->count_pending = false;  // its count is the fallback list's, not the set's
        if (rc)
            break;
        // the new active list: every particle of the full list still active
        SCHECK(lp::launch_compact(full, saved_count, ps->dst, ps->dorder[1 - c0],
                                  ps->dcount + (1 - c0), ps->n_launch, stream));
        ps->cur = 1 - c0;
        SCHECK(hipEventRecord(E.e[4], stream));
        E.live = true;
        SCHECK(hipMemcpyAsync(dna + q, saved_count, 4, hipMemcpyDeviceToDevice, stream));
        nf_sum += nf;
        st->segments++;
    }
    pset_destroy(cs);
    // the state back in id order, the active list as ids
    hipLaunchKernelGGL(k_unpermute, dim3(nb), dim3(256), 0, stream, pid, un, ps->dx, ps->dy,
                       ps->dst, tx, ty, tst);
    SCHECK(hipGetLastError());
    SCHECK(hipMemcpyAsync(ps->dx, tx, (size_t)n * 8, hipMemcpyDeviceToDevice, stream));
    SCHECK(hipMemcpyAsync(ps->dy, ty, (size_t)n * 8, hipMemcpyDeviceToDevice, stream));
    SCHECK(hipMemcpyAsync(ps->dst, tst, (size_t)n, hipMemcpyDeviceToDevice, stream));
    hipLaunchKernelGGL(k_map_ids, dim3(nb), dim3(256), 0, stream, pid, ps->dcount + ps->cur,
                       ps->dorder[ps->cur], ps->dorder[1 - ps->cur]);
    SCHECK(hipGetLastError());
    SCHECK(hipMemcpyAsync(ps->dcount + (1 - ps->cur), ps->dcount + ps->cur, 4,
                          hipMemcpyDeviceToDevice, stream));
    ps->cur = 1 - ps->cur;
    if (rc)
        return rc;
    st->total_ms = ttot.stop_ms(stream);
    ev[0].account(st);
    ev[1].account(st);
    std::vector<uint32_t> na((size_t)st->segments);
    if (!na.empty())
        SCHECK(hipMemcpy(na.data(), dna, na.size() * 4, hipMemcpyDeviceToHost));
    for (uint32_t v : na)
        st->evaluated += v;
    st->fallback = (int64_t)nf_sum;
    st->accepted = st->evaluated - st->fallback;  // every active particle is one or the other
    return LP_OK;
}
