// advect.hip -- per-particle RK4 advection through gridded velocity snapshots.
//
// One particle per lane; each lane keeps its position in registers for all the
// steps of a launch.  Every RK stage samples the velocity as in the paper's field
// access fieldset.F[time, lon, lat, depth] (Sect. 2.1.2): find the cell on the
// rectilinear grid (Sect. 2.4), interpolate linearly in space (bilinear in 2D,
// trilinear in 3D; Sect. 2.3), then linearly between the two bracketing
// snapshots (Sect. 2.4), and on a spherical mesh convert m/s to degrees/s
// (Sect. 4.2.2).  The stages combine with the classical RK4 weights (Sect. 2.1.1,
// Eq. 1); the Brownian term of Eq. (1) is the optional Philox kick (Sect. 4.2.7).
// Particles that leave the grid or end in a land cell get status bits instead of
// moving (the recovery kernels of Sect. 2.1.2).
//
// Storage types: LP_F64 / LP_F32 snapshots are interpolated in FP64; LP_BF16 and
// LP_F16_SCALED snapshots are interpolated in FP32 and only the position update
// runs in FP64.
#include <type_traits>

#include "lp_internal.h"

namespace lp {

// The counter slot of this block (see kCountSlots).
__device__ inline unsigned long long *count_slot(unsigned long long *c)
{
    return c + (blockIdx.x % kCountSlots) * kCountStride;
}

namespace {

constexpr uint8_t ST_OOB = 1, ST_LAND = 2, ST_DELETED = 4, ST_AGED = 8;

// Blocks are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).  Map
// the hardware block id so that each XCD works on one contiguous range of the
// (tile-sorted) particle order and keeps that region's stencils in its own L2.
__device__ inline uint32_t xcd_block(uint32_t b, uint32_t nb)
{
    const uint32_t q = nb >> 3, r = nb & 7u;
    const uint32_t x = b & 7u, local = b >> 3;
    return x * q + (x < r ? x : r) + local;
}

// What a reload reads in place of an absent per-cell table (no land mask, or no latitude
// tables on a flat mesh): a zero in device memory, so that the read needs no branch and
// goes out with the reload's other reads instead of after them.
__device__ double kAbsentTable = 0.0;  // never written; not const, so it sits in global memory as the tables do

// The cell search of a reload, in three phases that the reload runs across all three
// axes before moving on, so that the axes' memory reads overlap: the guess (as in
// locate), one 16-byte read of the guessed cell's two faces c[g] and c[g + 1], and the
// correction against them.  The result is locate's index, with the faces of its cell.
// x must lie in [c0, c(n-1)].
__device__ inline int axis_guess(const AxisDev &a, double x)
{
    int g;
    if (a.uniform) {
        g = (int)((x - a.lo) * a.ginv);
    } else {
        int b = (int)((x - a.lo) * a.ginv);
        b = b < kGuessBins - 1 ? b : kGuessBins - 1;
        g = a.guess[b];
    }
    return g < 0 ? 0 : (g > a.n - 2 ? a.n - 2 : g);
}

__device__ inline void axis_faces(const AxisDev &a, int g, double &lo, double &hi)
{
    // 8-byte alignment suffices for a global vector load
    typedef double FacePair __attribute__((ext_vector_type(2), aligned(8)));
    const FacePair p = *reinterpret_cast<const FacePair *>(a.c + g);
    lo = p.x;
    hi = p.y;
}

__device__ inline void axis_correct(const AxisDev &a, double x, int &g, double &lo, double &hi)
{
    while (g > 0 && lo > x) {
        --g;
        hi = lo;
        lo = a.c[g];
    }
    while (g < a.n - 2 && hi <= x) {
        ++g;
        lo = hi;
        hi = a.c[g + 1];
    }
}

// One axis's cell search split in two phases, so that a caller can run each phase
// across all its axes and their reads overlap: find_start takes the guess and issues
// the reads of the guessed cell (its faces, and its inverse width when the fraction is
// wanted); find_finish corrects against the faces, reading the width again only if the
// cell moved.  The result is the largest i in [0, n-2] with c[i] <= x, for x in
// [c0, c(n-1)]; the guess (closed form for a uniform axis, a bin table otherwise) only
// decides where the search starts, so the index follows the stored grid exactly.
struct AxisFind {
    int g, g0;
    double lo, hi, rw;
};

__device__ inline bool on_axis(const AxisDev &a, double x) { return x >= a.lo && x <= a.hi; }

template <bool FRAC>
__device__ inline void find_start(const AxisDev &a, double x, AxisFind &s)
{
    s.g = s.g0 = axis_guess(a, x);
    axis_faces(a, s.g, s.lo, s.hi);
    if constexpr (FRAC)
        s.rw = a.rw[s.g];
}

template <bool FRAC>
__device__ inline void find_finish(const AxisDev &a, double x, AxisFind &s)
{
    axis_correct(a, x, s.g, s.lo, s.hi);
    if constexpr (FRAC) {
        if (s.g != s.g0)
            s.rw = a.rw[s.g];
    }
}

// Cell search on one axis: the cell index i and the fraction (x - c[i]) / (c[i+1] - c[i]),
// or false if x is NaN or outside [c0, c(n-1)].
__device__ inline bool locate(const AxisDev &a, double x, int &i, double &f)
{
    if (!on_axis(a, x))
        return false;
    AxisFind s;
    find_start<true>(a, x, s);
    find_finish<true>(a, x, s);
    i = s.g;
    f = (x - s.lo) * s.rw;
    return true;
}

template <int ST> struct Real { using T = double; };
template <> struct Real<kBF16> { using T = float; };
template <> struct Real<kF16S> { using T = float; };

__device__ inline float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ inline float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }
__device__ inline float f16_lo(uint32_t w)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w & 0xFFFFu));
}
__device__ inline float f16_hi(uint32_t w)
{
    return (float)__builtin_bit_cast(_Float16, (uint16_t)(w >> 16));
}

// Load (U, V[, W]) of one node of one snapshot slot.
template <int ST, bool IS3D>
__device__ inline void load_node(const char *slot, size_t node, const float *sc,
                                 typename Real<ST>::T v[3])
{
    if constexpr (ST == kF64) {
        if constexpr (IS3D) {
            const double4 q = reinterpret_cast<const double4 *>(slot)[node];
            v[0] = q.x; v[1] = q.y; v[2] = q.z;
        } else {
            const double2 q = reinterpret_cast<const double2 *>(slot)[node];
            v[0] = q.x; v[1] = q.y; v[2] = 0.0;
        }
    } else if constexpr (ST == kF32) {
        if constexpr (IS3D) {
            const float4 q = reinterpret_cast<const float4 *>(slot)[node];
            v[0] = q.x; v[1] = q.y; v[2] = q.z;
        } else {
            const float2 q = reinterpret_cast<const float2 *>(slot)[node];
            v[0] = q.x; v[1] = q.y; v[2] = 0.0;
        }
    } else if constexpr (ST == kBF16) {
        if constexpr (IS3D) {
            const uint2 q = reinterpret_cast<const uint2 *>(slot)[node];
            v[0] = bf16_lo(q.x); v[1] = bf16_hi(q.x); v[2] = bf16_lo(q.y);
        } else {
            const uint32_t q = reinterpret_cast<const uint32_t *>(slot)[node];
            v[0] = bf16_lo(q); v[1] = bf16_hi(q); v[2] = 0.f;
        }
    } else {
        if constexpr (IS3D) {
            const uint2 q = reinterpret_cast<const uint2 *>(slot)[node];
            v[0] = f16_lo(q.x) * sc[0]; v[1] = f16_hi(q.x) * sc[1]; v[2] = f16_lo(q.y) * sc[2];
        } else {
            const uint32_t q = reinterpret_cast<const uint32_t *>(slot)[node];
            v[0] = f16_lo(q) * sc[0]; v[1] = f16_hi(q) * sc[1]; v[2] = 0.f;
        }
    }
}

struct Cell {
    int i, j, k;
    double xi, eta, zeta;
};

// The cell of a point (as locate on each axis), the axes searched together so that their
// reads overlap; false if the point is outside the grid or NaN.  The fractions are
// computed only if FRAC (else zero); in 2D, k and zeta are zero.
template <bool IS3D, bool FRAC>
__device__ inline bool locate_point(const GridDev &g, double x, double y, double z, Cell &c)
{
    if (!(on_axis(g.ax, x) && on_axis(g.ay, y) && (!IS3D || on_axis(g.az, z))))
        return false;
    AxisFind fx, fy, fz;
    find_start<FRAC>(g.ax, x, fx);
    find_start<FRAC>(g.ay, y, fy);
    if constexpr (IS3D)
        find_start<FRAC>(g.az, z, fz);
    find_finish<FRAC>(g.ax, x, fx);
    find_finish<FRAC>(g.ay, y, fy);
    if constexpr (IS3D)
        find_finish<FRAC>(g.az, z, fz);
    c.i = fx.g;
    c.j = fy.g;
    c.k = IS3D ? fz.g : 0;
    c.xi = FRAC ? (x - fx.lo) * fx.rw : 0.0;
    c.eta = FRAC ? (y - fy.lo) * fy.rw : 0.0;
    c.zeta = FRAC && IS3D ? (z - fz.lo) * fz.rw : 0.0;
    return true;
}

// The status a step's end point takes: ST_OOB off the grid (or NaN), ST_LAND in a land
// cell, else 0.  Without a land mask (a branch uniform across the launch) only the
// bounds matter and no memory is read; with one, only the horizontal cell is searched.
template <bool IS3D>
__device__ inline uint8_t point_status(const GridDev &g, double x, double y, double z)
{
    if (!(on_axis(g.ax, x) && on_axis(g.ay, y) && (!IS3D || on_axis(g.az, z))))
        return ST_OOB;
    if (!g.landcell)
        return 0;
    Cell cs;
    locate_point<false, false>(g, x, y, 0.0, cs);
    return g.landcell[(size_t)cs.j * (size_t)(g.ax.n - 1) + (size_t)cs.i] ? ST_LAND : 0;
}

// Bilinear interpolation of level k in one slot: the four corner weights times the
// corner values, summed in the order (0,0), (1,0), (1,1), (0,1).
template <int ST, bool IS3D>
__device__ inline void bilinear(const AdvectParams &P, const char *slot, int sidx, int k,
                                const Cell &c, typename Real<ST>::T out[3])
{
    using R = typename Real<ST>::T;
    const size_t nx = (size_t)P.g.ax.n;
    const size_t plane = nx * (size_t)P.g.ay.n;
    const size_t n00 = (size_t)k * plane + (size_t)c.j * nx + (size_t)c.i;
    const float *sc = nullptr;
    if constexpr (ST == kF16S)
        sc = P.f.scales + ((size_t)sidx * P.f.nzl + k) * 3;
    R f00[3], f10[3], f11[3], f01[3];
    load_node<ST, IS3D>(slot, n00, sc, f00);
    load_node<ST, IS3D>(slot, n00 + 1, sc, f10);
    load_node<ST, IS3D>(slot, n00 + nx + 1, sc, f11);
    load_node<ST, IS3D>(slot, n00 + nx, sc, f01);
    const R xi = (R)c.xi, eta = (R)c.eta;
    const R w00 = ((R)1 - xi) * ((R)1 - eta), w10 = xi * ((R)1 - eta);
    const R w11 = xi * eta, w01 = ((R)1 - xi) * eta;
#pragma unroll
    for (int q = 0; q < (IS3D ? 3 : 2); ++q)
        out[q] = ((w00 * f00[q] + w10 * f10[q]) + w11 * f11[q]) + w01 * f01[q];
}

template <int ST, bool IS3D>
__device__ inline void spatial(const AdvectParams &P, int sidx, const Cell &c,
                               typename Real<ST>::T out[3])
{
    using R = typename Real<ST>::T;
    const char *slot = static_cast<const char *>(P.f.slots) + (size_t)sidx * P.f.slot_bytes;
    if constexpr (!IS3D) {
        bilinear<ST, false>(P, slot, sidx, 0, c, out);
        out[2] = (R)0;
    } else {
        R lo[3], hi[3];
        bilinear<ST, true>(P, slot, sidx, c.k, c, lo);
        bilinear<ST, true>(P, slot, sidx, c.k + 1, c, hi);
        const R z = (R)c.zeta;
#pragma unroll
        for (int q = 0; q < 3; ++q)
            out[q] = ((R)1 - z) * lo[q] + z * hi[q];
    }
}

// A sample's velocity in coordinate units per second (degrees on the sphere).
template <int ST>
__device__ inline bool sample_finish(const AdvectParams &P, double y,
                                     const typename Real<ST>::T v[3], double k[3])
{
    using R = typename Real<ST>::T;
    if (P.g.spherical) {
        if constexpr (sizeof(R) == 8) {
            k[0] = v[0] / (kMetresPerDegree * cos(y * kDegToRad));
            k[1] = v[1] / kMetresPerDegree;
        } else {
            const float cl = cosf((float)(y * kDegToRad));
            k[0] = (double)(v[0] / ((float)kMetresPerDegree * cl));
            k[1] = (double)(v[1] / (float)kMetresPerDegree);
        }
    } else {
        k[0] = (double)v[0];
        k[1] = (double)v[1];
    }
    k[2] = (double)v[2];
    return true;
}

// The four corner values of cell (i, j) in one 2D slot, in the order bilinear sums them:
// (0,0), (1,0), (1,1), (0,1).
template <int ST>
__device__ inline void corners2(const AdvectParams &P, int sidx, int i, int j,
                                typename Real<ST>::T f[4][3])
{
    const size_t nx = (size_t)P.g.ax.n;
    const char *slot = static_cast<const char *>(P.f.slots) + (size_t)sidx * P.f.slot_bytes;
    const size_t n00 = (size_t)j * nx + (size_t)i;
    const float *sc = ST == kF16S ? P.f.scales + (size_t)sidx * P.f.nzl * 3 : nullptr;
    load_node<ST, false>(slot, n00, sc, f[0]);
    load_node<ST, false>(slot, n00 + 1, sc, f[1]);
    load_node<ST, false>(slot, n00 + nx + 1, sc, f[2]);
    load_node<ST, false>(slot, n00 + nx, sc, f[3]);
}

// bilinear's sum on corner values already read
template <int ST>
__device__ inline void bilinear_from(const typename Real<ST>::T f[4][3], double xi, double eta,
                                     typename Real<ST>::T out[3])
{
    using R = typename Real<ST>::T;
    const R x = (R)xi, e = (R)eta;
    const R w00 = ((R)1 - x) * ((R)1 - e), w10 = x * ((R)1 - e);
    const R w11 = x * e, w01 = ((R)1 - x) * e;
#pragma unroll
    for (int q = 0; q < 2; ++q)
        out[q] = ((w00 * f[0][q] + w10 * f[1][q]) + w11 * f[2][q]) + w01 * f[3][q];
    out[2] = (R)0;
}

// The 2D gather of one stage with its reads overlapped: the corner values of the
// guessed cell (inside the grid, whatever the guess) are read together with that
// cell's faces and widths, and read again only where the correction moves the cell.
// The arithmetic is the same as locate_point followed by spatial.
template <int ST, bool STEADY>
__device__ inline bool gather2(const AdvectParams &P, const TimeEntry &te, double x, double y,
                               typename Real<ST>::T a[3], typename Real<ST>::T b[3])
{
    using R = typename Real<ST>::T;
    const GridDev &g = P.g;
    if (!(on_axis(g.ax, x) && on_axis(g.ay, y)))
        return false;
    AxisFind fx, fy;
    find_start<true>(g.ax, x, fx);
    find_start<true>(g.ay, y, fy);
    R fa[4][3], fb[4][3];
    corners2<ST>(P, te.sa, fx.g, fy.g, fa);
    if constexpr (!STEADY)
        corners2<ST>(P, te.sb, fx.g, fy.g, fb);
    find_finish<true>(g.ax, x, fx);
    find_finish<true>(g.ay, y, fy);
    if (fx.g != fx.g0 || fy.g != fy.g0) {
        corners2<ST>(P, te.sa, fx.g, fy.g, fa);
        if constexpr (!STEADY)
            corners2<ST>(P, te.sb, fx.g, fy.g, fb);
    }
    double xi = (x - fx.lo) * fx.rw, eta = (y - fy.lo) * fy.rw;
    if (P.nearest) {
        xi = xi < 0.5 ? 0.0 : 1.0;
        eta = eta < 0.5 ? 0.0 : 1.0;
    }
    bilinear_from<ST>(fa, xi, eta, a);
    if constexpr (!STEADY)
        bilinear_from<ST>(fb, xi, eta, b);
    return true;
}

// Velocity at a stage point in coordinate units per second; false if outside.  SPEC
// reads the corners of the guessed cell together with its faces (2D only): the RKF45
// lane on FP32 fields gains 4% from it; in the RK4 gather kernels the registers it
// holds cost as much as it saves, and the other storage forms of the RKF45 lane spill.
template <int ST, bool IS3D, bool STEADY, bool SPEC = false>
__device__ inline bool sample(const AdvectParams &P, const TimeEntry &te, double x, double y,
                              double z, double k[3])
{
    using R = typename Real<ST>::T;
    R v[3];
    if constexpr (SPEC && !IS3D) {
        R a[3], b[3];
        if (!gather2<ST, STEADY>(P, te, x, y, a, b))
            return false;
        if constexpr (STEADY) {
#pragma unroll
            for (int q = 0; q < 3; ++q)
                v[q] = a[q];
        } else {
            const R tau = (R)te.tau;
#pragma unroll
            for (int q = 0; q < 3; ++q)
                v[q] = ((R)1 - tau) * a[q] + tau * b[q];
        }
        return sample_finish<ST>(P, y, v, k);
    }
    Cell c;
    if (!locate_point<IS3D, true>(P.g, x, y, z, c))
        return false;
    if (P.nearest) {
        c.xi = c.xi < 0.5 ? 0.0 : 1.0;
        c.eta = c.eta < 0.5 ? 0.0 : 1.0;
        c.zeta = c.zeta < 0.5 ? 0.0 : 1.0;
    }
    if constexpr (STEADY) {
        spatial<ST, IS3D>(P, te.sa, c, v);
    } else {
        R a[3], b[3];
        spatial<ST, IS3D>(P, te.sa, c, a);
        spatial<ST, IS3D>(P, te.sb, c, b);
        const R tau = (R)te.tau;
#pragma unroll
        for (int q = 0; q < 3; ++q)
            v[q] = ((R)1 - tau) * a[q] + tau * b[q];
    }
    return sample_finish<ST>(P, y, v, k);
}

// Philox4x32-10 (Salmon et al., SC'11): ten Philox-4x32 rounds, key bumped by the
// Weyl constants between rounds.
__device__ inline void philox4x32_10(uint32_t c[4], uint32_t k0, uint32_t k1)
{
    constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    constexpr uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        if (r) {
            k0 += W0;
            k1 += W1;
        }
        // one 32 x 32 -> 64-bit product each (a single v_mad_u64_u32)
        const uint64_t p0 = (uint64_t)M0 * c[0], p1 = (uint64_t)M1 * c[2];
        const uint32_t lo0 = (uint32_t)p0, hi0 = (uint32_t)(p0 >> 32);
        const uint32_t lo1 = (uint32_t)p1, hi1 = (uint32_t)(p1 >> 32);
        const uint32_t n0 = hi1 ^ c[1] ^ k0, n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
}

__device__ inline double unit53(uint32_t a, uint32_t b)
{
    const uint64_t m = (((uint64_t)a << 32) | (uint64_t)b) >> 11;
    return (double)m * 0x1p-53 + 0x1p-54;
}

// 1 / d to within an ulp or two: hardware reciprocal refined by two Newton steps
__device__ inline double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    return r;
}

// sin and cos of 2 pi u for u in [0, 1].  The argument is a fraction of a turn, so the
// reduction to a quarter turn is exact: 4u = q + f with q = rint(4u) and |f| <= 1/2,
// 2 pi u = q pi/2 + f pi/2.  sin(f pi/2) and cos(f pi/2) come from their Taylor series
// in f (coefficients (pi/2)^n / n!), cut after the f^17 and f^16 terms (the first
// terms left out are below 1e-19 and 3e-18 at |f| = 1/2), and the quadrant q mod 4
// rotates the pair.
// The polynomial coefficients of sincos_turn and log_unit, in constant memory: the
// Brownian kernels read them with scalar loads inside their step loop (an index the
// compiler cannot prove constant keeps the loads there), so that they do not sit in
// vector registers across the loop.
__constant__ double kBmCoef[28] = {
    // sin(f pi/2) / f, highest power first (9)
    0x1.aaec32af93359p-38, -0x1.6fadb9f155744p-31, 0x1.e8f434d018d63p-25,
    -0x1.e3074fde8871fp-19, 0x1.50783487ee782p-13, -0x1.32d2cce62bd86p-8,
    0x1.466bc6775aae2p-4, -0x1.4abbce625be53p-1, 0x1.921fb54442d18p+0,
    // (cos(f pi/2) - 1) / f^2, highest power first (8)
    0x1.20c62c2f2d7f5p-34, -0x1.b6e24f44b128fp-28, 0x1.f9d38a3763cc3p-22,
    -0x1.a6d1f2a204a8cp-16, 0x1.e1f506891babbp-11, -0x1.55d3c7e3cbffap-6,
    0x1.03c1f081b5ac4p-2, -0x1.3bd3cc9be45dep+0,
    // atanh series 1/19 .. 1/3 (9)
    1.0 / 19.0, 1.0 / 17.0, 1.0 / 15.0, 1.0 / 13.0, 1.0 / 11.0, 1.0 / 9.0, 1.0 / 7.0,
    1.0 / 5.0, 1.0 / 3.0,
    // log 2, head and tail (2)
    0x1.62e42fefa3800p-1, 0x1.ef35793c76730p-45};

__device__ inline void sincos_turn(double u, double &sn, double &cs,
                                   const double *k = kBmCoef)
{
    const double t = 4.0 * u;
    const double q = rint(t);
    const double f = t - q;  // exact
    const double f2 = f * f;
    double ps = k[0];
#pragma unroll
    for (int i = 1; i < 9; ++i)
        ps = fma(ps, f2, k[i]);
    const double S = ps * f;
    double pc = k[9];
#pragma unroll
    for (int i = 10; i < 17; ++i)
        pc = fma(pc, f2, k[i]);
    const double C = fma(pc, f2, 1.0);
    const int qi = (int)q;
    double a = (qi & 1) ? C : S, b = (qi & 1) ? S : C;
    sn = (qi & 2) ? -a : a;
    cs = ((qi + 1) & 2) ? -b : b;
}

// Natural logarithm of u in (0, 1] (the uniforms of unit53).  u = m 2^e with m in
// [sqrt(1/2), sqrt(2)); log m = 2 atanh(s) with s = (m - 1) / (m + 1), |s| < 0.1716,
// from the series atanh(s) = s + s^3/3 + s^5/5 + ..., cut after s^19 (the first term
// left out is below 2.4e-17 relative); e log 2 with log 2 split into a head whose
// products with |e| < 2^11 are exact and a tail.  Within about two ulps.
__device__ inline double log_unit(double u, const double *k = kBmCoef)
{
    int e;
    double m = frexp(u, &e);  // m in [1/2, 1)
    if (m < 0.70710678118654752) {
        m = 2.0 * m;
        e -= 1;
    }
    const double num = m - 1.0, den = m + 1.0;  // num exact
    double r = __builtin_amdgcn_rcp(den);
    r = fma(fma(-den, r, 1.0), r, r);
    r = fma(fma(-den, r, 1.0), r, r);
    double sq = num * r;
    sq = fma(fma(-den, sq, num), r, sq);  // s to within an ulp
    const double z = sq * sq;
    double p = k[17];
#pragma unroll
    for (int i = 18; i < 26; ++i)
        p = fma(p, z, k[i]);
    const double s2 = 2.0 * sq;
    const double lm = fma(s2 * z, p, s2);  // log m
    const double de = (double)e;
    return fma(de, k[26], fma(de, k[27], lm));
}

// Square root of x in [2^-60, 2^60]: the hardware reciprocal square root refined by two
// Newton steps for 1/sqrt(x), then y = x r with one correction (x - y^2) r / 2.  Within
// about an ulp.
__device__ inline double sqrt_mid(double x)
{
    double r = __builtin_amdgcn_rsq(x);
    const double hx = 0.5 * x;
    r = r * fma(-hx * r, r, 1.5);
    r = r * fma(-hx * r, r, 1.5);
    const double y = x * r;
    return fma(fma(-y, y, x), 0.5 * r, y);
}

// cos of a latitude in degrees, |lat| <= 90: a quarter turn at most, through the turn
// form (lat / 360 of a turn; the division rounds once, as lat * pi / 180 does).
__device__ inline double cos_deg(double lat)
{
    double sn, cs;
    sincos_turn(lat * (1.0 / 360.0), sn, cs);
    return cs;
}

// Two standard normals from two uniforms (Box-Muller); k: the coefficient table.
__device__ inline void box_muller(double u1, double u2, double &n1, double &n2,
                                  const double *k = kBmCoef)
{
    const double r = sqrt_mid(-2.0 * log_unit(u1, k));
    double sn, cs;
    sincos_turn(u2, sn, cs, k);
    n1 = r * cs;
    n2 = r * sn;
}

// The random term of Eq. (1) for one step, in metres: sqrt(2 Kh |dt|) times the two
// normals drawn from the particle's Philox words for (id, step).
// LOOP_LOADS: read the Box-Muller coefficients inside the step loop (P.zero is 0 at
// run time, but the compiler cannot know it, so the scalar loads stay in the loop
// instead of the constants occupying vector registers across it).  That pays in the
// flat Brownian kernels (it takes them from 3 to 4 waves per SIMD); the spherical
// ones, with the metric's extra state, are faster with the constants in place.
template <bool LOOP_LOADS>
__device__ inline void brownian_metres(const AdvectParams &P, uint32_t id, int64_t step,
                                       double dt, double &dx, double &dy)
{
    uint32_t w[4] = {id, (uint32_t)step, 0u, 0u};
    philox4x32_10(w, P.run_id, P.seed);
    double n1, n2;
    box_muller(unit53(w[0], w[1]), unit53(w[2], w[3]), n1, n2,
               LOOP_LOADS ? kBmCoef + (P.zero & (uint32_t)step) : kBmCoef);
    const double sig = sqrt(2.0 * P.Kh * fabs(dt));
    dx = sig * n1;
    dy = sig * n2;
}

template <int ST, bool IS3D, bool STEADY, bool BROWN>
__device__ inline uint8_t rk4_step(const AdvectParams &P, int s, uint32_t id, double &x,
                                   double &y, double &z, bool horizontal = false)
{
    const TimeEntry e0 = P.tab[2 * s], e1 = P.tab[2 * s + 1], e2 = P.tab[2 * s + 2];
    const double dt = P.dt, hd = 0.5 * dt;
    // a stage whose point is off the grid leaves its slope at zero and the later
    // stages run on (a sample only reads the cell it located); the step then fails
    double k1[3] = {0.0, 0.0, 0.0}, k2[3] = {0.0, 0.0, 0.0}, k3[3] = {0.0, 0.0, 0.0},
           k4[3] = {0.0, 0.0, 0.0};
    bool ok = sample<ST, IS3D, STEADY>(P, e0, x, y, z, k1);
    double xs, ys, zs = z;
    if (P.scheme) {  // Euler forward
        xs = x + k1[0] * dt;
        ys = y + k1[1] * dt;
        if constexpr (IS3D)
            zs = z + k1[2] * dt;
    } else {
        ok = sample<ST, IS3D, STEADY>(P, e1, x + k1[0] * hd, y + k1[1] * hd, z + k1[2] * hd,
                                      k2) & ok;
        ok = sample<ST, IS3D, STEADY>(P, e1, x + k2[0] * hd, y + k2[1] * hd, z + k2[2] * hd,
                                      k3) & ok;
        ok = sample<ST, IS3D, STEADY>(P, e2, x + k3[0] * dt, y + k3[1] * dt, z + k3[2] * dt,
                                      k4) & ok;
        xs = x + ((((k1[0] + 2.0 * k2[0]) + 2.0 * k3[0]) + k4[0]) * dt) / 6.0;
        ys = y + ((((k1[1] + 2.0 * k2[1]) + 2.0 * k3[1]) + k4[1]) * dt) / 6.0;
        if constexpr (IS3D)
            zs = z + ((((k1[2] + 2.0 * k2[2]) + 2.0 * k3[2]) + k4[2]) * dt) / 6.0;
    }
    if (!ok)
        return ST_OOB;
    if constexpr (IS3D) {
        if (horizontal)  // a dwelling particle keeps its depth
            zs = z;
    }
    if (BROWN && P.Kh > 0.0) {
        double dx, dy;
        brownian_metres<false>(P, id, P.step0 + s, dt, dx, dy);
        if (P.g.spherical) {
            dx = dx * recip(kMetresPerDegree * cos_deg(ys));
            dy = dy / kMetresPerDegree;
        }
        xs = xs + dx;
        ys = ys + dy;
    }
    if (const uint8_t e = point_status<IS3D>(P.g, xs, ys, zs))
        return e;
    x = xs;
    y = ys;
    z = zs;
    return 0;
}

// Tracer at (x, y, z) for the time entry te: trilinear (bilinear in 2D) on the
// float tracer slots in FP64, then linear in time; false outside the grid.
template <bool IS3D, bool STEADY>
__device__ inline bool sample_tracer(const AdvectParams &P, const TimeEntry &te, double x,
                                     double y, double z, double &val)
{
    Cell c;
    if (!locate_point<IS3D, true>(P.g, x, y, z, c))
        return false;
    const size_t nx = (size_t)P.g.ax.n, plane = nx * (size_t)P.g.ay.n;
    auto level = [&](int slot, int k) {
        const float *F = P.f.tracer + ((size_t)slot * P.f.nzl + (size_t)k) * plane;
        const size_t n00 = (size_t)c.j * nx + (size_t)c.i;
        const double w00 = (1.0 - c.xi) * (1.0 - c.eta), w10 = c.xi * (1.0 - c.eta);
        const double w11 = c.xi * c.eta, w01 = (1.0 - c.xi) * c.eta;
        return ((w00 * (double)F[n00] + w10 * (double)F[n00 + 1]) +
                w11 * (double)F[n00 + nx + 1]) + w01 * (double)F[n00 + nx];
    };
    auto spatial_t = [&](int slot) {
        if constexpr (!IS3D)
            return level(slot, 0);
        return (1.0 - c.zeta) * level(slot, c.k) + c.zeta * level(slot, c.k + 1);
    };
    if constexpr (STEADY)
        val = spatial_t(te.sa);
    else
        val = (1.0 - te.tau) * spatial_t(te.sa) + te.tau * spatial_t(te.sb);
    return true;
}

// The worked example's kernels ahead of the advection of step s (sinking, age,
// tracer sample); returns a status to stop with, or 0.  The sinking update is
// rounded as written (no contraction) so that reaching the dwelling depth is the
// same decision as in a plain FP64 evaluation.
template <bool IS3D, bool STEADY>
__device__ inline uint8_t behave_pre(const AdvectParams &P, int s, double x, double y,
                                     double &z, double &temp, double &age, bool &horizontal)
{
    const bool sinking = IS3D && P.sink_speed > 0.0;
    if (sinking && z > P.dwell_depth) {
        const double zn = __dadd_rn(z, __dmul_rn(P.sink_speed, P.dt));
        z = zn > P.dwell_depth ? zn : P.dwell_depth;
    }
    const bool dwelling = !sinking || z <= P.dwell_depth;
    if (P.maxage > 0.0 && dwelling) {
        age = age + fabs(P.dt);
        if (age >= P.maxage)
            return (uint8_t)(ST_AGED | ST_DELETED);
    }
    if (P.sample) {
        double v;
        if (!sample_tracer<IS3D, STEADY>(P, P.tab[2 * s], x, y, z, v))
            return (uint8_t)(ST_OOB | (P.policy == 0 ? ST_DELETED : 0));
        temp = v;
    }
    horizontal = sinking && dwelling;
    return 0;
}

// The Brownian term is a compile-time mode here as in the cached kernels: its
// constants would otherwise stay in registers across the step loop of every launch.
template <int ST, bool IS3D, bool STEADY, bool BROWN>
__global__ __launch_bounds__(kBlock) void k_advect(AdvectParams P)
{
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t k = blk * kBlock + threadIdx.x;
    const uint32_t nact = *P.n_active;
    long long steps = 0;
    if (k < nact) {
        const uint32_t id = P.order[k];
        uint8_t st = P.status[id];
        if (st == 0) {
            double x = P.x[id], y = P.y[id], z = IS3D ? P.z[id] : 0.0;
            double temp = 0.0, age = 0.0;
            if (P.behave) {
                temp = P.temp[id];
                age = P.age[id];
            }
            for (int s = 0; s < P.nsteps; ++s) {
                ++steps;
                bool horizontal = false;
                if (P.behave) {
                    const uint8_t b = behave_pre<IS3D, STEADY>(P, s, x, y, z, temp, age,
                                                               horizontal);
                    if (b) {
                        st = b;
                        break;
                    }
                }
                const uint8_t e =
                    rk4_step<ST, IS3D, STEADY, BROWN>(P, s, id, x, y, z, horizontal);
                if (e) {
                    st = (uint8_t)(e | (P.policy == 0 ? ST_DELETED : 0));
                    break;
                }
            }
            P.x[id] = x;
            P.y[id] = y;
            if constexpr (IS3D)
                P.z[id] = z;
            if (P.behave) {
                P.temp[id] = temp;
                P.age[id] = age;
            }
            if (st)
                P.status[id] = st;
        }
    }
    for (int off = 32; off > 0; off >>= 1)
        steps += __shfl_xor(steps, off, 64);
    if ((threadIdx.x & 63) == 0 && steps)
        atomicAdd(count_slot(P.psteps), (unsigned long long)steps);
}

// ---------------------------------------------------------------- adaptive RKF45
// The Runge-Kutta-Fehlberg option of Sect. 2.1.1 with a per-particle step |dt| 2^e.
// Each lane runs its own sequence of attempts from t_start to t_end, so its stage
// times are its own: the bracketing snapshots of each stage time are found per
// lane in the resident-snapshot table, with the same arithmetic as the host's
// stage-time table (periodic fields first map t into [T0, T0 + period)).
// fmod(a, P) for P > 0 (and |a / P| < 2^51), bit for bit: the remainder a - n P
// with n = trunc(a / P) is exactly representable, so once the estimate of n from
// a / P is corrected by at most one, the fused multiply-add returns it unrounded.
__device__ inline double exact_fmod(double a, double P, double invP)
{
    double n = trunc(a * invP);
    double r = fma(-n, P, a);
    if (a >= 0.0) {
        if (r < 0.0) {
            n -= 1.0;
            r = fma(-n, P, a);
        } else if (r >= P) {
            n += 1.0;
            r = fma(-n, P, a);
        }
    } else {
        if (r > 0.0) {
            n += 1.0;
            r = fma(-n, P, a);
        } else if (r <= -P) {
            n -= 1.0;
            r = fma(-n, P, a);
        }
    }
    return r;
}

// A lane's current bracket: the resident-table index lo and the times around it.
struct LaneTime {
    double t_lo, t_hi;
    int32_t lo, sa, sb;
};

__device__ inline TimeEntry bracket_lane(const AdvectParams &P, double t, LaneTime &b)
{
    const ResTime *r = P.res;
    const int m = P.nres;
    TimeEntry e;
    if (P.f.steady) {
        e.tau = 0.0;
        e.sa = e.sb = r[0].slot;
        return e;
    }
    const bool periodic = P.period > 0.0;
    double tp = t;
    double T0 = 0.0;
    if (periodic) {
        T0 = r[0].t;
        double q = exact_fmod(t - T0, P.period, P.inv_period);
        if (q < 0.0)
            q += P.period;
        tp = T0 + q;
    }
    // fast path: still inside the lane's bracket (strictly below its upper end, so
    // the index is the largest one at or below tp, as in the host's search)
    if (!(b.lo >= 0 && tp >= b.t_lo && tp < b.t_hi)) {
        int lo = 0, hi = periodic ? m - 1 : m - 2;  // the host checked [t_start, t_end]
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (r[mid].t <= tp)
                lo = mid;
            else
                hi = mid - 1;
        }
        b.lo = lo;
        b.t_lo = r[lo].t;
        b.sa = r[lo].slot;
        if (lo + 1 < m) {
            b.t_hi = r[lo + 1].t;
            b.sb = r[lo + 1].slot;
        } else {  // periodic wrap: the first snapshot again, one period later
            b.t_hi = T0 + P.period;
            b.sb = r[0].slot;
        }
    }
    e.sa = b.sa;
    e.sb = b.sb;
    e.tau = (tp - b.t_lo) / (b.t_hi - b.t_lo);
    return e;
}

// Fehlberg 4(5) pair: nodes, stage matrix, fourth-order weights, and the
// differences fifth- minus fourth-order weights (the error estimate).
struct Fehlberg {
    static constexpr double c[6] = {0.0, 1.0 / 4.0, 3.0 / 8.0, 12.0 / 13.0, 1.0, 1.0 / 2.0};
    static constexpr double a[6][5] = {
        {0.0, 0.0, 0.0, 0.0, 0.0},
        {1.0 / 4.0, 0.0, 0.0, 0.0, 0.0},
        {3.0 / 32.0, 9.0 / 32.0, 0.0, 0.0, 0.0},
        {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0.0, 0.0},
        {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0.0},
        {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0}};
    static constexpr double b4[6] = {25.0 / 216.0, 0.0, 1408.0 / 2565.0, 2197.0 / 4104.0,
                                     -1.0 / 5.0, 0.0};
    static constexpr double b5[6] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0,
                                     -9.0 / 50.0, 2.0 / 55.0};
};

// One attempt of signed size h from p at time t: fourth-order end point p4 and
// error estimate ev (fifth minus fourth order); false if a stage leaves the grid.
template <int ST, bool IS3D, bool STEADY>
__device__ inline bool rkf45_attempt(const AdvectParams &P, double t, double h,
                                     const double p[3], double p4[3], double ev[3],
                                     LaneTime &lt)
{
    double k[6][3] = {};
    bool ok = true;  // as in the RK4 step: a failed stage leaves a zero slope
#pragma unroll
    for (int i = 0; i < 6; ++i) {
        double q[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            double s = 0.0;
#pragma unroll
            for (int j = 0; j < i; ++j)
                s = s + Fehlberg::a[i][j] * k[j][d];
            q[d] = p[d] + h * s;
        }
        const TimeEntry te = bracket_lane(P, t + Fehlberg::c[i] * h, lt);
        ok = sample<ST, IS3D, STEADY, ST == kF32>(P, te, q[0], q[1], q[2], k[i]) & ok;
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        double s4 = 0.0, se = 0.0;
#pragma unroll
        for (int i = 0; i < 6; ++i) {
            s4 = s4 + Fehlberg::b4[i] * k[i][d];
            se = se + (Fehlberg::b5[i] - Fehlberg::b4[i]) * k[i][d];
        }
        p4[d] = p[d] + h * s4;
        ev[d] = h * se;
    }
    if constexpr (!IS3D) {
        p4[2] = p[2];
        ev[2] = 0.0;
    }
    return ok;
}

// The step control shared by both RKF45 lanes: an attempt whose error length is
// above tol is retried at e - 1 (unless e is at its floor); an accepted one that
// passes the end-point checks moves the lane's time on and, if it was a full step
// with error at most tol / 32, raises e for the next one.
struct RkfState {
    double t;
    int32_t e, it;
    uint32_t id;
    uint8_t st;
};

__device__ inline bool rkf_accept(const AdvectParams &P, RkfState &s, double err,
                                  long long &acc, long long &rej)
{
    if (err > P.tol && s.e > P.emin) {
        --s.e;
        ++rej;
        return false;
    }
    ++acc;
    return true;
}

__device__ inline void rkf_commit(const AdvectParams &P, RkfState &s, double err, bool cut,
                                  double hs)
{
    s.t = cut ? P.t_end : s.t + hs;
    if (!cut && err <= P.tol * 0.03125 && s.e < P.emax)
        ++s.e;
}

// One particle's state for the gather form (2D or 3D): every stage gathers its
// stencil from the snapshots.
template <int ST, bool IS3D, bool STEADY>
struct GatherLane {
    RkfState s;
    double p[3];
    LaneTime lt;

    __device__ void begin(const AdvectParams &P, uint32_t id)
    {
        s.id = id;
        s.st = 0;
        s.t = P.t_start;
        s.e = P.hexp[id];
        s.it = 0;
        p[0] = P.x[id];
        p[1] = P.y[id];
        p[2] = IS3D ? P.z[id] : 0.0;
        lt.lo = -1;
    }

    // one attempt; true when the particle is done for this launch
    __device__ bool attempt(const AdvectParams &P, long long &acc, long long &rej)
    {
        const uint8_t extra = P.policy == 0 ? ST_DELETED : 0;
        if (s.t == P.t_end)
            return true;
        if (s.it++ >= P.max_iter) {  // never reached: see max_iter
            s.st = (uint8_t)(ST_OOB | extra);
            return true;
        }
        const double sg = P.dt > 0.0 ? 1.0 : -1.0;
        const double h = ldexp(fabs(P.dt), s.e);
        const double rem = sg > 0.0 ? P.t_end - s.t : s.t - P.t_end;
        const bool cut = h >= rem;
        const double hs = sg * (cut ? rem : h);
        double p4[3], ev[3];
        if (!rkf45_attempt<ST, IS3D, STEADY>(P, s.t, hs, p, p4, ev, lt)) {
            ++acc;
            s.st = (uint8_t)(ST_OOB | extra);
            return true;
        }
        double ex = ev[0], ey = ev[1];
        if (P.g.spherical) {
            ex = ex * (kMetresPerDegree * cos(p[1] * kDegToRad));
            ey = ey * kMetresPerDegree;
        }
        const double err = sqrt((ex * ex + ey * ey) + ev[2] * ev[2]);
        if (!rkf_accept(P, s, err, acc, rej))
            return false;
        if (const uint8_t e = point_status<IS3D>(P.g, p4[0], p4[1], p4[2])) {
            s.st = (uint8_t)(e | extra);
            return true;
        }
        p[0] = p4[0];
        p[1] = p4[1];
        p[2] = p4[2];
        rkf_commit(P, s, err, cut, hs);
        return s.t == P.t_end;
    }

    __device__ void finish(const AdvectParams &P)
    {
        P.x[s.id] = p[0];
        P.y[s.id] = p[1];
        if constexpr (IS3D)
            P.z[s.id] = p[2];
        P.hexp[s.id] = (int8_t)s.e;
        if (s.st)
            P.status[s.id] = s.st;
    }
};

// ---------------------------------------------------------------- 2D with a stencil cache
// Each lane keeps the stencil of the cell it is in, as the coefficients of the
// bilinear polynomial f = c0 + c1 xi + c2 eta + c3 xi eta of U and V for the
// earlier snapshot and for the difference (later - earlier).  A stage point in the
// cached cell then costs only arithmetic: the stencil is reloaded when the point
// leaves the cell or when the time bracket moves on.  The polynomial is the same
// bilinear interpolant as the corner-weight form (Sect. 2.3), and (1 - tau) f_a +
// tau f_b, taken on the coefficients or on the values, is the linear time
// interpolation (Sect. 2.4); only rounding differs.
// NL of the 16 coefficients (the last NL) sit in the lane's LDS slot and the others
// in registers: LDS frees registers, so more waves fit on a SIMD, at the cost of LDS
// reads every stage; the split is chosen per kernel mode (cache_lds_coefs).
template <class R, int NL>
struct Cell2 {
    double x0, ux, y0, uy;  // lower faces; exclusive upper faces (for the last cell the
                            // next double above the last node, so the domain's closed
                            // upper end needs no separate test)
    double rx, ry;          // inverse cell widths
    double cl, sl;          // cos and sin of the lower latitude face
    // U, V coefficients of the earlier snapshot [0..7] and of the later one [8..15]
    R *lc;                  // LDS: this lane's first 16-byte group of coefficients
                            // 16 - NL .. 15 (see cache_slot_ptr)
    uint32_t gs;            // elements from one of the lane's groups to the next
    R lr[NL < 16 ? 16 - NL : 1];  // registers: coefficients 0 .. 15 - NL
    bool land;
    static constexpr int G = 16 / (int)sizeof(R);  // coefficients per 16-byte group
    __device__ R &lds(int j) { return lc[(j / G) * gs + j % G]; }
    __device__ R lds(int j) const { return lc[(j / G) * gs + j % G]; }
    __device__ R &coef(int i) { return i < 16 - NL ? lr[i] : lds(i - (16 - NL)); }
    __device__ R coef(int i) const { return i < 16 - NL ? lr[i] : lds(i - (16 - NL)); }
    // no point is in the cell until the next reload (an empty x range also keeps a
    // NaN position out)
    __device__ void invalidate()
    {
        x0 = __builtin_inf();
        ux = -__builtin_inf();
    }
    // a fresh cell: every field defined (a stage whose point is off the grid still
    // evaluates the cell it has, and discards the result)
    __device__ void clear()
    {
        y0 = uy = rx = ry = cl = sl = 0.0;
        for (int i = 0; i < (NL < 16 ? 16 - NL : 1); ++i)
            lr[i] = (R)0;
        land = false;
        invalidate();
    }
};

// The 2D stencil cache in LDS is an array of 16-byte groups, group g of thread t at
// (g * blockDim + t) * 16 bytes: a wave's read of one group covers 1 KB of consecutive
// words (no bank conflicts) and a lane needs no padding, so NL doubles take exactly
// 8 NL bytes per lane (5 waves per SIMD of 16 coefficients fit the 160 KB).  Elements
// of R per lane, for the launch's LDS size:
template <class R, int NL>
constexpr int cache_slot() { return NL; }

template <class R, int NL>
__device__ inline R *cache_slot_ptr()
{
    extern __shared__ __attribute__((aligned(16))) unsigned char cache_lds[];
    return reinterpret_cast<R *>(cache_lds) + threadIdx.x * (16 / sizeof(R));
}

template <class R>
__device__ inline uint32_t cache_group_stride()
{
    return blockDim.x * (16 / (uint32_t)sizeof(R));
}

// How many coefficients the cached 2D kernels keep in LDS: with the Brownian term
// the kernel holds enough other state that the occupancy is the same either way, so
// all stay in registers; otherwise all go to LDS (with the unrolled stages, register
// coefficients cost a copy of themselves at every stage's join of the cached and
// reloaded paths).
template <int ST, bool BROWN>
constexpr int cache_lds_coefs() { return BROWN ? 0 : 16; }

// Metric modes of the cached kernels, fixed at compile time so that a launch carries
// only the code it runs: flat mesh; spherical with the latitude tables and a series
// whose length (3 or 4 terms) is read at run time; spherical with cells too tall for
// the series (library cos); spherical with the 2-term series (cells up to 0.3 degree,
// the common fine-grid case, with no branch on the length).
enum : int { kFlat = 0, kSphTable = 1, kSphLib = 2, kSphTable2 = 3 };

// Whether the cached 2D kernels keep the V coefficients in degrees of latitude per
// second (divided by M at the reload), so that a stage's northward slope needs no
// product: FP64 coefficients on the sphere.
template <class R, int MET>
constexpr bool v_in_degrees() { return sizeof(R) == 8 && MET != kFlat; }

template <class R>
__device__ inline void coeffs(const R f00, const R f10, const R f01, const R f11, R c[4])
{
    c[0] = f00;
    c[1] = f10 - f00;
    c[2] = f01 - f00;
    c[3] = (f11 - f10) - c[2];
}

template <class R>
__device__ inline R poly(const R c[4], R xi, R eta)
{
    return fma(eta, fma(xi, c[3], c[2]), fma(xi, c[1], c[0]));
}

template <int ST, bool STEADY, int MET, int NL>
__device__ inline bool reload2(const AdvectParams &P, Cell2<typename Real<ST>::T, NL> &c, int sa,
                               int sb, double x, double y)
{
    using R = typename Real<ST>::T;
    const AxisDev &ax = P.g.ax, &ay = P.g.ay;
    if (!(x >= ax.lo && x <= ax.hi && y >= ay.lo && y <= ay.hi))
        return false;
    // the cell search of both axes in phases, then every read of the cell issued before
    // any of its values is used (as in the 3D reload)
    int i = axis_guess(ax, x), j = axis_guess(ay, y);
    double xh, yh;
    axis_faces(ax, i, c.x0, xh);
    axis_faces(ay, j, c.y0, yh);
    axis_correct(ax, x, i, c.x0, xh);
    axis_correct(ay, y, j, c.y0, yh);
    c.ux = (i == ax.n - 2) ? nextafter(ax.hi, __builtin_inf()) : xh;
    c.uy = (j == ay.n - 2) ? nextafter(ay.hi, __builtin_inf()) : yh;
    const size_t nx = (size_t)ax.n;
    const size_t n00 = (size_t)j * nx + (size_t)i;
    const char *base = static_cast<const char *>(P.f.slots);
    const char *A = base + (size_t)sa * P.f.slot_bytes;
    const float *sca = ST == kF16S ? P.f.scales + (size_t)sa * P.f.nzl * 3 : nullptr;
    R p00[3], p10[3], p01[3], p11[3];
    load_node<ST, false>(A, n00, sca, p00);
    load_node<ST, false>(A, n00 + 1, sca, p10);
    load_node<ST, false>(A, n00 + nx, sca, p01);
    load_node<ST, false>(A, n00 + nx + 1, sca, p11);
    const char *B = base + (size_t)sb * P.f.slot_bytes;
    const float *scb = ST == kF16S ? P.f.scales + (size_t)sb * P.f.nzl * 3 : nullptr;
    R q00[3], q10[3], q01[3], q11[3];
    if constexpr (!STEADY) {
        load_node<ST, false>(B, n00, scb, q00);
        load_node<ST, false>(B, n00 + 1, scb, q10);
        load_node<ST, false>(B, n00 + nx, scb, q01);
        load_node<ST, false>(B, n00 + nx + 1, scb, q11);
    }
    c.rx = ax.rw[i];
    c.ry = ay.rw[j];
    const double clat = *(P.g.coslat ? P.g.coslat + j : &kAbsentTable);
    const double slat = *(P.g.coslat ? P.g.sinlat + j : &kAbsentTable);
    const uint32_t land = *(P.g.landcell ? P.g.landcell + ((size_t)j * (nx - 1) + (size_t)i)
                                         : reinterpret_cast<const uint8_t *>(&kAbsentTable));
    if constexpr (!STEADY) {
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            R ca[4], cb[4];
            coeffs<R>(q00[v], q10[v], q01[v], q11[v], cb);
            coeffs<R>(p00[v], p10[v], p01[v], p11[v], ca);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const R w = v == 1 && v_in_degrees<R, MET>() ? (R)(1.0 / kMetresPerDegree) : (R)1;
                c.coef(4 * v + q) = ca[q] * w;
                c.coef(8 + 4 * v + q) = cb[q] * w;
            }
        }
    } else {
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            R ca[4];
            coeffs<R>(p00[v], p10[v], p01[v], p11[v], ca);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const R w = v == 1 && v_in_degrees<R, MET>() ? (R)(1.0 / kMetresPerDegree) : (R)1;
                c.coef(4 * v + q) = ca[q] * w;
            }
        }
    }
    c.cl = kMetresPerDegree * clat;
    c.sl = kMetresPerDegree * slat;
    c.land = land != 0;
    return true;
}

template <class R, int NL>
__device__ inline bool in_cell(const Cell2<R, NL> &c, const AdvectParams &P, double x, double y)
{
    return x >= c.x0 && x < c.ux && y >= c.y0 && y < c.uy;
}

// Whether two time-table entries interpolate between the same two snapshots.
__device__ inline bool same_bracket(const TimeEntry &a, const TimeEntry &b)
{
    return a.sa == b.sa && a.sb == b.sb;
}

// The cached kernels' stencils hold the bracket of the stage before; this says, for
// stage q of step s, whether the bracket moves on there (or nothing is cached yet:
// the launch's first stage), so that the stage reloads whatever cell its point is
// in.  Every active lane of a wave runs the same stages, so the answer is
// wave-uniform and comes from the table alone: RK4's first stage reuses the entry of
// the previous step's last stage, its third the second's; Euler's only stage follows
// the previous step's.
struct BracketMoves {
    uint32_t bits;  // bit q: stage q reloads
    __device__ BracketMoves(const AdvectParams &P, int s, const TimeEntry &e0,
                            const TimeEntry &e1, const TimeEntry &e2)
    {
        const bool q0 = s == 0 || (P.scheme && !same_bracket(P.tab[2 * s - 2], e0));
        bits = (uint32_t)q0 | ((uint32_t)!same_bracket(e0, e1) << 1) |
               ((uint32_t)!same_bracket(e1, e2) << 3);
    }
    __device__ bool at(int q) const { return (bits >> q) & 1u; }
};


// cos of a latitude inside the cached cell: cos(l0 + dl) = cos l0 cos dl - sin l0 sin dl
// with dl = lat - l0 and cos dl, sin dl by their Taylor series, cut after 2, 3 or 4
// terms so that the truncation stays below a quarter ulp for the grid's tallest cell
// (0.3, 1.5 or 5 degrees).
__device__ inline double cos_series(double cl, double sl, double y0, double y, int terms)
{
    const double dl = (y - y0) * kDegToRad, d2 = dl * dl;
    double cd, sd;
    if (terms <= 2) {
        cd = fma(d2, fma(d2, 1.0 / 24.0, -0.5), 1.0);
        sd = dl * fma(d2, fma(d2, 1.0 / 120.0, -1.0 / 6.0), 1.0);
    } else if (terms == 3) {
        cd = fma(d2, fma(d2, fma(d2, -1.0 / 720.0, 1.0 / 24.0), -0.5), 1.0);
        sd = dl * fma(d2, fma(d2, fma(d2, -1.0 / 5040.0, 1.0 / 120.0), -1.0 / 6.0), 1.0);
    } else {
        cd = fma(d2, fma(d2, fma(d2, fma(d2, 1.0 / 40320.0, -1.0 / 720.0), 1.0 / 24.0), -0.5),
                 1.0);
        sd = dl * fma(d2, fma(d2, fma(d2, fma(d2, 1.0 / 362880.0, -1.0 / 5040.0), 1.0 / 120.0),
                              -1.0 / 6.0), 1.0);
    }
    return cl * cd - sl * sd;
}

template <int MET>
constexpr bool met_series() { return MET == kSphTable || MET == kSphTable2; }

// M cos(lat) inside a cell at most 0.3 degrees tall, for the slopes of the RK4 stages:
// cos(d) = 1 - d^2/2 + d^4/24 and sin(d) = d (1 - d^2/6) across the cell (d < 5.3e-3
// rad); the truncation, d^6/720 of the cosine and d^5/120 of the sine, stays below
// 4e-14 of the metric (1e-16 on the 0.1 degree grid).
__device__ inline double mcos_short(double cl, double sl, double y0, double y)
{
    const double dl = (y - y0) * kDegToRad, d2 = dl * dl;
    const double cd = fma(d2, fma(d2, 1.0 / 24.0, -0.5), 1.0);
    const double sd = dl * fma(d2, -1.0 / 6.0, 1.0);
    return fma(cl, cd, -sl * sd);
}

// 1/d for the slopes of the RK4 stages: the hardware reciprocal (about 25 bits) and one
// Newton step, within 11 ulp (1.2e-15 relative).
__device__ inline double recip_stage(double d)
{
    const double r = __builtin_amdgcn_rcp(d);
    return fma(fma(-d, r, 1.0), r, r);
}

template <int MET>
__device__ inline double cos_series_m(double cl, double sl, double y0, double y,
                                      const AdvectParams &P)
{
    return cos_series(cl, sl, y0, y, MET == kSphTable2 ? 2 : P.g.cos_terms);
}

// Metres per degree of longitude at latitude y inside the cached cell, M cos(lat): the
// cells keep M cos and M sin of their lower face, so the series gives the product.
template <int MET, class R, int NL>
__device__ inline double metres_lon(const Cell2<R, NL> &c, const AdvectParams &P, double y)
{
    if constexpr (MET == kSphLib)
        return kMetresPerDegree * cos(y * kDegToRad);
    else
        return cos_series_m<MET>(c.cl, c.sl, c.y0, y, P);
}



// 1 / (M cos(lat)) at a stage point inside the cached cell, for the slope of an RK4
// stage: the short series in cells of at most 0.3 degrees, else the cell's series (or
// the library cosine), then one Newton step on the hardware reciprocal.
template <int MET, class CellT>
__device__ inline double stage_metric(const CellT &c, const AdvectParams &P, double y)
{
    double m;
    if constexpr (MET == kSphLib)
        m = kMetresPerDegree * cos(y * kDegToRad);
    else if constexpr (MET == kSphTable2)
        m = mcos_short(c.cl, c.sl, c.y0, y);
    else
        m = cos_series_m<MET>(c.cl, c.sl, c.y0, y, P);
    return recip_stage(m);
}

// 1 / (M cos(lat)) at the end point of a step, for the metric of the Brownian term: the
// cached cell's series when the latitude is inside the cell's band (where the series
// holds), else the turn form of the cosine.
template <int MET, class CellT>
__device__ inline double inv_metres_lon(const CellT &c, const AdvectParams &P, double y)
{
    if (met_series<MET>() && y >= c.y0 && y < c.uy)
        return recip(cos_series_m<MET>(c.cl, c.sl, c.y0, y, P));
    return recip(kMetresPerDegree * cos_deg(y));
}

// The U and V coefficients at a stage's time, (1 - tau) earlier + tau later: exactly the
// earlier snapshot's at tau = 0 and the later one's at tau = 1, so a time that falls on a
// snapshot gives the same coefficients whichever of its two brackets the table names.
template <bool STEADY, class R, int NL>
__device__ inline void coefs_at(const Cell2<R, NL> &c, double tau_d, R tc[8])
{
    const R tau = (R)tau_d, omt = (R)1 - tau;
#pragma unroll
    for (int i = 0; i < 8; ++i)
        tc[i] = STEADY ? c.coef(i) : fma(tau, c.coef(8 + i), omt * c.coef(i));
}

// U and V at (xi, eta) and a stage's time from the two snapshots' values, with the
// same endpoint property (fewer operations when the coefficients are not kept).
template <bool STEADY, class R, int NL>
__device__ inline void values_at(const Cell2<R, NL> &c, double tau_d, R xi, R eta, R &u, R &v)
{
    R q[16];
#pragma unroll
    for (int i = 0; i < (STEADY ? 8 : 16); ++i)
        q[i] = c.coef(i);
    u = poly<R>(q + 0, xi, eta);
    v = poly<R>(q + 4, xi, eta);
    if constexpr (!STEADY) {
        const R tau = (R)tau_d, omt = (R)1 - tau;
        u = fma(tau, poly<R>(q + 8, xi, eta), omt * u);
        v = fma(tau, poly<R>(q + 12, xi, eta), omt * v);
    }
}

template <int ST, bool STEADY, int MET, int NL>
__device__ inline bool stage2(const AdvectParams &P, Cell2<typename Real<ST>::T, NL> &c,
                              const TimeEntry &e, bool fresh, double x, double y, double &kx,
                              double &ky)
{
    using R = typename Real<ST>::T;
    if (!in_cell(c, P, x, y) | fresh) {
        if (!reload2<ST, STEADY, MET, NL>(P, c, e.sa, e.sb, x, y))
            return false;
    }
    const R xi = (R)((x - c.x0) * c.rx), eta = (R)((y - c.y0) * c.ry);
    R u, v;
    values_at<STEADY>(c, e.tau, xi, eta, u, v);
    if constexpr (MET != kFlat) {
        kx = (double)u * stage_metric<MET>(c, P, y);
        ky = v_in_degrees<R, MET>() ? (double)v : (double)v * (1.0 / kMetresPerDegree);
    } else {
        kx = (double)u;
        ky = (double)v;
    }
    return true;
}

// A stage of the cached RK4 lane on the coefficients at the stage's time, tc = (1 - tau)
// earlier + tau later: U in tc[0..3], V in tc[4..7].  With keep, tc stands
// from the stage before, whose time entry was the same, unless the point leaves the
// cached cell (or the bracket moves), so such a stage reads no LDS.  A point off the
// grid leaves the cell as it was and returns false.
template <int ST, bool STEADY, int MET, int NL>
__device__ inline bool stage2_tc(const AdvectParams &P, Cell2<typename Real<ST>::T, NL> &c,
                                 const TimeEntry &e, bool fresh, bool keep, double x, double y,
                                 typename Real<ST>::T tc[8], double &kx, double &ky)
{
    using R = typename Real<ST>::T;
    bool ok = true;
    const bool moved = !in_cell(c, P, x, y) | fresh;
    if (moved)
        ok = reload2<ST, STEADY, MET, NL>(P, c, e.sa, e.sb, x, y);
    const R xi = (R)((x - c.x0) * c.rx), eta = (R)((y - c.y0) * c.ry);
    R u, v;
    if constexpr (NL == 0) {  // coefficients in registers: nothing is kept
        values_at<STEADY>(c, e.tau, xi, eta, u, v);
    } else {
        if (moved | !keep)
            coefs_at<STEADY>(c, e.tau, tc);
        u = poly<R>(tc + 0, xi, eta);
        v = poly<R>(tc + 4, xi, eta);
    }
    if constexpr (MET != kFlat) {
        kx = (double)u * stage_metric<MET>(c, P, y);
        ky = v_in_degrees<R, MET>() ? (double)v : (double)v * (1.0 / kMetresPerDegree);
    } else {
        kx = (double)u;
        ky = (double)v;
    }
    return ok;
}

// One particle (position k of the processing order) for all steps of the launch;
// returns the number of steps it started active.
template <int ST, bool STEADY, int MET, bool BROWN, uint32_t BS>
__device__ inline long long advect_lane_2d(const AdvectParams &P, uint32_t k, uint32_t nact)
{
    using R = typename Real<ST>::T;
    long long steps = 0;
    if (k < nact) {
        const uint32_t id = P.order[k];
        uint8_t st = P.status[id];
        if (st == 0) {
            double x = P.x[id], y = P.y[id];
            constexpr int NL = cache_lds_coefs<ST, BROWN>();
            Cell2<R, NL> c;
            c.clear();
            if constexpr (NL > 0) {
                c.lc = cache_slot_ptr<R, NL>();
                // a block size known at compile time makes every group's offset an
                // immediate of the LDS read
                c.gs = BS ? BS * (16 / (uint32_t)sizeof(R)) : cache_group_stride<R>();
            }
            R tc[8] = {};  // coefficients at the last stage's time
            const double dt = P.dt, dt6 = P.dt6;
            for (int s = 0; s < P.nsteps; ++s) {
                ++steps;
                const TimeEntry e0 = P.tab[2 * s], e1 = P.tab[2 * s + 1], e2 = P.tab[2 * s + 2];
                const BracketMoves moves(P, s, e0, e1, e2);
                uint8_t err = ST_OOB;
                // the four stages: offsets 0, dt/2, dt/2, dt from X_n along the previous
                // slope; weights 1, 2, 2, 1.  A stage whose point is off the grid leaves
                // its slope as it was and the later stages run on (their loads stay in
                // bounds: a reload only reads the cell it located); the step then fails.
                double kx = 0.0, ky = 0.0, sx = 0.0, sy = 0.0;
                bool ok = true;
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (q > 0 && P.scheme)  // Euler forward: one stage
                        break;
                    // stage constants (folded by the unrolling): time entry and
                    // offset along the previous slope; the slopes are summed with
                    // weights 1, 2, 2 here and stage 4's is added after the loop
                    const TimeEntry e = q == 0 ? e0 : (q == 3 ? e2 : e1);
                    const double h = q == 3 ? dt : P.hdt;  // (a scalar operand)
                    const double px = q == 0 ? x : x + kx * h, py = q == 0 ? y : y + ky * h;
                    // stage 3 has stage 2's time entry; RK4's stage 1 has the previous
                    // step's stage 4's (its bracket cannot have moved since)
                    const bool keep = NL > 0 && (q == 2 || (q == 0 && !P.scheme));
                    ok = stage2_tc<ST, STEADY, MET, NL>(P, c, e, moves.at(q), keep, px, py, tc,
                                                        kx, ky) & ok;
                    if (q == 0) {
                        sx = kx;
                        sy = ky;
                    } else if (q < 3) {
                        sx = fma(2.0, kx, sx);
                        sy = fma(2.0, ky, sy);
                    }
                }
                if (!ok)
                    goto fail;
                {
                    double xs, ys;
                    if (P.scheme) {  // Euler forward
                        xs = x + kx * dt;
                        ys = y + ky * dt;
                    } else {
                        xs = x + (sx + kx) * dt6;
                        ys = y + (sy + ky) * dt6;
                    }
                    if (BROWN && P.Kh > 0.0) {
                        double dx, dy;
                        brownian_metres<MET == kFlat>(P, id, P.step0 + s, dt, dx, dy);
                        if constexpr (MET != kFlat) {
                            dx = dx * inv_metres_lon<MET>(c, P, ys);
                            dy = dy / kMetresPerDegree;
                        }
                        xs = xs + dx;
                        ys = ys + dy;
                    }
                    bool land;
                    if (in_cell(c, P, xs, ys)) {
                        land = c.land;
                    } else {
                        const uint8_t e = point_status<false>(P.g, xs, ys, 0.0);
                        if (e & ST_OOB)
                            goto fail;
                        land = e != 0;
                    }
                    if (land) {
                        err = ST_LAND;
                        goto fail;
                    }
                    x = xs;
                    y = ys;
                }
                continue;
            fail:
                st = (uint8_t)(err | (P.policy == 0 ? ST_DELETED : 0));
                break;
            }
            // as in 3D, the Brownian kernels recompute the addresses from the id (the
            // offset is zero), which frees registers for the Philox state (+1.4%); in the
            // plain kernel the same change measured 0.6% slower
            const uint32_t sid = id + (BROWN ? P.zero : 0u);
            P.x[sid] = x;
            P.y[sid] = y;
            if (st)
                P.status[sid] = st;
        }
    }
    return steps;
}

// Occupancy targets: 4 waves per SIMD with the LDS cache (the 8 coefficients at the
// stage time that the lane keeps between stages take the registers of a fifth wave;
// the LDS saved, a quarter to a half of the reads, is worth more), 3 with the Brownian
// term.
template <int ST, bool STEADY, int MET, bool BROWN>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(
    BROWN ? 3 : (MET == kSphLib ? 1 : 4)))) void k_advect2d(
    AdvectParams P)
{
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t k = blk * kBlock + threadIdx.x;
    long long steps = advect_lane_2d<ST, STEADY, MET, BROWN, kBlock>(P, k, *P.n_active);
    for (int off = 32; off > 0; off >>= 1)
        steps += __shfl_xor(steps, off, 64);
    if ((threadIdx.x & 63) == 0 && steps)
        atomicAdd(count_slot(P.psteps), (unsigned long long)steps);
}

// ---------------------------------------------------------------- 2D RKF45 with the cache
// The adaptive scheme on the stencil cache (LDS slots): each of the six Fehlberg
// stages is a stage2() evaluation (the cached bilinear polynomials, reloaded when
// the stage point leaves the cell or the lane's time bracket moves on).  The stage
// loop is not unrolled; the tableau rows come from constant memory and the earlier
// slopes sit in five named registers, so nothing is indexed dynamically.
__constant__ double kRkfC[6] = {0.0, 1.0 / 4.0, 3.0 / 8.0, 12.0 / 13.0, 1.0, 1.0 / 2.0};
__constant__ double kRkfA[6][5] = {
    {0.0, 0.0, 0.0, 0.0, 0.0},
    {1.0 / 4.0, 0.0, 0.0, 0.0, 0.0},
    {3.0 / 32.0, 9.0 / 32.0, 0.0, 0.0, 0.0},
    {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0.0, 0.0},
    {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0.0},
    {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0}};
__constant__ double kRkfB4[6] = {25.0 / 216.0, 0.0, 1408.0 / 2565.0, 2197.0 / 4104.0,
                                 -1.0 / 5.0, 0.0};
__constant__ double kRkfE[6] = {16.0 / 135.0 - 25.0 / 216.0, 0.0,
                                6656.0 / 12825.0 - 1408.0 / 2565.0,
                                28561.0 / 56430.0 - 2197.0 / 4104.0, -9.0 / 50.0 + 1.0 / 5.0,
                                2.0 / 55.0};

template <int ST, bool STEADY, int MET>
struct CachedLane2 {
    using R = typename Real<ST>::T;
    RkfState s;
    double x, y;
    Cell2<R, 16> c;
    int32_t csa, csb;
    LaneTime lt;

    __device__ void begin(const AdvectParams &P, uint32_t id)
    {
        s.id = id;
        s.st = 0;
        s.t = P.t_start;
        s.e = P.hexp[id];
        s.it = 0;
        x = P.x[id];
        y = P.y[id];
        c.clear();
        c.lc = cache_slot_ptr<R, 16>();
        c.gs = cache_group_stride<R>();
        csa = csb = -1;
        lt.lo = -1;
    }

    __device__ bool attempt(const AdvectParams &P, long long &acc, long long &rej)
    {
        const uint8_t extra = P.policy == 0 ? ST_DELETED : 0;
        if (s.t == P.t_end)
            return true;
        if (s.it++ >= P.max_iter) {  // never reached: see max_iter
            s.st = (uint8_t)(ST_OOB | extra);
            return true;
        }
        const double sg = P.dt > 0.0 ? 1.0 : -1.0;
        const double h = ldexp(fabs(P.dt), s.e);
        const double rem = sg > 0.0 ? P.t_end - s.t : s.t - P.t_end;
        const bool cut = h >= rem;
        const double hs = sg * (cut ? rem : h);
        double k0x = 0.0, k0y = 0.0, k1x = 0.0, k1y = 0.0, k2x = 0.0, k2y = 0.0;
        double k3x = 0.0, k3y = 0.0, k4x = 0.0, k4y = 0.0;
        double s4x = 0.0, s4y = 0.0, sex = 0.0, sey = 0.0;
        bool ok = true;  // as in the RK4 lane: a failed stage sets the flag, the loop runs on
#pragma nounroll
        for (int q = 0; q < 6; ++q) {
            const double *a = kRkfA[q];
            const double ax = (((a[0] * k0x + a[1] * k1x) + a[2] * k2x) + a[3] * k3x) + a[4] * k4x;
            const double ay = (((a[0] * k0y + a[1] * k1y) + a[2] * k2y) + a[3] * k3y) + a[4] * k4y;
            const TimeEntry ent = bracket_lane(P, s.t + kRkfC[q] * hs, lt);
            if (ent.sa != csa || ent.sb != csb) {
                c.invalidate();
                csa = ent.sa;
                csb = ent.sb;
            }
            double kx = 0.0, ky = 0.0;
            ok = stage2<ST, STEADY, MET, 16>(P, c, ent, false, x + hs * ax, y + hs * ay, kx,
                                             ky) & ok;
            s4x = s4x + kRkfB4[q] * kx;
            s4y = s4y + kRkfB4[q] * ky;
            sex = sex + kRkfE[q] * kx;
            sey = sey + kRkfE[q] * ky;
            switch (q) {
            case 0: k0x = kx; k0y = ky; break;
            case 1: k1x = kx; k1y = ky; break;
            case 2: k2x = kx; k2y = ky; break;
            case 3: k3x = kx; k3y = ky; break;
            case 4: k4x = kx; k4y = ky; break;
            default: break;
            }
        }
        if (!ok) {
            ++acc;
            s.st = (uint8_t)(ST_OOB | extra);
            return true;
        }
        double ex = hs * sex, ey = hs * sey;
        if constexpr (MET != kFlat) {
            ex = ex * (kMetresPerDegree * cos(y * kDegToRad));
            ey = ey * kMetresPerDegree;
        }
        const double err = sqrt(ex * ex + ey * ey);
        if (!rkf_accept(P, s, err, acc, rej))
            return false;
        const double xs = x + hs * s4x, ys = y + hs * s4y;
        bool land;
        if (in_cell(c, P, xs, ys)) {
            land = c.land;
        } else {
            const uint8_t e = point_status<false>(P.g, xs, ys, 0.0);
            if (e & ST_OOB) {
                s.st = (uint8_t)(ST_OOB | extra);
                return true;
            }
            land = e != 0;
        }
        if (land) {
            s.st = (uint8_t)(ST_LAND | extra);
            return true;
        }
        x = xs;
        y = ys;
        rkf_commit(P, s, err, cut, hs);
        return s.t == P.t_end;
    }

    __device__ void finish(const AdvectParams &P)
    {
        P.x[s.id] = x;
        P.y[s.id] = y;
        P.hexp[s.id] = (int8_t)s.e;
        if (s.st)
            P.status[s.id] = s.st;
    }
};

// Persistent RKF45 launch with lane refill.  Particles need different numbers of
// attempts, so a wave that kept its 64 particles to the end would run as long as
// its slowest one.  Here a lane that is done takes the next particle instead: once
// a quarter of the wave is idle (or all of it), one lane reserves that many entries
// of the processing order with an atomic add on its XCD's queue (the order is cut
// into eight contiguous ranges, one per XCD, so neighbouring particles stay on one
// L2) and the idle lanes take them by rank.  A drained queue sends the wave on to
// the next XCD's range; the wave ends when every queue is drained and every lane is
// idle.  Each particle's arithmetic is the same as in a one-particle-per-lane launch.
template <class Lane>
__device__ inline void rkf45_refill(const AdvectParams &P)
{
    uint32_t *queues = P.queues;
    const uint32_t nact = *P.n_active;
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t home = blockIdx.x & 7u;
    uint32_t qtry = 0;
    bool busy = false;
    long long acc = 0, rej = 0;
    Lane L;
    for (;;) {
        const uint64_t idle = __ballot(!busy);
        const uint32_t nidle = (uint32_t)__popcll(idle);
        if (qtry < 8 && (nidle >= 16 || nidle == 64)) {
            const uint32_t x = (home + qtry) & 7u;
            const uint32_t lo = (uint32_t)(((uint64_t)nact * x) >> 3);
            const uint32_t hi = (uint32_t)(((uint64_t)nact * (x + 1)) >> 3);
            uint32_t t = 0;
            if (lane == 0)
                t = lo < hi ? atomicAdd(&queues[x], nidle) : 0u;
            t = __shfl(t, 0, 64);
            const uint32_t start = lo + t;
            const uint32_t avail = (lo < hi && start < hi) ? min(nidle, hi - start) : 0u;
            if (avail < nidle)
                ++qtry;
            if (!busy) {
                const uint32_t rank = (uint32_t)__popcll(idle & ((1ull << lane) - 1ull));
                if (rank < avail) {
                    L.begin(P, P.order[start + rank]);
                    busy = true;
                }
            }
        }
        if (__ballot(busy) == 0) {
            if (qtry >= 8)
                break;
            continue;
        }
        if (busy && L.attempt(P, acc, rej)) {
            L.finish(P);
            busy = false;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        acc += __shfl_xor(acc, off, 64);
        rej += __shfl_xor(rej, off, 64);
    }
    if (lane == 0) {
        if (acc)
            atomicAdd(count_slot(P.psteps), (unsigned long long)acc);
        if (rej)
            atomicAdd(count_slot(P.prej), (unsigned long long)rej);
    }
}

// 4 waves per SIMD in 2D (the kernel needs one register more than that allows)
template <int ST, bool IS3D, bool STEADY>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(IS3D ? 1 : 4))) void k_rkf45(AdvectParams P)
{
    rkf45_refill<GatherLane<ST, IS3D, STEADY>>(P);
}

template <int ST, bool STEADY, int MET>
__global__ __launch_bounds__(kBlock) void k_rkf45_2d(AdvectParams P)
{
    rkf45_refill<CachedLane2<ST, STEADY, MET>>(P);
}

// Persistent batched launch over many independent runs (each with its own grid,
// snapshots and particles).  The active particles of every run are cut into
// chunks of blockDim particles; the chunk items are split into 8 contiguous
// ranges, one per XCD, each with its own atomic counter.  A block takes items from
// the range of the XCD it runs on and, when that is exhausted, from the others;
// every block leaves once all 8 ranges are exhausted, so the grid always drains.
// Occupancy target: 4 waves per SIMD (at most 128 VGPRs) for the plain modes, where
// it costs one spill outside the step loop; 3 for the Brownian term and the library
// cosine, whose extra state would spill inside it.
template <int ST, bool STEADY, int MET, bool BROWN>
__global__ __launch_bounds__(512)
__attribute__((amdgpu_waves_per_eu(BROWN || MET == kSphLib ? 3 : 4))) void k_advect2d_batch(
    const AdvectParams *__restrict__ runs, const uint32_t *__restrict__ cstart, int nruns,
    uint32_t total, uint32_t *queues)
{
    __shared__ uint32_t item_s;
    const uint32_t home = blockIdx.x & 7u;
    uint32_t q = 0;  // queues tried so far
    for (;;) {
        if (threadIdx.x == 0) {
            uint32_t it = 0xFFFFFFFFu;
            while (q < 8) {
                const uint32_t x = (home + q) & 7u;
                const uint32_t lo = (uint32_t)(((uint64_t)total * x) >> 3);
                const uint32_t hi = (uint32_t)(((uint64_t)total * (x + 1)) >> 3);
                if (lo < hi) {
                    const uint32_t t = atomicAdd(&queues[x], 1u);
                    if (lo + t < hi) {
                        it = lo + t;
                        break;
                    }
                }
                ++q;
            }
            item_s = it;
        }
        __syncthreads();
        const uint32_t it = __builtin_amdgcn_readfirstlane(item_s);
        __syncthreads();
        if (it == 0xFFFFFFFFu)
            break;
        int lo = 0, hi = nruns - 1;  // run r: cstart[r] <= it < cstart[r + 1]
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (cstart[mid] <= it)
                lo = mid;
            else
                hi = mid - 1;
        }
        const int r = __builtin_amdgcn_readfirstlane(lo);
        const AdvectParams &P = runs[r];
        const uint32_t k = (it - cstart[r]) * blockDim.x + threadIdx.x;
        long long steps = advect_lane_2d<ST, STEADY, MET, BROWN, 0>(P, k, *P.n_active);
        for (int off = 32; off > 0; off >>= 1)
            steps += __shfl_xor(steps, off, 64);
        if ((threadIdx.x & 63) == 0 && steps)
            atomicAdd(count_slot(P.psteps), (unsigned long long)steps);
    }
}

// ---------------------------------------------------------------- 3D with a stencil cache
// Same scheme in three dimensions: the trilinear interpolant of U, V, W in the
// cached cell written as c0 + c1 xi + c2 eta + c3 zeta + c4 xi eta + c5 xi zeta +
// c6 eta zeta + c7 xi eta zeta, for the earlier snapshot and the difference.  With
// DL the 24 difference coefficients sit in the lane's LDS slot instead of registers.
template <class R, bool DL>
struct Cell3 {
    double x0, ux, y0, uy, z0, uz;
    double rx, ry, rz;
    double cl, sl;
    R a[3][8];
    R dr[DL ? 1 : 3][8];    // registers (not DL)
    R *dl;                  // LDS slot (DL): variable v at [8 v .. 8 v + 7]
    bool land;
    __device__ R &d(int v, int q) { return DL ? dl[8 * v + q] : dr[DL ? 0 : v][q]; }
    // (DL) the cell's depth index, kept in the slot's padding after the coefficients
    __device__ int &kidx() { return *reinterpret_cast<int *>(dl + 24); }
    // as for the 2D cell: an empty x range until the next reload
    __device__ void invalidate()
    {
        x0 = __builtin_inf();
        ux = -__builtin_inf();
    }
    __device__ void clear()
    {
        y0 = uy = z0 = uz = rx = ry = rz = cl = sl = 0.0;
        land = false;
        invalidate();
    }
};

template <class R>
__device__ inline void coeffs3(const R f[8], R c[8])
{
    // f index = di + 2 dj + 4 dk
    c[0] = f[0];
    c[1] = f[1] - f[0];
    c[2] = f[2] - f[0];
    c[3] = f[4] - f[0];
    c[4] = (f[3] - f[2]) - c[1];
    c[5] = (f[5] - f[4]) - c[1];
    c[6] = (f[6] - f[4]) - c[2];
    c[7] = ((f[7] - f[6]) - (f[5] - f[4])) - ((f[3] - f[2]) - c[1]);
}

template <class R>
__device__ inline R poly3(const R c[8], R xi, R eta, R zeta)
{
    const R tx = fma(zeta, c[5], fma(eta, fma(zeta, c[7], c[4]), c[1]));
    const R r = fma(eta, fma(zeta, c[6], c[2]), fma(zeta, c[3], c[0]));
    return fma(xi, tx, r);
}

// LDS slot of the 3D cache: 24 coefficients plus 16 bytes (208 B for double, 112 B
// for float), conflict-free for 16-byte reads as in 2D.  Elements of R per lane.
template <class R>
constexpr int cache3_slot() { return (24 * (int)sizeof(R) + 16) / (int)sizeof(R); }

template <class R>
__device__ inline R *cache3_slot_ptr()
{
    extern __shared__ __attribute__((aligned(16))) unsigned char cache_lds[];
    return reinterpret_cast<R *>(cache_lds) + threadIdx.x * cache3_slot<R>();
}

// Whether the 3D kernel keeps the difference coefficients in LDS.  FP64 coefficients
// (FP32 and FP64 fields): the 48 VGPRs they free lift the kernel from 2 to 3 waves per
// SIMD (LDS then allows exactly 3).  FP32 coefficients (BF16 and scaled FP16 fields):
// the 24 VGPRs they free allow 4 waves (112 B per lane, 112 KB per CU).  Not with the
// Brownian term or the library cosine, whose extra state would spill inside the stage
// loop, and not in the steady case (no differences).
template <int ST, bool STEADY, int MET, bool BROWN>
constexpr bool cache3_lds()
{
    return !BROWN && !STEADY && MET != kSphLib;
}

// The raw storage word of one 3D node and the value of variable v in it.
template <int ST> struct NodeWord3 { using T = uint2; };     // BF16, FP16
template <> struct NodeWord3<kF64> { using T = double4; };
template <> struct NodeWord3<kF32> { using T = float4; };

template <int ST>
__device__ inline typename Real<ST>::T node_var(const typename NodeWord3<ST>::T &q, int v,
                                                const float *sc)
{
    if constexpr (ST == kF64 || ST == kF32)
        return v == 0 ? q.x : (v == 1 ? q.y : q.z);
    else if constexpr (ST == kBF16)
        return v == 0 ? bf16_lo(q.x) : (v == 1 ? bf16_hi(q.x) : bf16_lo(q.y));
    else
        return (v == 0 ? f16_lo(q.x) : (v == 1 ? f16_hi(q.x) : f16_lo(q.y))) * sc[v];
}

// With CARRY the cell keeps the coefficients at the stage time tau, a + tau d, in place of
// the earlier snapshot's a (see stage3).
template <int ST, bool STEADY, bool DL, bool CARRY = false>
__device__ inline bool reload3(const AdvectParams &P, Cell3<typename Real<ST>::T, DL> &c, int sa,
                               int sb, double x, double y, double z, double tau = 0.0)
{
    using R = typename Real<ST>::T;
    const AxisDev &ax = P.g.ax, &ay = P.g.ay, &az = P.g.az;
    if (!(x >= ax.lo && x <= ax.hi && y >= ay.lo && y <= ay.hi && z >= az.lo && z <= az.hi))
        return false;
    // A point still between the cached cell's depth faces keeps its level (most cell
    // changes are horizontal), which spares the depth axis's bin-table guess and face
    // reads, the longest chain of the search on a non-uniform axis.  The level sits in
    // the LDS slot, so only the LDS-cached forms keep it.
    const bool keep_k = DL && z >= c.z0 && z < c.uz;
    int i = axis_guess(ax, x), j = axis_guess(ay, y), k = 0;
    double xh, yh, zh = 0.0;
    if (keep_k)
        k = c.kidx();
    else
        k = axis_guess(az, z);
    axis_faces(ax, i, c.x0, xh);
    axis_faces(ay, j, c.y0, yh);
    if (!keep_k)
        axis_faces(az, k, c.z0, zh);
    axis_correct(ax, x, i, c.x0, xh);
    axis_correct(ay, y, j, c.y0, yh);
    if (!keep_k) {
        axis_correct(az, z, k, c.z0, zh);
        c.uz = (k == az.n - 2) ? nextafter(az.hi, __builtin_inf()) : zh;
    }
    if constexpr (DL)
        c.kidx() = k;
    c.ux = (i == ax.n - 2) ? nextafter(ax.hi, __builtin_inf()) : xh;
    c.uy = (j == ay.n - 2) ? nextafter(ay.hi, __builtin_inf()) : yh;
    const size_t nx = (size_t)ax.n, plane = nx * (size_t)ay.n;
    const size_t n000 = (size_t)k * plane + (size_t)j * nx + (size_t)i;
    const size_t off[8] = {0, 1, nx, nx + 1, plane, plane + 1, plane + nx, plane + nx + 1};
    const char *base = static_cast<const char *>(P.f.slots);
    using W = typename NodeWord3<ST>::T;
    // Every read of the reload is issued before any of its values is used, so that the
    // reads overlap: the eight nodes' raw words of both snapshots, then the cell's widths,
    // its latitude's cosine and sine and its land flag.  The words are converted one
    // variable at a time (fewer live registers than converting every node up front).
    const W *A = reinterpret_cast<const W *>(base + (size_t)sa * P.f.slot_bytes);
    const W *B = reinterpret_cast<const W *>(base + (size_t)sb * P.f.slot_bytes);
    // FP64 words (32 bytes) of both snapshots would hold 128 registers in flight: those
    // read the second snapshot's after converting the first's
    constexpr bool kBothAtOnce = !STEADY && sizeof(W) <= 16;
    W wa[8], wb[8];
#pragma unroll
    for (int q = 0; q < 8; ++q)
        wa[q] = A[n000 + off[q]];
    if constexpr (kBothAtOnce) {
#pragma unroll
        for (int q = 0; q < 8; ++q)
            wb[q] = B[n000 + off[q]];
    }
    c.rx = ax.rw[i];
    c.ry = ay.rw[j];
    c.rz = az.rw[k];
    const double clat = *(P.g.coslat ? P.g.coslat + j : &kAbsentTable);
    const double slat = *(P.g.coslat ? P.g.sinlat + j : &kAbsentTable);
    const uint32_t land = *(P.g.landcell ? P.g.landcell + ((size_t)j * (nx - 1) + (size_t)i)
                                         : reinterpret_cast<const uint8_t *>(&kAbsentTable));
    {
        const float *sc = ST == kF16S ? P.f.scales + ((size_t)sa * P.f.nzl + k) * 3 : nullptr;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            R f[8];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                f[q] = node_var<ST>(wa[q], v, sc + (q >> 2) * 3);
            coeffs3<R>(f, c.a[v]);
        }
    }
    if constexpr (!STEADY) {
        if constexpr (!kBothAtOnce) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                wb[q] = B[n000 + off[q]];
        }
        const float *sc = ST == kF16S ? P.f.scales + ((size_t)sb * P.f.nzl + k) * 3 : nullptr;
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            R f[8], cb[8];
#pragma unroll
            for (int q = 0; q < 8; ++q)
                f[q] = node_var<ST>(wb[q], v, sc + (q >> 2) * 3);
            coeffs3<R>(f, cb);
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const R dq = cb[q] - c.a[v][q];
                c.d(v, q) = dq;
                if constexpr (CARRY)
                    c.a[v][q] = fma((R)tau, dq, c.a[v][q]);
            }
        }
    }
    c.cl = kMetresPerDegree * clat;
    c.sl = kMetresPerDegree * slat;
    c.land = land != 0;
    return true;
}

template <class R, bool DL>
__device__ inline bool in_cell3(const Cell3<R, DL> &c, const AdvectParams &P, double x, double y,
                                double z)
{
    return x >= c.x0 && x < c.ux && y >= c.y0 && y < c.uy && z >= c.z0 && z < c.uz;
}

// With FP64 coefficients the cell carries the coefficients at the last stage's time,
// c = a + tau d, and a stage at time tau' first advances them by (tau' - tau) d, then
// evaluates one trilinear polynomial instead of two (the polynomial is linear in its
// coefficients, so the value is the same up to rounding).  Every lane of a launch shares
// the stage times, so tau_prev, the previous stage's time, is one value for the wave; a
// lane that reloads here gets its coefficients at tau' from the reload and skips the
// advance, and stages at the previous stage's time (the first and third of RK4; the
// last stage of a step and the first of the next share a time) skip it for the whole
// wave: per step two advances of 24 products instead of four second polynomials.
template <int ST, bool STEADY, int MET, bool DL>
__device__ inline bool stage3(const AdvectParams &P, Cell3<typename Real<ST>::T, DL> &c,
                              const TimeEntry &e, bool fresh, double x, double y, double z,
                              double k[3], double tau_prev)
{
    using R = typename Real<ST>::T;
    constexpr bool CARRY = !STEADY && sizeof(R) == 8;
    const bool re = !in_cell3(c, P, x, y, z) | fresh;
    if (re) {
        if (!reload3<ST, STEADY, DL, CARRY>(P, c, e.sa, e.sb, x, y, z, e.tau))
            return false;
    }
    const R xi = (R)((x - c.x0) * c.rx), eta = (R)((y - c.y0) * c.ry);
    const R zeta = (R)((z - c.z0) * c.rz);
    R v[3];
    if constexpr (CARRY) {
        const double dtau = e.tau - tau_prev;
        if (dtau != 0.0) {
            const R dl = re ? (R)0 : (R)dtau;
#pragma unroll
            for (int q = 0; q < 3; ++q)
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    c.a[q][i] = fma(dl, c.d(q, i), c.a[q][i]);
        }
#pragma unroll
        for (int q = 0; q < 3; ++q)
            v[q] = poly3<R>(c.a[q], xi, eta, zeta);
    } else {
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            v[q] = poly3<R>(c.a[q], xi, eta, zeta);
            if constexpr (!STEADY) {
                R dq[8];
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    dq[i] = c.d(q, i);
                v[q] = fma((R)e.tau, poly3<R>(dq, xi, eta, zeta), v[q]);
            }
        }
    }
    if constexpr (MET != kFlat) {
        k[0] = (double)v[0] * stage_metric<MET>(c, P, y);
        k[1] = (double)v[1] * (1.0 / kMetresPerDegree);
    } else {
        k[0] = (double)v[0];
        k[1] = (double)v[1];
    }
    k[2] = (double)v[2];
    return true;
}

// With BEHAVE the worked example's kernels (sinking, age, tracer sample; Sect. 3.3) run
// ahead of each step as in the gather kernel, with the same code, and the advection
// keeps the depth of a dwelling particle.  Occupancy targets: 3 waves per SIMD with
// FP64 coefficients in LDS, 4 with FP32 ones, else 2 (Brownian) or 1.
template <int ST, bool STEADY, int MET, bool BROWN, bool BEHAVE>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu(cache3_lds<ST, STEADY, MET, BROWN>() ? (sizeof(typename Real<ST>::T) == 8 ? 3 : 4) : (BROWN ? 2 : 1)))) void k_advect3d(
    AdvectParams P)
{
    using R = typename Real<ST>::T;
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t kk = blk * kBlock + threadIdx.x;
    const uint32_t nact = *P.n_active;
    long long steps = 0;
    if (kk < nact) {
        const uint32_t id = P.order[kk];
        uint8_t st = P.status[id];
        if (st == 0) {
            double x = P.x[id], y = P.y[id], z = P.z[id];
            double temp = 0.0, age = 0.0;
            if constexpr (BEHAVE) {
                temp = P.temp[id];
                age = P.age[id];
            }
            constexpr bool DL = cache3_lds<ST, STEADY, MET, BROWN>();
            Cell3<R, DL> c;
            c.clear();
            if constexpr (DL)
                c.dl = cache3_slot_ptr<R>();
            const double dt = P.dt, dt6 = P.dt6;
            double tau_prev = P.tab[0].tau;  // the time of the cell's coefficients (stage3)
            for (int s = 0; s < P.nsteps; ++s) {
                ++steps;
                const TimeEntry e0 = P.tab[2 * s], e1 = P.tab[2 * s + 1], e2 = P.tab[2 * s + 2];
                const BracketMoves moves(P, s, e0, e1, e2);
                uint8_t err = ST_OOB;
                bool horizontal = false;
                if constexpr (BEHAVE) {
                    const uint8_t b =
                        behave_pre<true, STEADY>(P, s, x, y, z, temp, age, horizontal);
                    if (b) {
                        st = b;
                        break;
                    }
                }
                double k[3] = {0.0, 0.0, 0.0}, sm[3] = {0.0, 0.0, 0.0};
                const int nst = P.scheme ? 1 : 4;
                bool ok = true;  // as in 2D: a failed stage leaves its slope, the step fails
                // The four stages side by side: with FP32 coefficients (+11% on the BF16
                // and FP16 forms), and with FP64 ones for FP32 fields in the 2-term and flat
                // metric modes without the behaviour or Brownian terms (+8.7% on cfg2, no
                // spill in the loop). The other FP64 forms spill more unrolled (the
                // behaviour kernels lost 1.9%, the 3/4-term series spills 92 B), so they
                // keep the rolled loop.
                constexpr bool kUnrollF64 = ST == kF32 && !BEHAVE && !BROWN &&
                                            (MET == kSphTable2 || MET == kFlat);
                constexpr int kUnroll = sizeof(R) == 4 || kUnrollF64 ? 4 : 1;
#pragma unroll kUnroll
                for (int q = 0; q < nst; ++q) {
                    const TimeEntry e = q == 0 ? e0 : (q == 3 ? e2 : e1);
                    // (stage 1 adds a zero slope, so its offset is immaterial; the
                    // half step comes in with the launch, as a scalar operand)
                    const double h = q == 3 ? dt : P.hdt;
                    ok = stage3<ST, STEADY, MET, DL>(P, c, e, moves.at(q), x + k[0] * h,
                                                     y + k[1] * h, z + k[2] * h, k, tau_prev) &
                         ok;
                    tau_prev = e.tau;
                    const double wq = q == 0 ? 1.0 : (q == 3 ? 0.0 : 2.0);
#pragma unroll
                    for (int v = 0; v < 3; ++v)
                        sm[v] = fma(wq, k[v], sm[v]);
                }
                if (!ok)
                    goto fail;
                {
                    double xs, ys, zs;
                    if (P.scheme) {  // Euler forward
                        xs = x + k[0] * dt;
                        ys = y + k[1] * dt;
                        zs = z + k[2] * dt;
                    } else {
                        xs = x + (sm[0] + k[0]) * dt6;
                        ys = y + (sm[1] + k[1]) * dt6;
                        zs = z + (sm[2] + k[2]) * dt6;
                    }
                    if (BEHAVE && horizontal)  // a dwelling particle keeps its depth
                        zs = z;
                    if (BROWN && P.Kh > 0.0) {
                        double dx, dy;
                        brownian_metres<MET == kFlat>(P, id, P.step0 + s, dt, dx, dy);
                        if constexpr (MET != kFlat) {
                            dx = dx * inv_metres_lon<MET>(c, P, ys);
                            dy = dy / kMetresPerDegree;
                        }
                        xs = xs + dx;
                        ys = ys + dy;
                    }
                    bool land;
                    if (in_cell3(c, P, xs, ys, zs)) {
                        land = c.land;
                    } else {
                        const uint8_t e = point_status<true>(P.g, xs, ys, zs);
                        if (e & ST_OOB)
                            goto fail;
                        land = e != 0;
                    }
                    if (land) {
                        err = ST_LAND;
                        goto fail;
                    }
                    x = xs;
                    y = ys;
                    z = zs;
                }
                continue;
            fail:
                st = (uint8_t)(err | (P.policy == 0 ? ST_DELETED : 0));
                break;
            }
            // the stores index with an offset the compiler cannot fold (zero), so that it
            // recomputes their addresses here instead of keeping the loads' 64-bit addresses
            // live across the step loop (which spilled one of them)
            const uint32_t sid = id + P.zero;
            P.x[sid] = x;
            P.y[sid] = y;
            P.z[sid] = z;
            if constexpr (BEHAVE) {
                P.temp[sid] = temp;
                P.age[sid] = age;
            }
            if (st)
                P.status[sid] = st;
        }
    }
    for (int off = 32; off > 0; off >>= 1)
        steps += __shfl_xor(steps, off, 64);
    if ((threadIdx.x & 63) == 0 && steps)
        atomicAdd(count_slot(P.psteps), (unsigned long long)steps);
}

__global__ void k_philox_normals(uint32_t run_id, uint32_t seed, int64_t n, const uint32_t *pid,
                                 const uint32_t *step, uint32_t *words, double *normals)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n)
        return;
    uint32_t w[4] = {pid[i], step[i], 0u, 0u};
    philox4x32_10(w, run_id, seed);
    if (words) {
        words[4 * i] = w[0];
        words[4 * i + 1] = w[1];
        words[4 * i + 2] = w[2];
        words[4 * i + 3] = w[3];
    }
    if (normals) {
        box_muller(unit53(w[0], w[1]), unit53(w[2], w[3]), normals[2 * i], normals[2 * i + 1]);
    }
}

template <int ST, bool IS3D>
__global__ void k_slot_values(const char *slot, const float *scales, size_t plane, int nzl,
                              float *U, float *V, float *W)
{
    using R = typename Real<ST>::T;
    const size_t total = plane * (size_t)nzl;
    for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < total;
         i += (size_t)gridDim.x * blockDim.x) {
        const float *sc = ST == kF16S ? scales + (i / plane) * 3 : nullptr;
        R v[3];
        load_node<ST, IS3D>(slot, i, sc, v);
        U[i] = (float)v[0];
        V[i] = (float)v[1];
        if (W)
            W[i] = (float)v[2];
    }
}

__global__ void k_lat_tables(const double *lat, int ny, double *cl, double *sl)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < ny) {
        double s, c;
        sincos(lat[j] * kDegToRad, &s, &c);
        cl[j] = c;
        sl[j] = s;
    }
}

// Output record (or cell-index query) of the particles with id = r * stride.
__global__ void k_record(RecordParams R)
{
    for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < R.nper;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t id = r * R.stride;
        const double x = R.x[id], y = R.y[id];
        const double z = R.z ? R.z[id] : 0.0;
        int i = -1, j = -1, k = R.g.az.n ? -1 : 0;
        double f;
        bool in = locate(R.g.ax, x, i, f) && locate(R.g.ay, y, j, f);
        if (in && R.g.az.n)
            in = locate(R.g.az, z, k, f);
        if (!in) {
            i = -1;
            j = -1;
            k = -1;
        }
        if (R.rx) R.rx[r] = x;
        if (R.ry) R.ry[r] = y;
        if (R.rz) R.rz[r] = z;
        if (R.rst) R.rst[r] = R.status[id];
        if (R.ci) R.ci[r] = i;
        if (R.cj) R.cj[r] = j;
        if (R.ck) R.ck[r] = k;
        if (R.rtemp) R.rtemp[r] = R.temp[id];
        if (R.rage) R.rage[r] = R.age[id];
    }
}

template <bool B> using BoolC = std::integral_constant<bool, B>;
template <int I> using IntC = std::integral_constant<int, I>;

// Calls f(steady, metric mode, Brownian) with compile-time constants chosen from the
// launch: the cached kernels are instantiated per combination.
template <class F>
hipError_t dispatch_cached(const AdvectParams &p, bool steady, F &&f)
{
    const int met = !p.g.spherical
                        ? kFlat
                        : (p.g.coslat ? (p.g.cos_terms == 2 ? kSphTable2 : kSphTable) : kSphLib);
    const bool brown = p.Kh > 0.0;
    auto with_met = [&](auto stc) {
        auto with_brown = [&](auto m) {
            if (brown)
                f(stc, m, BoolC<true>{});
            else
                f(stc, m, BoolC<false>{});
        };
        if (met == kFlat)
            with_brown(IntC<kFlat>{});
        else if (met == kSphTable2)
            with_brown(IntC<kSphTable2>{});
        else if (met == kSphTable)
            with_brown(IntC<kSphTable>{});
        else
            with_brown(IntC<kSphLib>{});
    };
    if (steady)
        with_met(BoolC<true>{});
    else
        with_met(BoolC<false>{});
    return hipGetLastError();
}

template <int ST, bool IS3D>
hipError_t launch3(const AdvectParams &p, bool steady, uint32_t n_launch, hipStream_t s)
{
    const uint32_t blocks = (n_launch + kBlock - 1) / kBlock;
    if (blocks == 0)
        return hipSuccess;
    // the cached kernels interpolate linearly; the worked-example kernels run in the 3D
    // cached kernel for FP32 / FP64 fields without a Brownian term, else in the gather
    constexpr bool kBehaveCached = IS3D && (ST == kF32 || ST == kF64);
    if (!p.cache || p.nearest || (p.behave && (!kBehaveCached || p.Kh > 0.0))) {
        const bool brown = p.Kh > 0.0;
        if (steady && brown)
            hipLaunchKernelGGL((k_advect<ST, IS3D, true, true>), dim3(blocks), dim3(kBlock), 0,
                               s, p);
        else if (steady)
            hipLaunchKernelGGL((k_advect<ST, IS3D, true, false>), dim3(blocks), dim3(kBlock), 0,
                               s, p);
        else if (brown)
            hipLaunchKernelGGL((k_advect<ST, IS3D, false, true>), dim3(blocks), dim3(kBlock), 0,
                               s, p);
        else
            hipLaunchKernelGGL((k_advect<ST, IS3D, false, false>), dim3(blocks), dim3(kBlock),
                               0, s, p);
        return hipGetLastError();
    }
    const dim3 g(blocks), b(kBlock);
    if constexpr (!IS3D) {
        using R = typename Real<ST>::T;
        return dispatch_cached(p, steady, [&](auto stc, auto met, auto brown) {
            const size_t lds =
                (size_t)kBlock *
                cache_slot<R, cache_lds_coefs<ST, decltype(brown)::value>()>() * sizeof(R);
            hipLaunchKernelGGL((k_advect2d<ST, decltype(stc)::value, decltype(met)::value,
                                           decltype(brown)::value>),
                               g, b, lds, s, p);
        });
    } else {
        using R = typename Real<ST>::T;
        return dispatch_cached(p, steady, [&](auto stc, auto met, auto brown) {
            constexpr bool dl = cache3_lds<ST, decltype(stc)::value, decltype(met)::value,
                                           decltype(brown)::value>();
            const size_t lds = dl ? (size_t)kBlock * cache3_slot<R>() * sizeof(R) : 0;
            if constexpr (kBehaveCached && !decltype(brown)::value) {
                if (p.behave) {
                    hipLaunchKernelGGL((k_advect3d<ST, decltype(stc)::value, decltype(met)::value,
                                                   false, true>),
                                       g, b, lds, s, p);
                    return;
                }
            }
            hipLaunchKernelGGL((k_advect3d<ST, decltype(stc)::value, decltype(met)::value,
                                           decltype(brown)::value, false>),
                               g, b, lds, s, p);
        });
    }
}

}  // namespace

hipError_t launch_advect(int store, bool is3d, const AdvectParams &p, uint32_t n_launch,
                         hipStream_t s)
{
    const bool steady = p.f.steady != 0;
    switch (store) {
    case kF64: return is3d ? launch3<kF64, true>(p, steady, n_launch, s)
                           : launch3<kF64, false>(p, steady, n_launch, s);
    case kF32: return is3d ? launch3<kF32, true>(p, steady, n_launch, s)
                           : launch3<kF32, false>(p, steady, n_launch, s);
    case kBF16: return is3d ? launch3<kBF16, true>(p, steady, n_launch, s)
                            : launch3<kBF16, false>(p, steady, n_launch, s);
    case kF16S: return is3d ? launch3<kF16S, true>(p, steady, n_launch, s)
                            : launch3<kF16S, false>(p, steady, n_launch, s);
    }
    return hipErrorInvalidValue;
}

namespace {

// Persistent grid: as many blocks as fit on the device at once (no more than the
// particles need); the eight queues are cleared on the stream first.
template <class K>
hipError_t launch_persistent(K kern, const AdvectParams &p, uint32_t n_launch, hipStream_t s,
                             size_t lds = 0)
{
    int per_cu = 0, cus = 0, dev = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, kBlock, lds);
    if (e != hipSuccess)
        return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    uint32_t grid = (uint32_t)(per_cu > 0 ? per_cu : 1) * (uint32_t)(cus > 0 ? cus : 1);
    const uint32_t need = (n_launch + kBlock - 1) / kBlock;
    grid = grid < need ? grid : need;
    if ((e = launch_fill_u32(p.queues, 0u, 8, s)) != hipSuccess)
        return e;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(kBlock), lds, s, p);
    return hipGetLastError();
}

template <int ST, bool IS3D>
hipError_t rkf3(const AdvectParams &p, bool steady, uint32_t n_launch, hipStream_t s)
{
    if (n_launch == 0)
        return hipSuccess;
    if constexpr (!IS3D) {
        if (p.cache && !p.nearest) {
            using R = typename Real<ST>::T;
            const size_t lds = (size_t)kBlock * cache_slot<R, 16>() * sizeof(R);
            hipError_t e = hipSuccess;
            (void)dispatch_cached(p, steady, [&](auto stc, auto met, auto) {
                e = launch_persistent(k_rkf45_2d<ST, decltype(stc)::value, decltype(met)::value>,
                                      p, n_launch, s, lds);
            });
            return e;
        }
    }
    return steady ? launch_persistent(k_rkf45<ST, IS3D, true>, p, n_launch, s)
                  : launch_persistent(k_rkf45<ST, IS3D, false>, p, n_launch, s);
}

}  // namespace

hipError_t launch_rkf45(int store, bool is3d, const AdvectParams &p, uint32_t n_launch,
                        hipStream_t s)
{
    const bool steady = p.f.steady != 0;
    if (!p.res || p.nres < 1 || (!steady && p.period <= 0.0 && p.nres < 2) || !p.hexp ||
        !p.prej || !p.queues)
        return hipErrorInvalidValue;
    switch (store) {
    case kF64: return is3d ? rkf3<kF64, true>(p, steady, n_launch, s)
                           : rkf3<kF64, false>(p, steady, n_launch, s);
    case kF32: return is3d ? rkf3<kF32, true>(p, steady, n_launch, s)
                           : rkf3<kF32, false>(p, steady, n_launch, s);
    case kBF16: return is3d ? rkf3<kBF16, true>(p, steady, n_launch, s)
                            : rkf3<kBF16, false>(p, steady, n_launch, s);
    case kF16S: return is3d ? rkf3<kF16S, true>(p, steady, n_launch, s)
                            : rkf3<kF16S, false>(p, steady, n_launch, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_philox_normals(uint32_t run_id, uint32_t seed, int64_t n, const uint32_t *pid,
                                 const uint32_t *step, uint32_t *words, double *normals,
                                 hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_philox_normals, dim3((uint32_t)((n + 255) / 256)), dim3(256), 0, s,
                       run_id, seed, n, pid, step, words, normals);
    return hipGetLastError();
}

hipError_t launch_slot_values(int store, bool is3d, const void *slot, const float *scales,
                              size_t plane, int nzl, float *U, float *V, float *W, hipStream_t s)
{
    const size_t total = plane * (size_t)nzl;
    size_t nb = (total + 255) / 256;
    const dim3 g((uint32_t)(nb > 32768 ? 32768 : nb)), b(256);
    const char *sl = static_cast<const char *>(slot);
#define LP_SV(ST, D3) hipLaunchKernelGGL((k_slot_values<ST, D3>), g, b, 0, s, sl, scales, plane, nzl, U, V, W)
    switch (store) {
    case kF64: if (is3d) LP_SV(kF64, true); else LP_SV(kF64, false); break;
    case kF32: if (is3d) LP_SV(kF32, true); else LP_SV(kF32, false); break;
    case kBF16: if (is3d) LP_SV(kBF16, true); else LP_SV(kBF16, false); break;
    case kF16S: if (is3d) LP_SV(kF16S, true); else LP_SV(kF16S, false); break;
    default: return hipErrorInvalidValue;
    }
#undef LP_SV
    return hipGetLastError();
}

hipError_t launch_lat_tables(const double *lat, int ny, double *coslat, double *sinlat,
                              hipStream_t s)
{
    hipLaunchKernelGGL(k_lat_tables, dim3((ny + 255) / 256), dim3(256), 0, s, lat, ny, coslat,
                       sinlat);
    return hipGetLastError();
}

template <int ST, bool STEADY, int MET, bool BROWN>
hipError_t batch3(const AdvectParams *runs, const uint32_t *cstart, int nruns, uint32_t total,
                  uint32_t *queues, int block, hipStream_t s, int *grid_out)
{
    auto kern = k_advect2d_batch<ST, STEADY, MET, BROWN>;
    using R = typename Real<ST>::T;
    const size_t lds =
        (size_t)block * cache_slot<R, cache_lds_coefs<ST, BROWN>()>() * sizeof(R);
    int per_cu = 0, cus = 0, dev = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, lds);
    if (e != hipSuccess)
        return e;
    if ((e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
        return e;
    int grid = per_cu * cus;
    if (grid < 1)
        grid = 1;
    if ((uint32_t)grid > total)
        grid = (int)(total ? total : 1);
    if (grid_out)
        *grid_out = grid;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), lds, s, runs, cstart, nruns, total, queues);
    return hipGetLastError();
}

hipError_t launch_advect_batch(int store, bool steady, int met, bool brown,
                               const AdvectParams *runs, const uint32_t *cstart, int nruns,
                               uint32_t total, uint32_t *queues, int block, hipStream_t s,
                               int *grid_out)
{
    hipError_t e = launch_fill_u32(queues, 0u, 8, s);
    if (e != hipSuccess || total == 0)
        return e;
    auto go = [&](auto st) -> hipError_t {
        constexpr int ST = decltype(st)::value;
        AdvectParams q{};  // only the mode fields matter to the dispatcher
        q.g.spherical = met != kFlat;
        q.g.coslat = (met == kSphTable || met == kSphTable2)
                         ? reinterpret_cast<const double *>(1)
                         : nullptr;
        q.g.cos_terms = met == kSphTable2 ? 2 : 3;
        q.Kh = brown ? 1.0 : 0.0;
        hipError_t r = hipSuccess;
        (void)dispatch_cached(q, steady, [&](auto stc, auto m, auto b) {
            r = batch3<ST, decltype(stc)::value, decltype(m)::value, decltype(b)::value>(
                runs, cstart, nruns, total, queues, block, s, grid_out);
        });
        return r;
    };
    switch (store) {
    case kF64: return go(IntC<kF64>{});
    case kF32: return go(IntC<kF32>{});
    case kBF16: return go(IntC<kBF16>{});
    case kF16S: return go(IntC<kF16S>{});
    }
    return hipErrorInvalidValue;
}

hipError_t launch_record(const RecordParams &p, hipStream_t s)
{
    if (p.nper <= 0)
        return hipSuccess;
    int64_t blocks = (p.nper + 255) / 256;
    if (blocks > 65536)
        blocks = 65536;
    hipLaunchKernelGGL(k_record, dim3((uint32_t)blocks), dim3(256), 0, s, p);
    return hipGetLastError();
}

}  // namespace lp
