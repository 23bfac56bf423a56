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
#include "lp_internal.h"

namespace lp {

namespace {

constexpr uint8_t ST_OOB = 1, ST_LAND = 2, ST_DELETED = 4;

// Blocks are dispatched round-robin over the 8 XCDs (block b -> XCD b % 8).  Map
// the hardware block id so that each XCD works on one contiguous range of the
// (tile-sorted) particle order and keeps that region's stencils in its own L2.
__device__ inline uint32_t xcd_block(uint32_t b, uint32_t nb)
{
    const uint32_t q = nb >> 3, r = nb & 7u;
    const uint32_t x = b & 7u, local = b >> 3;
    return x * q + (x < r ? x : r) + local;
}

// Cell search on one axis: the largest i in [0, n-2] with c[i] <= x, or false if x
// is NaN or outside [c0, c(n-1)].  The guess (closed form for a uniform axis, a
// bin table otherwise) is corrected against the stored coordinates, so the index
// follows the stored grid exactly.
__device__ inline bool locate(const AxisDev &a, double x, int &i, double &f)
{
    if (!(x >= a.lo && x <= a.hi))
        return false;
    int g;
    if (a.uniform) {
        g = (int)((x - a.lo) * a.ginv);
    } else {
        int b = (int)((x - a.lo) * a.ginv);
        b = b < kGuessBins - 1 ? b : kGuessBins - 1;
        g = a.guess[b];
    }
    g = g < 0 ? 0 : (g > a.n - 2 ? a.n - 2 : g);
    while (g > 0 && a.c[g] > x)
        --g;
    while (g < a.n - 2 && a.c[g + 1] <= x)
        ++g;
    i = g;
    f = (x - a.c[g]) * a.rw[g];
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

// Velocity at a stage point in coordinate units per second; false if outside.
template <int ST, bool IS3D, bool STEADY>
__device__ inline bool sample(const AdvectParams &P, const TimeEntry &te, double x, double y,
                              double z, double k[3])
{
    using R = typename Real<ST>::T;
    Cell c;
    if (!locate(P.g.ax, x, c.i, c.xi) || !locate(P.g.ay, y, c.j, c.eta))
        return false;
    c.k = 0;
    c.zeta = 0.0;
    if constexpr (IS3D) {
        if (!locate(P.g.az, z, c.k, c.zeta))
            return false;
    }
    if (P.nearest) {
        c.xi = c.xi < 0.5 ? 0.0 : 1.0;
        c.eta = c.eta < 0.5 ? 0.0 : 1.0;
        c.zeta = c.zeta < 0.5 ? 0.0 : 1.0;
    }
    R v[3];
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
        const uint32_t lo0 = M0 * c[0], hi0 = __umulhi(M0, c[0]);
        const uint32_t lo1 = M1 * c[2], hi1 = __umulhi(M1, c[2]);
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

template <int ST, bool IS3D, bool STEADY>
__device__ inline uint8_t rk4_step(const AdvectParams &P, int s, uint32_t id, double &x,
                                   double &y, double &z)
{
    const TimeEntry e0 = P.tab[2 * s], e1 = P.tab[2 * s + 1], e2 = P.tab[2 * s + 2];
    const double dt = P.dt, hd = 0.5 * dt;
    double k1[3], k2[3], k3[3], k4[3];
    if (!sample<ST, IS3D, STEADY>(P, e0, x, y, z, k1))
        return ST_OOB;
    double xs, ys, zs = z;
    if (P.scheme) {  // Euler forward
        xs = x + k1[0] * dt;
        ys = y + k1[1] * dt;
        if constexpr (IS3D)
            zs = z + k1[2] * dt;
    } else {
        if (!sample<ST, IS3D, STEADY>(P, e1, x + k1[0] * hd, y + k1[1] * hd, z + k1[2] * hd,
                                      k2))
            return ST_OOB;
        if (!sample<ST, IS3D, STEADY>(P, e1, x + k2[0] * hd, y + k2[1] * hd, z + k2[2] * hd,
                                      k3))
            return ST_OOB;
        if (!sample<ST, IS3D, STEADY>(P, e2, x + k3[0] * dt, y + k3[1] * dt, z + k3[2] * dt,
                                      k4))
            return ST_OOB;
        xs = x + ((((k1[0] + 2.0 * k2[0]) + 2.0 * k3[0]) + k4[0]) * dt) / 6.0;
        ys = y + ((((k1[1] + 2.0 * k2[1]) + 2.0 * k3[1]) + k4[1]) * dt) / 6.0;
        if constexpr (IS3D)
            zs = z + ((((k1[2] + 2.0 * k2[2]) + 2.0 * k3[2]) + k4[2]) * dt) / 6.0;
    }
    if (P.Kh > 0.0) {
        uint32_t c[4] = {id, (uint32_t)(P.step0 + s), 0u, 0u};
        philox4x32_10(c, P.run_id, P.seed);
        const double u1 = unit53(c[0], c[1]), u2 = unit53(c[2], c[3]);
        const double r = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincos((2.0 * 3.141592653589793) * u2, &sn, &cs);
        const double sig = sqrt(2.0 * P.Kh * dt);
        double dx = sig * (r * cs), dy = sig * (r * sn);
        if (P.g.spherical) {
            dx = dx / (kMetresPerDegree * cos(ys * kDegToRad));
            dy = dy / kMetresPerDegree;
        }
        xs = xs + dx;
        ys = ys + dy;
    }
    int ci, cj, ck;
    double f;
    if (!locate(P.g.ax, xs, ci, f) || !locate(P.g.ay, ys, cj, f))
        return ST_OOB;
    if constexpr (IS3D) {
        if (!locate(P.g.az, zs, ck, f))
            return ST_OOB;
    }
    if (P.g.landcell && P.g.landcell[(size_t)cj * (size_t)(P.g.ax.n - 1) + (size_t)ci])
        return ST_LAND;
    x = xs;
    y = ys;
    z = zs;
    return 0;
}

template <int ST, bool IS3D, bool STEADY>
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
            for (int s = 0; s < P.nsteps; ++s) {
                ++steps;
                const uint8_t e = rk4_step<ST, IS3D, STEADY>(P, s, id, x, y, z);
                if (e) {
                    st = (uint8_t)(e | (P.policy == 0 ? ST_DELETED : 0));
                    break;
                }
            }
            P.x[id] = x;
            P.y[id] = y;
            if constexpr (IS3D)
                P.z[id] = z;
            if (st)
                P.status[id] = st;
        }
    }
    for (int off = 32; off > 0; off >>= 1)
        steps += __shfl_xor(steps, off, 64);
    if ((threadIdx.x & 63) == 0 && steps)
        atomicAdd(P.psteps, (unsigned long long)steps);
}

// ---------------------------------------------------------------- adaptive RKF45
// The Runge-Kutta-Fehlberg option of Sect. 2.1.1 with a per-particle step |dt| 2^e.
// Each lane runs its own sequence of attempts from t_start to t_end, so its stage
// times are its own: the bracketing snapshots of each stage time are found per
// lane in the resident-snapshot table, with the same arithmetic as the host's
// stage-time table (periodic fields first map t into [T0, T0 + period)).
__device__ inline TimeEntry bracket_lane(const AdvectParams &P, double t)
{
    const ResTime *r = P.res;
    const int m = P.nres;
    TimeEntry e;
    if (P.f.steady) {
        e.tau = 0.0;
        e.sa = e.sb = r[0].slot;
        return e;
    }
    if (P.period > 0.0) {
        const double T0 = r[0].t;
        double q = fmod(t - T0, P.period);
        if (q < 0.0)
            q += P.period;
        const double tp = T0 + q;
        int lo = 0, hi = m - 1;  // largest k with r[k].t <= tp (r[0].t <= tp)
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (r[mid].t <= tp)
                lo = mid;
            else
                hi = mid - 1;
        }
        const double tn = lo + 1 < m ? r[lo + 1].t : T0 + P.period;
        e.sa = r[lo].slot;
        e.sb = lo + 1 < m ? r[lo + 1].slot : r[0].slot;
        e.tau = (tp - r[lo].t) / (tn - r[lo].t);
        return e;
    }
    int lo = 0, hi = m - 2;  // largest k <= m-2 with r[k].t <= t (the host checked
    while (lo < hi) {        // that [t_start, t_end] lies inside the table)
        const int mid = (lo + hi + 1) >> 1;
        if (r[mid].t <= t)
            lo = mid;
        else
            hi = mid - 1;
    }
    e.sa = r[lo].slot;
    e.sb = r[lo + 1].slot;
    e.tau = (t - r[lo].t) / (r[lo + 1].t - r[lo].t);
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
                                     const double p[3], double p4[3], double ev[3])
{
    double k[6][3];
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
        const TimeEntry te = bracket_lane(P, t + Fehlberg::c[i] * h);
        if (!sample<ST, IS3D, STEADY>(P, te, q[0], q[1], q[2], k[i]))
            return false;
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
    return true;
}

template <int ST, bool IS3D, bool STEADY>
__global__ __launch_bounds__(kBlock) void k_rkf45(AdvectParams P)
{
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t k = blk * kBlock + threadIdx.x;
    const uint32_t nact = *P.n_active;
    long long acc = 0, rej = 0;
    if (k < nact) {
        const uint32_t id = P.order[k];
        uint8_t st = P.status[id];
        if (st == 0) {
            const uint8_t extra = P.policy == 0 ? ST_DELETED : 0;
            double p[3] = {P.x[id], P.y[id], IS3D ? P.z[id] : 0.0};
            int e = P.hexp[id];
            const double sg = P.dt > 0.0 ? 1.0 : -1.0, adt = fabs(P.dt);
            const double te = P.t_end;
            double t = P.t_start;
            // every attempt either lowers e (at most e - emin times in a row) or moves
            // t by at least the floor step, so max_iter is never reached
            for (int it = 0; t != te; ++it) {
                if (it >= P.max_iter) {
                    st = (uint8_t)(ST_OOB | extra);
                    break;
                }
                const double h = ldexp(adt, e);
                const double rem = sg > 0.0 ? te - t : t - te;
                const bool cut = h >= rem;
                const double hs = sg * (cut ? rem : h);
                double p4[3], ev[3];
                if (!rkf45_attempt<ST, IS3D, STEADY>(P, t, hs, p, p4, ev)) {
                    ++acc;
                    st = (uint8_t)(ST_OOB | extra);
                    break;
                }
                double ex = ev[0], ey = ev[1];
                if (P.g.spherical) {
                    ex = ex * (kMetresPerDegree * cos(p[1] * kDegToRad));
                    ey = ey * kMetresPerDegree;
                }
                const double err = sqrt((ex * ex + ey * ey) + ev[2] * ev[2]);
                if (err > P.tol && e > P.emin) {
                    --e;
                    ++rej;
                    continue;
                }
                ++acc;
                int ci, cj, ck;
                double f;
                if (!locate(P.g.ax, p4[0], ci, f) || !locate(P.g.ay, p4[1], cj, f)) {
                    st = (uint8_t)(ST_OOB | extra);
                    break;
                }
                if constexpr (IS3D) {
                    if (!locate(P.g.az, p4[2], ck, f)) {
                        st = (uint8_t)(ST_OOB | extra);
                        break;
                    }
                }
                if (P.g.landcell &&
                    P.g.landcell[(size_t)cj * (size_t)(P.g.ax.n - 1) + (size_t)ci]) {
                    st = (uint8_t)(ST_LAND | extra);
                    break;
                }
                p[0] = p4[0];
                p[1] = p4[1];
                p[2] = p4[2];
                t = cut ? te : t + hs;
                if (!cut && err <= P.tol * 0.03125 && e < P.emax)
                    ++e;
            }
            P.x[id] = p[0];
            P.y[id] = p[1];
            if constexpr (IS3D)
                P.z[id] = p[2];
            P.hexp[id] = (int8_t)e;
            if (st)
                P.status[id] = st;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        acc += __shfl_xor(acc, off, 64);
        rej += __shfl_xor(rej, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        if (acc)
            atomicAdd(P.psteps, (unsigned long long)acc);
        if (rej)
            atomicAdd(P.prej, (unsigned long long)rej);
    }
}

// ---------------------------------------------------------------- 2D with a stencil cache
// Each lane keeps the stencil of the cell it is in, as the coefficients of the
// bilinear polynomial f = c0 + c1 xi + c2 eta + c3 xi eta of U and V for the
// earlier snapshot and for the difference (later - earlier).  A stage point in the
// cached cell then costs only arithmetic: the stencil is reloaded when the point
// leaves the cell or when the time bracket moves on.  The polynomial is the same
// bilinear interpolant as the corner-weight form (Sect. 2.3), and f_a + tau (f_b -
// f_a) is the same linear time interpolation (Sect. 2.4); only rounding differs.
template <class R>
struct Cell2 {
    double x0, ux, y0, uy;  // lower faces; exclusive upper faces (+inf for the last cell)
    double rx, ry;          // inverse cell widths
    double cl, sl;          // cos and sin of the lower latitude face
    R a[2][4];              // earlier snapshot: U, V coefficients
    R d[2][4];              // later minus earlier
    bool land;
    bool valid;
};

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

template <int ST, bool STEADY>
__device__ inline bool reload2(const AdvectParams &P, Cell2<typename Real<ST>::T> &c, int sa,
                               int sb, double x, double y)
{
    using R = typename Real<ST>::T;
    int i, j;
    double f;
    if (!locate(P.g.ax, x, i, f) || !locate(P.g.ay, y, j, f))
        return false;
    const AxisDev &ax = P.g.ax, &ay = P.g.ay;
    c.x0 = ax.c[i];
    c.ux = (i == ax.n - 2) ? __builtin_inf() : ax.c[i + 1];
    c.rx = ax.rw[i];
    c.y0 = ay.c[j];
    c.uy = (j == ay.n - 2) ? __builtin_inf() : ay.c[j + 1];
    c.ry = ay.rw[j];
    if (P.g.coslat) {
        c.cl = P.g.coslat[j];
        c.sl = P.g.sinlat[j];
    }
    const size_t nx = (size_t)ax.n;
    c.land = P.g.landcell ? P.g.landcell[(size_t)j * (nx - 1) + (size_t)i] != 0 : false;
    const size_t n00 = (size_t)j * nx + (size_t)i;
    const char *base = static_cast<const char *>(P.f.slots);
    const char *A = base + (size_t)sa * P.f.slot_bytes;
    const float *sca = ST == kF16S ? P.f.scales + (size_t)sa * P.f.nzl * 3 : nullptr;
    R p00[3], p10[3], p01[3], p11[3];
    load_node<ST, false>(A, n00, sca, p00);
    load_node<ST, false>(A, n00 + 1, sca, p10);
    load_node<ST, false>(A, n00 + nx, sca, p01);
    load_node<ST, false>(A, n00 + nx + 1, sca, p11);
    if constexpr (!STEADY) {
        const char *B = base + (size_t)sb * P.f.slot_bytes;
        const float *scb = ST == kF16S ? P.f.scales + (size_t)sb * P.f.nzl * 3 : nullptr;
        R q00[3], q10[3], q01[3], q11[3];
        load_node<ST, false>(B, n00, scb, q00);
        load_node<ST, false>(B, n00 + 1, scb, q10);
        load_node<ST, false>(B, n00 + nx, scb, q01);
        load_node<ST, false>(B, n00 + nx + 1, scb, q11);
#pragma unroll
        for (int v = 0; v < 2; ++v) {
            R cb[4];
            coeffs<R>(q00[v], q10[v], q01[v], q11[v], cb);
            coeffs<R>(p00[v], p10[v], p01[v], p11[v], c.a[v]);
#pragma unroll
            for (int q = 0; q < 4; ++q)
                c.d[v][q] = cb[q] - c.a[v][q];
        }
    } else {
#pragma unroll
        for (int v = 0; v < 2; ++v)
            coeffs<R>(p00[v], p10[v], p01[v], p11[v], c.a[v]);
    }
    c.valid = true;
    return true;
}

template <class R>
__device__ inline bool in_cell(const Cell2<R> &c, const AdvectParams &P, double x, double y)
{
    return c.valid && x >= c.x0 && x < c.ux && x <= P.g.ax.hi && y >= c.y0 && y < c.uy &&
           y <= P.g.ay.hi;
}

// 1 / d to within an ulp or two: hardware reciprocal refined by two Newton steps
__device__ inline double recip(double d)
{
    double r = __builtin_amdgcn_rcp(d);
    r = fma(fma(-d, r, 1.0), r, r);
    r = fma(fma(-d, r, 1.0), r, r);
    return r;
}

// cos of a latitude inside the cached cell: cos(l0 + dl) = cos l0 cos dl - sin l0 sin dl
// with dl = lat - l0 (at most 5 degrees) and cos dl, sin dl by their Taylor series to
// order dl^8 / dl^9 (truncation below 1e-17).
template <class R>
__device__ inline double cos_lat(const Cell2<R> &c, const AdvectParams &P, double y)
{
    if (!P.g.coslat)
        return cos(y * kDegToRad);
    const double dl = (y - c.y0) * kDegToRad, d2 = dl * dl;
    const double cd = fma(d2, fma(d2, fma(d2, fma(d2, 1.0 / 40320.0, -1.0 / 720.0), 1.0 / 24.0),
                                  -0.5), 1.0);
    const double sd = dl * fma(d2, fma(d2, fma(d2, fma(d2, 1.0 / 362880.0, -1.0 / 5040.0),
                                                1.0 / 120.0), -1.0 / 6.0), 1.0);
    return c.cl * cd - c.sl * sd;
}

template <int ST, bool STEADY, bool SPH>
__device__ inline bool stage2(const AdvectParams &P, Cell2<typename Real<ST>::T> &c,
                              const TimeEntry &e, double x, double y, double &kx, double &ky)
{
    using R = typename Real<ST>::T;
    if (!in_cell(c, P, x, y)) {
        if (!reload2<ST, STEADY>(P, c, e.sa, e.sb, x, y))
            return false;
    }
    R xi = (R)((x - c.x0) * c.rx), eta = (R)((y - c.y0) * c.ry);
    if (P.nearest) {
        xi = xi < (R)0.5 ? (R)0 : (R)1;
        eta = eta < (R)0.5 ? (R)0 : (R)1;
    }
    R u = poly<R>(c.a[0], xi, eta), v = poly<R>(c.a[1], xi, eta);
    if constexpr (!STEADY) {
        const R tau = (R)e.tau;
        u = fma(tau, poly<R>(c.d[0], xi, eta), u);
        v = fma(tau, poly<R>(c.d[1], xi, eta), v);
    }
    if constexpr (SPH) {
        kx = (double)u * recip(kMetresPerDegree * cos_lat(c, P, y));
        ky = (double)v * (1.0 / kMetresPerDegree);
    } else {
        kx = (double)u;
        ky = (double)v;
    }
    return true;
}

// One particle (position k of the processing order) for all steps of the launch;
// returns the number of steps it started active.
template <int ST, bool STEADY, bool SPH>
__device__ inline long long advect_lane_2d(const AdvectParams &P, uint32_t k, uint32_t nact)
{
    using R = typename Real<ST>::T;
    long long steps = 0;
    if (k < nact) {
        const uint32_t id = P.order[k];
        uint8_t st = P.status[id];
        if (st == 0) {
            double x = P.x[id], y = P.y[id];
            Cell2<R> c;
            c.valid = false;
            int csa = -1, csb = -1;  // bracket the cached stencils belong to
            const double dt = P.dt, hd = 0.5 * dt, dt6 = dt * (1.0 / 6.0);
            for (int s = 0; s < P.nsteps; ++s) {
                ++steps;
                const TimeEntry e0 = P.tab[2 * s], e1 = P.tab[2 * s + 1], e2 = P.tab[2 * s + 2];
                uint8_t err = ST_OOB;
                // the four stages: offsets 0, dt/2, dt/2, dt from X_n along the previous
                // slope; weights 1, 2, 2, 1
                double kx = 0.0, ky = 0.0, sx = 0.0, sy = 0.0;
                const int nst = P.scheme ? 1 : 4;
#pragma nounroll
                for (int q = 0; q < nst; ++q) {
                    const TimeEntry e = q == 0 ? e0 : (q == 3 ? e2 : e1);
                    const double h = q == 0 ? 0.0 : (q == 3 ? dt : hd);
                    if (e.sa != csa || e.sb != csb) {
                        c.valid = false;
                        csa = e.sa;
                        csb = e.sb;
                    }
                    if (!stage2<ST, STEADY, SPH>(P, c, e, x + kx * h, y + ky * h, kx, ky))
                        goto fail;
                    if (q == 1 || q == 2) {
                        sx += 2.0 * kx;
                        sy += 2.0 * ky;
                    } else if (q == 0) {
                        sx = kx;
                        sy = ky;
                    }
                }
                {
                    double xs, ys;
                    if (P.scheme) {  // Euler forward
                        xs = x + kx * dt;
                        ys = y + ky * dt;
                    } else {
                        xs = x + (sx + kx) * dt6;
                        ys = y + (sy + ky) * dt6;
                    }
                    if (P.Kh > 0.0) {
                        uint32_t w[4] = {id, (uint32_t)(P.step0 + s), 0u, 0u};
                        philox4x32_10(w, P.run_id, P.seed);
                        const double u1 = unit53(w[0], w[1]), u2 = unit53(w[2], w[3]);
                        const double r = sqrt(-2.0 * log(u1));
                        double sn, cs;
                        sincos((2.0 * 3.141592653589793) * u2, &sn, &cs);
                        const double sig = sqrt(2.0 * P.Kh * dt);
                        double dx = sig * (r * cs), dy = sig * (r * sn);
                        if constexpr (SPH) {
                            dx = dx / (kMetresPerDegree * cos(ys * kDegToRad));
                            dy = dy / kMetresPerDegree;
                        }
                        xs = xs + dx;
                        ys = ys + dy;
                    }
                    bool land;
                    if (in_cell(c, P, xs, ys)) {
                        land = c.land;
                    } else {
                        int ci, cj;
                        double f;
                        if (!locate(P.g.ax, xs, ci, f) || !locate(P.g.ay, ys, cj, f))
                            goto fail;
                        land = P.g.landcell &&
                               P.g.landcell[(size_t)cj * (size_t)(P.g.ax.n - 1) + (size_t)ci];
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
            P.x[id] = x;
            P.y[id] = y;
            if (st)
                P.status[id] = st;
        }
    }
    return steps;
}

template <int ST, bool STEADY, bool SPH>
__global__ __launch_bounds__(kBlock) void k_advect2d(AdvectParams P)
{
    const uint32_t blk = xcd_block(blockIdx.x, gridDim.x);
    const uint32_t k = blk * kBlock + threadIdx.x;
    long long steps = advect_lane_2d<ST, STEADY, SPH>(P, k, *P.n_active);
    for (int off = 32; off > 0; off >>= 1)
        steps += __shfl_xor(steps, off, 64);
    if ((threadIdx.x & 63) == 0 && steps)
        atomicAdd(P.psteps, (unsigned long long)steps);
}

// Persistent batched launch over many independent runs (each with its own grid,
// snapshots and particles).  The active particles of every run are cut into
// chunks of blockDim particles; the chunk items are split into 8 contiguous
// ranges, one per XCD, each with its own atomic counter.  A block takes items from
// the range of the XCD it runs on and, when that is exhausted, from the others;
// every block leaves once all 8 ranges are exhausted, so the grid always drains.
template <int ST, bool STEADY, bool SPH>
__global__ __launch_bounds__(512) void k_advect2d_batch(const AdvectParams *runs,
                                                        const uint32_t *cstart, int nruns,
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
        long long steps = advect_lane_2d<ST, STEADY, SPH>(P, k, *P.n_active);
        for (int off = 32; off > 0; off >>= 1)
            steps += __shfl_xor(steps, off, 64);
        if ((threadIdx.x & 63) == 0 && steps)
            atomicAdd(P.psteps, (unsigned long long)steps);
    }
}

// ---------------------------------------------------------------- 3D with a stencil cache
// Same scheme in three dimensions: the trilinear interpolant of U, V, W in the
// cached cell written as c0 + c1 xi + c2 eta + c3 zeta + c4 xi eta + c5 xi zeta +
// c6 eta zeta + c7 xi eta zeta, for the earlier snapshot and the difference.
template <class R>
struct Cell3 {
    double x0, ux, y0, uy, z0, uz;
    double rx, ry, rz;
    double cl, sl;
    R a[3][8];
    R d[3][8];
    bool land;
    bool valid;
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

template <int ST, bool STEADY>
__device__ inline bool reload3(const AdvectParams &P, Cell3<typename Real<ST>::T> &c, int sa,
                               int sb, double x, double y, double z)
{
    using R = typename Real<ST>::T;
    int i, j, k;
    double f;
    if (!locate(P.g.ax, x, i, f) || !locate(P.g.ay, y, j, f) || !locate(P.g.az, z, k, f))
        return false;
    const AxisDev &ax = P.g.ax, &ay = P.g.ay, &az = P.g.az;
    c.x0 = ax.c[i];
    c.ux = (i == ax.n - 2) ? __builtin_inf() : ax.c[i + 1];
    c.rx = ax.rw[i];
    c.y0 = ay.c[j];
    c.uy = (j == ay.n - 2) ? __builtin_inf() : ay.c[j + 1];
    c.ry = ay.rw[j];
    c.z0 = az.c[k];
    c.uz = (k == az.n - 2) ? __builtin_inf() : az.c[k + 1];
    c.rz = az.rw[k];
    if (P.g.coslat) {
        c.cl = P.g.coslat[j];
        c.sl = P.g.sinlat[j];
    }
    const size_t nx = (size_t)ax.n, plane = nx * (size_t)ay.n;
    c.land = P.g.landcell ? P.g.landcell[(size_t)j * (nx - 1) + (size_t)i] != 0 : false;
    const size_t n000 = (size_t)k * plane + (size_t)j * nx + (size_t)i;
    const size_t off[8] = {0, 1, nx, nx + 1, plane, plane + 1, plane + nx, plane + nx + 1};
    const char *base = static_cast<const char *>(P.f.slots);
    {
        const char *A = base + (size_t)sa * P.f.slot_bytes;
        R fa[3][8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float *sc = ST == kF16S ? P.f.scales + ((size_t)sa * P.f.nzl + k + (q >> 2)) * 3
                                          : nullptr;
            R v[3];
            load_node<ST, true>(A, n000 + off[q], sc, v);
            fa[0][q] = v[0];
            fa[1][q] = v[1];
            fa[2][q] = v[2];
        }
#pragma unroll
        for (int v = 0; v < 3; ++v)
            coeffs3<R>(fa[v], c.a[v]);
    }
    if constexpr (!STEADY) {
        const char *B = base + (size_t)sb * P.f.slot_bytes;
        R fb[3][8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float *sc = ST == kF16S ? P.f.scales + ((size_t)sb * P.f.nzl + k + (q >> 2)) * 3
                                          : nullptr;
            R v[3];
            load_node<ST, true>(B, n000 + off[q], sc, v);
            fb[0][q] = v[0];
            fb[1][q] = v[1];
            fb[2][q] = v[2];
        }
#pragma unroll
        for (int v = 0; v < 3; ++v) {
            R cb[8];
            coeffs3<R>(fb[v], cb);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                c.d[v][q] = cb[q] - c.a[v][q];
        }
    }
    c.valid = true;
    return true;
}

template <class R>
__device__ inline bool in_cell3(const Cell3<R> &c, const AdvectParams &P, double x, double y,
                                double z)
{
    return c.valid && x >= c.x0 && x < c.ux && x <= P.g.ax.hi && y >= c.y0 && y < c.uy &&
           y <= P.g.ay.hi && z >= c.z0 && z < c.uz && z <= P.g.az.hi;
}

template <int ST, bool STEADY, bool SPH>
__device__ inline bool stage3(const AdvectParams &P, Cell3<typename Real<ST>::T> &c,
                              const TimeEntry &e, double x, double y, double z, double k[3])
{
    using R = typename Real<ST>::T;
    if (!in_cell3(c, P, x, y, z)) {
        if (!reload3<ST, STEADY>(P, c, e.sa, e.sb, x, y, z))
            return false;
    }
    R xi = (R)((x - c.x0) * c.rx), eta = (R)((y - c.y0) * c.ry);
    R zeta = (R)((z - c.z0) * c.rz);
    if (P.nearest) {
        xi = xi < (R)0.5 ? (R)0 : (R)1;
        eta = eta < (R)0.5 ? (R)0 : (R)1;
        zeta = zeta < (R)0.5 ? (R)0 : (R)1;
    }
    R v[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        v[q] = poly3<R>(c.a[q], xi, eta, zeta);
        if constexpr (!STEADY)
            v[q] = fma((R)e.tau, poly3<R>(c.d[q], xi, eta, zeta), v[q]);
    }
    if constexpr (SPH) {
        double cosl;
        if (P.g.coslat) {
            const double dl = (y - c.y0) * kDegToRad, d2 = dl * dl;
            const double cd = fma(d2, fma(d2, fma(d2, fma(d2, 1.0 / 40320.0, -1.0 / 720.0),
                                                  1.0 / 24.0), -0.5), 1.0);
            const double sd = dl * fma(d2, fma(d2, fma(d2, fma(d2, 1.0 / 362880.0,
                                                                -1.0 / 5040.0), 1.0 / 120.0),
                                                -1.0 / 6.0), 1.0);
            cosl = c.cl * cd - c.sl * sd;
        } else {
            cosl = cos(y * kDegToRad);
        }
        k[0] = (double)v[0] * recip(kMetresPerDegree * cosl);
        k[1] = (double)v[1] * (1.0 / kMetresPerDegree);
    } else {
        k[0] = (double)v[0];
        k[1] = (double)v[1];
    }
    k[2] = (double)v[2];
    return true;
}

template <int ST, bool STEADY, bool SPH>
__global__ __launch_bounds__(kBlock) void k_advect3d(AdvectParams P)
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
            Cell3<R> c;
            c.valid = false;
            int csa = -1, csb = -1;
            const double dt = P.dt, hd = 0.5 * dt, dt6 = dt * (1.0 / 6.0);
            for (int s = 0; s < P.nsteps; ++s) {
                ++steps;
                const TimeEntry e0 = P.tab[2 * s], e1 = P.tab[2 * s + 1], e2 = P.tab[2 * s + 2];
                uint8_t err = ST_OOB;
                double k[3] = {0.0, 0.0, 0.0}, sm[3] = {0.0, 0.0, 0.0};
                const int nst = P.scheme ? 1 : 4;
#pragma nounroll
                for (int q = 0; q < nst; ++q) {
                    const TimeEntry e = q == 0 ? e0 : (q == 3 ? e2 : e1);
                    const double h = q == 0 ? 0.0 : (q == 3 ? dt : hd);
                    if (e.sa != csa || e.sb != csb) {
                        c.valid = false;
                        csa = e.sa;
                        csb = e.sb;
                    }
                    if (!stage3<ST, STEADY, SPH>(P, c, e, x + k[0] * h, y + k[1] * h,
                                                 z + k[2] * h, k))
                        goto fail;
#pragma unroll
                    for (int v = 0; v < 3; ++v)
                        sm[v] = q == 0 ? k[v] : (q == 3 ? sm[v] : fma(2.0, k[v], sm[v]));
                }
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
                    if (P.Kh > 0.0) {
                        uint32_t w[4] = {id, (uint32_t)(P.step0 + s), 0u, 0u};
                        philox4x32_10(w, P.run_id, P.seed);
                        const double u1 = unit53(w[0], w[1]), u2 = unit53(w[2], w[3]);
                        const double r = sqrt(-2.0 * log(u1));
                        double sn, cs;
                        sincos((2.0 * 3.141592653589793) * u2, &sn, &cs);
                        const double sig = sqrt(2.0 * P.Kh * dt);
                        double dx = sig * (r * cs), dy = sig * (r * sn);
                        if constexpr (SPH) {
                            dx = dx / (kMetresPerDegree * cos(ys * kDegToRad));
                            dy = dy / kMetresPerDegree;
                        }
                        xs = xs + dx;
                        ys = ys + dy;
                    }
                    bool land;
                    if (in_cell3(c, P, xs, ys, zs)) {
                        land = c.land;
                    } else {
                        int ci, cj, ck;
                        double f;
                        if (!locate(P.g.ax, xs, ci, f) || !locate(P.g.ay, ys, cj, f) ||
                            !locate(P.g.az, zs, ck, f))
                            goto fail;
                        land = P.g.landcell &&
                               P.g.landcell[(size_t)cj * (size_t)(P.g.ax.n - 1) + (size_t)ci];
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
            P.x[id] = x;
            P.y[id] = y;
            P.z[id] = z;
            if (st)
                P.status[id] = st;
        }
    }
    for (int off = 32; off > 0; off >>= 1)
        steps += __shfl_xor(steps, off, 64);
    if ((threadIdx.x & 63) == 0 && steps)
        atomicAdd(P.psteps, (unsigned long long)steps);
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
        const double u1 = unit53(w[0], w[1]), u2 = unit53(w[2], w[3]);
        const double r = sqrt(-2.0 * log(u1));
        double sn, cs;
        sincos((2.0 * 3.141592653589793) * u2, &sn, &cs);
        normals[2 * i] = r * cs;
        normals[2 * i + 1] = r * sn;
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
    }
}

template <int ST, bool IS3D>
hipError_t launch3(const AdvectParams &p, bool steady, uint32_t n_launch, hipStream_t s)
{
    const uint32_t blocks = (n_launch + kBlock - 1) / kBlock;
    if (blocks == 0)
        return hipSuccess;
    if (!p.cache) {
        if (steady)
            hipLaunchKernelGGL((k_advect<ST, IS3D, true>), dim3(blocks), dim3(kBlock), 0, s, p);
        else
            hipLaunchKernelGGL((k_advect<ST, IS3D, false>), dim3(blocks), dim3(kBlock), 0, s, p);
        return hipGetLastError();
    }
    if constexpr (!IS3D) {
        const dim3 g(blocks), b(kBlock);
        if (p.g.spherical) {
            if (steady)
                hipLaunchKernelGGL((k_advect2d<ST, true, true>), g, b, 0, s, p);
            else
                hipLaunchKernelGGL((k_advect2d<ST, false, true>), g, b, 0, s, p);
        } else {
            if (steady)
                hipLaunchKernelGGL((k_advect2d<ST, true, false>), g, b, 0, s, p);
            else
                hipLaunchKernelGGL((k_advect2d<ST, false, false>), g, b, 0, s, p);
        }
        return hipGetLastError();
    } else {
        const dim3 g(blocks), b(kBlock);
        if (p.g.spherical) {
            if (steady)
                hipLaunchKernelGGL((k_advect3d<ST, true, true>), g, b, 0, s, p);
            else
                hipLaunchKernelGGL((k_advect3d<ST, false, true>), g, b, 0, s, p);
        } else {
            if (steady)
                hipLaunchKernelGGL((k_advect3d<ST, true, false>), g, b, 0, s, p);
            else
                hipLaunchKernelGGL((k_advect3d<ST, false, false>), g, b, 0, s, p);
        }
        return hipGetLastError();
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

template <int ST, bool IS3D>
hipError_t rkf3(const AdvectParams &p, bool steady, uint32_t n_launch, hipStream_t s)
{
    const uint32_t blocks = (n_launch + kBlock - 1) / kBlock;
    if (blocks == 0)
        return hipSuccess;
    if (steady)
        hipLaunchKernelGGL((k_rkf45<ST, IS3D, true>), dim3(blocks), dim3(kBlock), 0, s, p);
    else
        hipLaunchKernelGGL((k_rkf45<ST, IS3D, false>), dim3(blocks), dim3(kBlock), 0, s, p);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_rkf45(int store, bool is3d, const AdvectParams &p, uint32_t n_launch,
                        hipStream_t s)
{
    const bool steady = p.f.steady != 0;
    if (!p.res || p.nres < 1 || (!steady && p.period <= 0.0 && p.nres < 2) || !p.hexp ||
        !p.prej)
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

template <int ST, bool STEADY, bool SPH>
hipError_t batch3(const AdvectParams *runs, const uint32_t *cstart, int nruns, uint32_t total,
                  uint32_t *queues, int block, hipStream_t s, int *grid_out)
{
    auto kern = k_advect2d_batch<ST, STEADY, SPH>;
    int per_cu = 0, cus = 0, dev = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, block, 0);
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
    hipLaunchKernelGGL(kern, dim3(grid), dim3(block), 0, s, runs, cstart, nruns, total, queues);
    return hipGetLastError();
}

hipError_t launch_advect_batch(int store, bool steady, bool spherical, const AdvectParams *runs,
                               const uint32_t *cstart, int nruns, uint32_t total,
                               uint32_t *queues, int block, hipStream_t s, int *grid_out)
{
    hipError_t e = launch_fill_u32(queues, 0u, 8, s);
    if (e != hipSuccess || total == 0)
        return e;
#define LP_B(ST)                                                                                \
    if (spherical)                                                                              \
        return steady ? batch3<ST, true, true>(runs, cstart, nruns, total, queues, block, s, grid_out)  \
                      : batch3<ST, false, true>(runs, cstart, nruns, total, queues, block, s, grid_out); \
    return steady ? batch3<ST, true, false>(runs, cstart, nruns, total, queues, block, s, grid_out)     \
                  : batch3<ST, false, false>(runs, cstart, nruns, total, queues, block, s, grid_out);
    switch (store) {
    case kF64: { LP_B(kF64) }
    case kF32: { LP_B(kF32) }
    case kBF16: { LP_B(kBF16) }
    case kF16S: { LP_B(kF16S) }
    }
#undef LP_B
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
