/*
 * lp_oracle.c -- plain FP64 reference for Lagrangian RK4 advection on rectilinear
 * grids.  TEST INFRASTRUCTURE ONLY: it is built and called by the tests, the smoke
 * check and the CPU-baseline leg of the benchmark, never by the product library.
 * It shares no source with the HIP path.  Compiled with -O2 -ffp-contract=off so
 * every product and sum is rounded exactly where it is written.
 *
 * What it follows (Lange & van Sebille, Parcels v0.9):
 *   - the trajectory equation, Eq. (1), integrated with the classical fourth-order
 *     Runge-Kutta scheme (Sect. 2.1.1, the default integrator);
 *   - field sampling fieldset.F[time, lon, lat, depth] (Sect. 2.1.2) done as linear
 *     interpolation in space and linear interpolation in time, on grids whose axes
 *     depend on lon only, lat only or depth only (Sect. 2.3, Sect. 2.4);
 *   - conversion of m/s to degrees/s on a spherical mesh (Sect. 4.2.2);
 *   - per-particle error states handled by recovery (delete on leaving the
 *     domain, Sect. 2.1.2 and Sect. 3.3);
 *   - a Brownian displacement with uniform Kh (the behaviour term of Eq. (1),
 *     Sect. 2.1.2 and Sect. 4.2.7), drawn with Philox4x32-10 (Salmon et al.,
 *     "Parallel random numbers: as easy as 1, 2, 3", SC'11);
 *   - the alternative integrators named in Sect. 2.1.1: Euler forward and the
 *     adaptive Runge-Kutta-Fehlberg pair RKF45 (Fehlberg, NASA TR R-315, 1969),
 *     with the step-size control read below;
 *   - the custom kernels of the worked example (Sect. 3.3): sinking, age with
 *     deletion at a maximum age, and sampling of a tracer (temperature), run
 *     before the advection of each step.
 *
 * Readings where the paper is silent (each one is listed with its reason in the
 * design notes): classical RK4 tableau; lower-cell rule at a node with the last
 * node in the last cell; space first, then time; metres per degree 1852*60;
 * cos(lat) taken at each stage point; a step is rejected whole if any stage
 * point or the end point leaves the domain; a land cell has four land corners.
 * RKF45 (the paper names it only): the fourth-order solution advances the
 * particle; the error is the length in metres of the fifth-minus-fourth-order
 * difference; each particle's step is |dt| 2^e with an integer e in [emin, emax]
 * that starts at 0; a step with error above tol is retried at half the size
 * (unless e = emin), an accepted step with error at most tol/32 doubles the next
 * one (up to emax); the step is cut short to land on the end of the output
 * interval, and a cut step leaves e as it was.
 * Worked-example kernels (their code is not in the text): each step first sinks
 * a particle deeper than its dwelling depth by w_s dt, not past that depth (a
 * time-backward run raises it back to where it lived); then a particle at or
 * above the dwelling depth ages by |dt| and is deleted once its age reaches
 * maxage; then the tracer is sampled at the step's start; then RK4 advects it,
 * horizontally only while it is at its dwelling depth.
 */
#include <math.h>
#include <stdint.h>
#include <stddef.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_ST_OOB 1u
#define OR_ST_LAND 2u
#define OR_ST_DELETED 4u
#define OR_ST_AGED 8u

#define OR_OK 0
#define OR_EINVAL (-1)
#define OR_ETIME (-4)

/* metres per degree (one nautical mile per arc minute) and degrees to radians */
static const double OR_M = 111120.0;
static const double OR_D = 0.017453292519943295;

typedef struct {
    int nx, ny, nz;          /* nz = 0: two-dimensional field set */
    const double *X, *Y, *Z; /* strictly increasing axes */
    int spherical;
    int nt;
    const double *T;         /* snapshot times, strictly increasing */
    double period;           /* > 0: the snapshots repeat with this period */
    int stored_f32;          /* 1: U, V, W hold float; 0: double */
    const void *U, *V, *W;   /* [nt][max(nz,1)][ny][nx], i fastest */
    const unsigned char *land; /* [ny][nx] node mask (1 = land) or NULL */
    const void *tracer;      /* scalar tracer, laid out like U, or NULL */
    int tracer_f32;          /* 1: the tracer holds float */
} or_fieldset;

typedef struct {
    int policy;              /* 0: delete on error, 1: freeze on error */
    double Kh;               /* horizontal diffusivity, 0 = no Brownian term */
    uint32_t run_id, seed;   /* Philox key */
    int scheme;              /* 0: classical RK4, 1: Euler forward, 2: RKF45 (Sect. 2.1.1) */
    int nearest;             /* 1: nearest-neighbour instead of linear in space (Sect. 2.3) */
    double tol;              /* RKF45: error tolerance per step in metres */
    int emin, emax;          /* RKF45: range of the step exponent e, step = |dt| 2^e */
    double sink_speed;       /* m/s, > 0: the sinking kernel (3D) */
    double dwell_depth;      /* m: depth the particle lives at */
    double maxage;           /* s, > 0: the age kernel deletes at this age */
    int sample;              /* 1: sample the tracer into the particle's temp */
} or_options;

/* ---------------------------------------------------------------- cell search */
/* Locate x on axis X[0..n-1]: returns 1 if x is NaN or outside [X0, X(n-1)];
 * otherwise idx = the largest i in [0, n-2] with X[i] <= x and
 * frac = (x - X[i]) / (X[i+1] - X[i]).  A point on the last node is in the last
 * cell with frac = 1. */
int or_locate(double x, const double *X, int n, int *idx, double *frac)
{
    if (x != x || x < X[0] || x > X[n - 1])
        return 1;
    int lo = 0, hi = n - 2;
    while (lo < hi) {
        int mid = lo + (hi - lo + 1) / 2;
        if (X[mid] <= x)
            lo = mid;
        else
            hi = mid - 1;
    }
    *idx = lo;
    *frac = (x - X[lo]) / (X[lo + 1] - X[lo]);
    return 0;
}

static double rd(const or_fieldset *fs, const void *F, size_t off)
{
    const int f32 = F == fs->tracer ? fs->tracer_f32 : fs->stored_f32;
    if (f32)
        return (double)((const float *)F)[off];
    return ((const double *)F)[off];
}

/* bilinear interpolation on level k of snapshot s: the four corner weights times
 * the corner values, products evaluated first, then summed left to right */
static double bilinear(const or_fieldset *fs, const void *F, int s, int k,
                       int i, int j, double xi, double eta)
{
    size_t nx = (size_t)fs->nx, ny = (size_t)fs->ny;
    size_t nzl = fs->nz > 0 ? (size_t)fs->nz : 1;
    size_t base = (((size_t)s * nzl) + (size_t)k) * ny * nx;
    double f00 = rd(fs, F, base + (size_t)j * nx + (size_t)i);
    double f10 = rd(fs, F, base + (size_t)j * nx + (size_t)i + 1);
    double f11 = rd(fs, F, base + ((size_t)j + 1) * nx + (size_t)i + 1);
    double f01 = rd(fs, F, base + ((size_t)j + 1) * nx + (size_t)i);
    double p0 = ((1.0 - xi) * (1.0 - eta)) * f00;
    double p1 = (xi * (1.0 - eta)) * f10;
    double p2 = (xi * eta) * f11;
    double p3 = ((1.0 - xi) * eta) * f01;
    return ((p0 + p1) + p2) + p3;
}

typedef struct {
    int i, j, k;
    double xi, eta, zeta;
} or_cell;

static double spatial(const or_fieldset *fs, const void *F, int s, const or_cell *c)
{
    if (fs->nz <= 0)
        return bilinear(fs, F, s, 0, c->i, c->j, c->xi, c->eta);
    double lo = bilinear(fs, F, s, c->k, c->i, c->j, c->xi, c->eta);
    double hi = bilinear(fs, F, s, c->k + 1, c->i, c->j, c->xi, c->eta);
    return (1.0 - c->zeta) * lo + c->zeta * hi;
}

/* ---------------------------------------------------------------- time bracket */
/* Bracketing snapshots for time t.  nt == 1: steady (s0 = s1 = 0, tau = 0).
 * Periodic: t is first mapped into [T0, T0 + period) and the snapshot after the
 * last one is the first one again, at T0 + period.  Otherwise t must lie in
 * [T0, T(nt-1)]. */
int or_time_bracket(const or_fieldset *fs, double t, int *s0, int *s1, double *tau)
{
    const double *T = fs->T;
    int nt = fs->nt;
    if (nt == 1) {
        *s0 = 0;
        *s1 = 0;
        *tau = 0.0;
        return OR_OK;
    }
    if (fs->period > 0.0) {
        double r = fmod(t - T[0], fs->period);
        if (r < 0.0)
            r += fs->period;
        double tp = T[0] + r;
        int s = 0;
        for (int q = 0; q < nt; q++)
            if (T[q] <= tp)
                s = q;
        double tnext = (s + 1 < nt) ? T[s + 1] : T[0] + fs->period;
        *s0 = s;
        *s1 = (s + 1 < nt) ? s + 1 : 0;
        *tau = (tp - T[s]) / (tnext - T[s]);
        return OR_OK;
    }
    if (t != t || t < T[0] || t > T[nt - 1])
        return OR_ETIME;
    int s = 0;
    for (int q = 0; q <= nt - 2; q++)
        if (T[q] <= t)
            s = q;
    *s0 = s;
    *s1 = s + 1;
    *tau = (t - T[s]) / (T[s + 1] - T[s]);
    return OR_OK;
}

/* ---------------------------------------------------------------- sampling */
/* Velocity at (x, y, z, t) in coordinate units per second.  Returns 1 if the
 * point is outside the grid (the caller has checked t).  Nearest-neighbour
 * sampling snaps each cell fraction to its nearer node (a fraction of exactly 0.5
 * to the upper one), which turns the linear weights into one unit weight; time
 * stays linear. */
static int sample_mode(const or_fieldset *fs, double x, double y, double z, double t,
                       double out[3], int nearest)
{
    or_cell c = {0, 0, 0, 0.0, 0.0, 0.0};
    if (or_locate(x, fs->X, fs->nx, &c.i, &c.xi))
        return 1;
    if (or_locate(y, fs->Y, fs->ny, &c.j, &c.eta))
        return 1;
    if (fs->nz > 0 && or_locate(z, fs->Z, fs->nz, &c.k, &c.zeta))
        return 1;
    if (nearest) {
        c.xi = c.xi < 0.5 ? 0.0 : 1.0;
        c.eta = c.eta < 0.5 ? 0.0 : 1.0;
        c.zeta = c.zeta < 0.5 ? 0.0 : 1.0;
    }
    int s0, s1;
    double tau;
    if (or_time_bracket(fs, t, &s0, &s1, &tau) != OR_OK)
        return 2;
    double u, v, w = 0.0;
    if (fs->nt == 1) {
        u = spatial(fs, fs->U, 0, &c);
        v = spatial(fs, fs->V, 0, &c);
        if (fs->nz > 0)
            w = spatial(fs, fs->W, 0, &c);
    } else {
        u = (1.0 - tau) * spatial(fs, fs->U, s0, &c) + tau * spatial(fs, fs->U, s1, &c);
        v = (1.0 - tau) * spatial(fs, fs->V, s0, &c) + tau * spatial(fs, fs->V, s1, &c);
        if (fs->nz > 0)
            w = (1.0 - tau) * spatial(fs, fs->W, s0, &c) + tau * spatial(fs, fs->W, s1, &c);
    }
    if (fs->spherical) {
        out[0] = u / (OR_M * cos(y * OR_D));
        out[1] = v / OR_M;
    } else {
        out[0] = u;
        out[1] = v;
    }
    out[2] = w;
    return 0;
}

int or_sample(const or_fieldset *fs, double x, double y, double z, double t, double out[3])
{
    return sample_mode(fs, x, y, z, t, out, 0);
}

int or_sample_nearest(const or_fieldset *fs, double x, double y, double z, double t,
                      double out[3])
{
    return sample_mode(fs, x, y, z, t, out, 1);
}

/* Tracer value at (x, y, z, t), linear in space and time like the velocity.
 * Returns 1 outside the grid, 2 outside the snapshots, 3 without a tracer. */
int or_sample_tracer(const or_fieldset *fs, double x, double y, double z, double t,
                     double *val)
{
    if (!fs->tracer)
        return 3;
    or_cell c = {0, 0, 0, 0.0, 0.0, 0.0};
    if (or_locate(x, fs->X, fs->nx, &c.i, &c.xi) || or_locate(y, fs->Y, fs->ny, &c.j, &c.eta))
        return 1;
    if (fs->nz > 0 && or_locate(z, fs->Z, fs->nz, &c.k, &c.zeta))
        return 1;
    int s0, s1;
    double tau;
    if (or_time_bracket(fs, t, &s0, &s1, &tau) != OR_OK)
        return 2;
    if (fs->nt == 1)
        *val = spatial(fs, fs->tracer, 0, &c);
    else
        *val = (1.0 - tau) * spatial(fs, fs->tracer, s0, &c) +
               tau * spatial(fs, fs->tracer, s1, &c);
    return 0;
}

/* ---------------------------------------------------------------- Philox4x32-10 */
/* Counter-based generator of Salmon et al. (SC'11): ten rounds of the four-word
 * Philox round, each multiplying words 0 and 2 by the two round multipliers and
 * xoring the high halves into the other words together with the key; the key is
 * bumped by the two Weyl constants between rounds. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) {
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0;
        c1 = lo1;
        c2 = n2;
        c3 = lo0;
    }
    out[0] = c0;
    out[1] = c1;
    out[2] = c2;
    out[3] = c3;
}

/* Uniform in (0, 1) from two words: the top 53 bits of (a:b) scaled by 2^-53,
 * plus 2^-54 so that neither end is reached. */
static double or_unit(uint32_t a, uint32_t b)
{
    uint64_t m = (((uint64_t)a << 32) | (uint64_t)b) >> 11;
    return (double)m * 1.1102230246251565e-16 + 5.551115123125783e-17;
}

/* Two standard normals for (run, seed, particle, step) by Box-Muller. */
void or_normals(uint32_t run_id, uint32_t seed, uint32_t pid, uint32_t step, double n[2])
{
    uint32_t ctr[4] = {pid, step, 0u, 0u};
    uint32_t key[2] = {run_id, seed};
    uint32_t w[4];
    or_philox4x32_10(ctr, key, w);
    double u1 = or_unit(w[0], w[1]);
    double u2 = or_unit(w[2], w[3]);
    double r = sqrt(-2.0 * log(u1));
    double a = (2.0 * 3.141592653589793) * u2;
    n[0] = r * cos(a);
    n[1] = r * sin(a);
}

/* ---------------------------------------------------------------- one RK4 step */
static int in_domain(const or_fieldset *fs, double x, double y, double z, or_cell *c)
{
    if (or_locate(x, fs->X, fs->nx, &c->i, &c->xi))
        return 0;
    if (or_locate(y, fs->Y, fs->ny, &c->j, &c->eta))
        return 0;
    if (fs->nz > 0 && or_locate(z, fs->Z, fs->nz, &c->k, &c->zeta))
        return 0;
    return 1;
}

static int land_cell(const or_fieldset *fs, int i, int j)
{
    const unsigned char *L = fs->land;
    size_t nx = (size_t)fs->nx;
    return L[(size_t)j * nx + i] && L[(size_t)j * nx + i + 1] &&
           L[((size_t)j + 1) * nx + i] && L[((size_t)j + 1) * nx + i + 1];
}

/* Advance one particle by step n (time t_org + n dt to t_org + (n+1) dt). */
static void rk4_step(const or_fieldset *fs, const or_options *opt, double t_org, double dt,
                     int64_t n, uint32_t pid, double *px, double *py, double *pz,
                     unsigned char *st, int horizontal)
{
    const int is3d = fs->nz > 0;
    const unsigned char err_extra = opt->policy == 0 ? OR_ST_DELETED : 0;
    double tn = t_org + (double)n * dt;
    double th = t_org + ((double)n + 0.5) * dt;
    double te = t_org + ((double)n + 1.0) * dt;
    double x = *px, y = *py, z = is3d ? *pz : 0.0;
    double hd = 0.5 * dt;
    double k1[3], k2[3], k3[3], k4[3];
    double xs, ys, zs;
    const int nn = opt->nearest;

    if (sample_mode(fs, x, y, z, tn, k1, nn))
        goto out_of_bounds;
    if (opt->scheme == 1) { /* Euler forward: one slope at the start of the step */
        xs = x + k1[0] * dt;
        ys = y + k1[1] * dt;
        zs = z + k1[2] * dt;
    } else {
        double x2 = x + k1[0] * hd, y2 = y + k1[1] * hd, z2 = z + k1[2] * hd;
        if (sample_mode(fs, x2, y2, z2, th, k2, nn))
            goto out_of_bounds;
        double x3 = x + k2[0] * hd, y3 = y + k2[1] * hd, z3 = z + k2[2] * hd;
        if (sample_mode(fs, x3, y3, z3, th, k3, nn))
            goto out_of_bounds;
        double x4 = x + k3[0] * dt, y4 = y + k3[1] * dt, z4 = z + k3[2] * dt;
        if (sample_mode(fs, x4, y4, z4, te, k4, nn))
            goto out_of_bounds;
        xs = x + ((((k1[0] + 2.0 * k2[0]) + 2.0 * k3[0]) + k4[0]) * dt) / 6.0;
        ys = y + ((((k1[1] + 2.0 * k2[1]) + 2.0 * k3[1]) + k4[1]) * dt) / 6.0;
        zs = z + ((((k1[2] + 2.0 * k2[2]) + 2.0 * k3[2]) + k4[2]) * dt) / 6.0;
    }
    if (horizontal)
        zs = z;

    if (opt->Kh > 0.0) {
        double nn[2];
        or_normals(opt->run_id, opt->seed, pid, (uint32_t)n, nn);
        /* sigma = sqrt(2 Kh dt) with dt a duration (Sect. 4.2.7): |dt| when running
         * backward in time */
        double sig = sqrt(2.0 * opt->Kh * fabs(dt));
        double dx = sig * nn[0], dy = sig * nn[1];
        if (fs->spherical) {
            dx = dx / (OR_M * cos(ys * OR_D));
            dy = dy / OR_M;
        }
        xs = xs + dx;
        ys = ys + dy;
    }

    or_cell c;
    if (!in_domain(fs, xs, ys, zs, &c))
        goto out_of_bounds;
    if (fs->land && land_cell(fs, c.i, c.j)) {
        *st = (unsigned char)(OR_ST_LAND | err_extra);
        return;
    }
    *px = xs;
    *py = ys;
    if (is3d)
        *pz = zs;
    return;

out_of_bounds:
    *st = (unsigned char)(OR_ST_OOB | err_extra);
}

/* One step of the worked example's kernel chain for one particle: sinking, age,
 * tracer sample (all at the step's start), then the advection. */
static void behave_step(const or_fieldset *fs, const or_options *opt, double t_org, double dt,
                        int64_t n, uint32_t pid, double *px, double *py, double *pz,
                        unsigned char *st, double *temp, double *age)
{
    const unsigned char err_extra = opt->policy == 0 ? OR_ST_DELETED : 0;
    const int is3d = fs->nz > 0;
    const int sinking = is3d && opt->sink_speed > 0.0;
    if (sinking && *pz > opt->dwell_depth) {
        double zn = *pz + opt->sink_speed * dt;
        *pz = zn > opt->dwell_depth ? zn : opt->dwell_depth;
    }
    const int dwelling = !sinking || *pz <= opt->dwell_depth;
    if (opt->maxage > 0.0 && dwelling) {
        *age = *age + fabs(dt);
        if (*age >= opt->maxage) {
            *st = (unsigned char)(OR_ST_AGED | OR_ST_DELETED);
            return;
        }
    }
    if (opt->sample) {
        double v;
        if (or_sample_tracer(fs, *px, *py, is3d ? *pz : 0.0, t_org + (double)n * dt, &v)) {
            *st = (unsigned char)(OR_ST_OOB | err_extra);
            return;
        }
        *temp = v;
    }
    rk4_step(fs, opt, t_org, dt, n, pid, px, py, pz, st, sinking && dwelling);
}

/* Check that every stage time of steps step0 .. step0+nsteps-1 has snapshots. */
static int check_time(const or_fieldset *fs, double t_org, double dt, int64_t step0, int64_t nsteps)
{
    if (fs->nt == 1 || fs->period > 0.0)
        return OR_OK;
    double ta = t_org + (double)step0 * dt;
    double tb = t_org + (double)(step0 + nsteps) * dt;
    double lo = ta < tb ? ta : tb, hi = ta < tb ? tb : ta;
    if (lo < fs->T[0] || hi > fs->T[fs->nt - 1])
        return OR_ETIME;
    return OR_OK;
}

/* Advance n particles through steps step0 .. step0+nsteps-1.  Particles with a
 * nonzero status are not advanced.  *psteps is increased by the number of
 * (particle, step) pairs that started active.  Returns OR_ETIME if the run needs
 * a time outside the snapshots (nothing is changed then). */
int or_advance(const or_fieldset *fs, int64_t n, double *x, double *y, double *z,
               unsigned char *status, const uint32_t *pid, double t_org, double dt,
               int64_t step0, int64_t nsteps, const or_options *opt, int64_t *psteps,
               int nthreads, double *temp, double *age)
{
    const int behave = opt->sample || opt->maxage > 0.0 || (fs->nz > 0 && opt->sink_speed > 0.0);
    if (behave && (!temp || !age || (opt->sample && !fs->tracer)))
        return OR_EINVAL;
    if (dt == 0.0 || nsteps < 0 || n < 0)
        return OR_EINVAL;
    if (check_time(fs, t_org, dt, step0, nsteps) != OR_OK)
        return OR_ETIME;
    int64_t total = 0;
#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(static) num_threads(nthreads) reduction(+ : total)
#endif
    for (int64_t p = 0; p < n; p++) {
        int64_t active = 0;
        for (int64_t q = 0; q < nsteps; q++) {
            if (status[p])
                break;
            active++;
            if (behave)
                behave_step(fs, opt, t_org, dt, step0 + q, pid[p], &x[p], &y[p],
                            z ? &z[p] : NULL, &status[p], &temp[p], &age[p]);
            else
                rk4_step(fs, opt, t_org, dt, step0 + q, pid[p], &x[p], &y[p],
                         z ? &z[p] : NULL, &status[p], 0);
        }
        total += active;
    }
    if (psteps)
        *psteps += total;
    return OR_OK;
}

/* ---------------------------------------------------------------- RKF45 */
/* The Fehlberg 4(5) pair: stage nodes c, stage matrix a (row i uses the slopes
 * before it), fourth-order weights b4 and fifth-order weights b5. */
static const double RKF_C[6] = {0.0, 1.0 / 4.0, 3.0 / 8.0, 12.0 / 13.0, 1.0, 1.0 / 2.0};
static const double RKF_A[6][5] = {
    {0.0, 0.0, 0.0, 0.0, 0.0},
    {1.0 / 4.0, 0.0, 0.0, 0.0, 0.0},
    {3.0 / 32.0, 9.0 / 32.0, 0.0, 0.0, 0.0},
    {1932.0 / 2197.0, -7200.0 / 2197.0, 7296.0 / 2197.0, 0.0, 0.0},
    {439.0 / 216.0, -8.0, 3680.0 / 513.0, -845.0 / 4104.0, 0.0},
    {-8.0 / 27.0, 2.0, -3544.0 / 2565.0, 1859.0 / 4104.0, -11.0 / 40.0}};
static const double RKF_B4[6] = {25.0 / 216.0, 0.0, 1408.0 / 2565.0, 2197.0 / 4104.0,
                                 -1.0 / 5.0, 0.0};
static const double RKF_B5[6] = {16.0 / 135.0, 0.0, 6656.0 / 12825.0, 28561.0 / 56430.0,
                                 -9.0 / 50.0, 2.0 / 55.0};

/* One RKF45 attempt of signed size h from p at time t: the fourth-order end point
 * p4, the fifth-order end point p5 (may be NULL) and the error estimate
 * err = p5 - p4, written as h times the weight differences times the slopes.
 * Returns 1 if a stage point lies outside the grid, 2 outside the snapshots. */
int or_rkf45_attempt(const or_fieldset *fs, int nearest, double t, double h, const double p[3],
                     double p4[3], double p5[3], double err[3])
{
    double k[6][3];
    for (int i = 0; i < 6; i++) {
        double q[3];
        for (int d = 0; d < 3; d++) {
            double s = 0.0;
            for (int j = 0; j < i; j++)
                s = s + RKF_A[i][j] * k[j][d];
            q[d] = p[d] + h * s;
        }
        int rc = sample_mode(fs, q[0], q[1], q[2], t + RKF_C[i] * h, k[i], nearest);
        if (rc)
            return rc;
    }
    for (int d = 0; d < 3; d++) {
        double s4 = 0.0, s5 = 0.0, se = 0.0;
        for (int i = 0; i < 6; i++) {
            s4 = s4 + RKF_B4[i] * k[i][d];
            s5 = s5 + RKF_B5[i] * k[i][d];
            se = se + (RKF_B5[i] - RKF_B4[i]) * k[i][d];
        }
        p4[d] = p[d] + h * s4;
        if (p5)
            p5[d] = p[d] + h * s5;
        err[d] = h * se;
    }
    if (fs->nz <= 0) {
        p4[2] = p[2];
        if (p5)
            p5[2] = p[2];
        err[2] = 0.0;
    }
    return 0;
}

/* Length in metres of a displacement (dx, dy, dz) taken at latitude y. */
double or_metres(const or_fieldset *fs, double y, const double e[3])
{
    double ex = e[0], ey = e[1], ez = e[2];
    if (fs->spherical) {
        ex = ex * (OR_M * cos(y * OR_D));
        ey = ey * OR_M;
    }
    return sqrt((ex * ex + ey * ey) + ez * ez);
}

/* Carry one particle from t_s to t_e (either direction, sign of dt) with adaptive
 * RKF45 steps; *pe is its step exponent.  Counts the attempts that were not
 * retried for accuracy (*acc) and the retried ones (*rej). */
static void rkf45_particle(const or_fieldset *fs, const or_options *opt, double t_s, double t_e,
                           double dt, double *px, double *py, double *pz, unsigned char *st,
                           signed char *pe, int64_t *acc, int64_t *rej)
{
    const int is3d = fs->nz > 0;
    const unsigned char err_extra = opt->policy == 0 ? OR_ST_DELETED : 0;
    const double sg = dt > 0.0 ? 1.0 : -1.0, adt = fabs(dt);
    double p[3] = {*px, *py, is3d ? *pz : 0.0};
    int e = *pe;
    double t = t_s;
    while (t != t_e) {
        const double h = ldexp(adt, e);
        const double rem = sg > 0.0 ? t_e - t : t - t_e;
        const int cut = h >= rem;
        const double hs = sg * (cut ? rem : h);
        double p4[3], ev[3];
        if (or_rkf45_attempt(fs, opt->nearest, t, hs, p, p4, NULL, ev)) {
            (*acc)++;
            *st = (unsigned char)(OR_ST_OOB | err_extra);
            break;
        }
        const double err = or_metres(fs, p[1], ev);
        if (err > opt->tol && e > opt->emin) {
            e--;
            (*rej)++;
            continue;
        }
        (*acc)++;
        or_cell c;
        if (!in_domain(fs, p4[0], p4[1], p4[2], &c)) {
            *st = (unsigned char)(OR_ST_OOB | err_extra);
            break;
        }
        if (fs->land && land_cell(fs, c.i, c.j)) {
            *st = (unsigned char)(OR_ST_LAND | err_extra);
            break;
        }
        p[0] = p4[0];
        p[1] = p4[1];
        p[2] = p4[2];
        t = cut ? t_e : t + hs;
        if (!cut && err <= opt->tol * 0.03125 && e < opt->emax)
            e++;
    }
    *px = p[0];
    *py = p[1];
    if (is3d)
        *pz = p[2];
    *pe = (signed char)e;
}

/* Advance n particles from t_s to t_e with RKF45 (opt->scheme is ignored).  The
 * smallest step |dt| 2^emin must move a time of magnitude max(|t_s|, |t_e|).
 * Returns OR_EINVAL for bad arguments and OR_ETIME if [t_s, t_e] is not covered. */
int or_advance_rkf45(const or_fieldset *fs, int64_t n, double *x, double *y, double *z,
                     unsigned char *status, signed char *exps, double t_s, double t_e,
                     double dt, const or_options *opt, int64_t *accepted, int64_t *rejected,
                     int nthreads)
{
    if (dt == 0.0 || n < 0 || !(opt->tol > 0.0) || opt->emin > 0 || opt->emax < 0 ||
        opt->emin < -30 || opt->emax > 30 || (t_e - t_s) * dt < 0.0)
        return OR_EINVAL;
    const double tm = fabs(t_s) > fabs(t_e) ? fabs(t_s) : fabs(t_e);
    if (tm + ldexp(fabs(dt), opt->emin) * 0.25 == tm && t_s != t_e)
        return OR_EINVAL;
    if (fs->nt > 1 && !(fs->period > 0.0)) {
        const double lo = t_s < t_e ? t_s : t_e, hi = t_s < t_e ? t_e : t_s;
        if (lo < fs->T[0] || hi > fs->T[fs->nt - 1])
            return OR_ETIME;
    }
    int64_t ta = 0, tr = 0;
#ifdef _OPENMP
    if (nthreads <= 0)
        nthreads = omp_get_max_threads();
#pragma omp parallel for schedule(dynamic, 64) num_threads(nthreads) reduction(+ : ta, tr)
#endif
    for (int64_t q = 0; q < n; q++) {
        if (status[q])
            continue;
        int64_t a = 0, r = 0;
        rkf45_particle(fs, opt, t_s, t_e, dt, &x[q], &y[q], z ? &z[q] : NULL, &status[q],
                       &exps[q], &a, &r);
        ta += a;
        tr += r;
    }
    if (accepted)
        *accepted += ta;
    if (rejected)
        *rejected += tr;
    return OR_OK;
}

/* Cell indices (O1 rule) of n positions; -1 on every axis for a point outside. */
void or_cell_indices(const or_fieldset *fs, int64_t n, const double *x, const double *y,
                     const double *z, int32_t *ci, int32_t *cj, int32_t *ck)
{
    for (int64_t p = 0; p < n; p++) {
        or_cell c = {0, 0, 0, 0.0, 0.0, 0.0};
        if (in_domain(fs, x[p], y[p], z ? z[p] : 0.0, &c)) {
            ci[p] = c.i;
            cj[p] = c.j;
            if (ck)
                ck[p] = fs->nz > 0 ? c.k : 0;
        } else {
            ci[p] = -1;
            cj[p] = -1;
            if (ck)
                ck[p] = -1;
        }
    }
}

int or_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
