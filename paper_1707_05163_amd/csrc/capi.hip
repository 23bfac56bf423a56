// capi.hip -- host side of the library: field sets with a ring of device snapshot
// slots, particle sets, and the execute loop that drives the kernels.
//
// The execute loop follows the paper's dynamic update loop (Sect. 2.2): advance
// every particle in steps of dt, write output at every output interval, and turn
// particle errors into recovery actions.  Field snapshots enter through a ring of
// device slots fed on the field set's own stream, the device counterpart of
// keeping three consecutive time slices and calling advancetime (Sect. 3.1,
// Sect. 3.4).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <utility>
#include <vector>

#include "../../include/lp.h"
#include "lp_internal.h"
#include "lp_objects.h"

using lp::AxisDev;
using lp::GridDev;
using lp::TimeEntry;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIPCHECK(expr)                                                                        \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess)                                                                 \
            return fail(e_ == hipErrorOutOfMemory ? LP_ENOMEM : LP_EDEVICE, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                    \
    } while (0)

template <class T>
int dalloc(T **p, size_t count)
{
    *p = nullptr;
    if (count == 0)
        return LP_OK;
    hipError_t e = hipMalloc((void **)p, count * sizeof(T));
    if (e != hipSuccess) {
        *p = nullptr;
        (void)hipGetLastError();
        return fail(LP_ENOMEM, "hipMalloc of %zu bytes failed: %s", count * sizeof(T),
                    hipGetErrorString(e));
    }
    return LP_OK;
}

template <class T>
void dfree(T *&p)
{
    if (p)
        (void)hipFree((void *)p);
    p = nullptr;
}

struct HostAxis {
    std::vector<double> c, rw;
    std::vector<int32_t> guess;
    bool uniform = true;
};

int build_axis(const double *src, int n, const char *name, HostAxis &h)
{
    if (!src || n < 2)
        return fail(LP_EINVAL, "axis %s needs at least 2 coordinates", name);
    h.c.assign(src, src + n);
    for (int i = 0; i + 1 < n; ++i)
        if (!(h.c[i + 1] > h.c[i]))
            return fail(LP_EINVAL, "axis %s is not strictly increasing at %d", name, i);
    h.rw.resize(n - 1);
    for (int i = 0; i + 1 < n; ++i)
        h.rw[i] = 1.0 / (h.c[i + 1] - h.c[i]);
    const double lo = h.c[0], hi = h.c[n - 1], dx = (hi - lo) / (n - 1);
    h.uniform = true;
    for (int i = 0; i < n; ++i)
        if (std::fabs(h.c[i] - (lo + i * dx)) > 0.25 * dx)
            h.uniform = false;
    if (!h.uniform) {
        h.guess.resize(lp::kGuessBins);
        int i = 0;
        for (int b = 0; b < lp::kGuessBins; ++b) {
            const double xb = lo + (hi - lo) * ((double)b / lp::kGuessBins);
            while (i < n - 2 && h.c[i + 1] <= xb)
                ++i;
            h.guess[b] = i;
        }
    }
    return LP_OK;
}

int upload_axis(const HostAxis &h, DevAxis &d, AxisDev &a)
{
    int rc;
    if ((rc = dalloc(&d.c, h.c.size())) || (rc = dalloc(&d.rw, h.rw.size())))
        return rc;
    HIPCHECK(hipMemcpy(d.c, h.c.data(), h.c.size() * sizeof(double), hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(d.rw, h.rw.data(), h.rw.size() * sizeof(double), hipMemcpyHostToDevice));
    if (!h.uniform) {
        if ((rc = dalloc(&d.guess, h.guess.size())))
            return rc;
        HIPCHECK(hipMemcpy(d.guess, h.guess.data(), h.guess.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice));
    }
    a.c = d.c;
    a.rw = d.rw;
    a.guess = d.guess;
    a.n = (int32_t)h.c.size();
    a.lo = h.c.front();
    a.hi = h.c.back();
    a.uniform = h.uniform ? 1 : 0;
    a.ginv = h.uniform ? (double)(a.n - 1) / (a.hi - a.lo) : (double)lp::kGuessBins / (a.hi - a.lo);
    return LP_OK;
}

void free_axis(DevAxis &d)
{
    dfree(d.c);
    dfree(d.rw);
    dfree(d.guess);
}

size_t node_bytes(int dtype, bool is3d)
{
    switch (dtype) {
    case LP_F64: return is3d ? 32 : 16;
    case LP_F32: return is3d ? 16 : 8;
    default: return is3d ? 8 : 4;
    }
}

}  // namespace

// ---------------------------------------------------------------- field sets
extern "C" int fieldset_create(const lp_grid_desc *g, lp_fieldset **out)
{
    if (!g || !out)
        return fail(LP_EINVAL, "null argument");
    *out = nullptr;
    if (g->nx < 2 || g->ny < 2 || (g->nz != 0 && g->nz < 2))
        return fail(LP_EINVAL, "grid needs nx, ny >= 2 and nz == 0 or >= 2");
    if (g->dtype < LP_F64 || g->dtype > LP_F16_SCALED)
        return fail(LP_EINVAL, "unknown dtype %d", g->dtype);
    if (g->mesh != LP_MESH_FLAT && g->mesh != LP_MESH_SPHERICAL)
        return fail(LP_EINVAL, "unknown mesh %d", g->mesh);
    if (g->capacity < 1)
        return fail(LP_EINVAL, "capacity must be >= 1");
    if (!(g->time_period >= 0.0))
        return fail(LP_EINVAL, "time_period must be >= 0");
    if (g->nz >= 2 && !g->depth)
        return fail(LP_EINVAL, "3D grid needs depth levels");
    if ((size_t)g->nx * g->ny > 0x7FFFFFFFull)
        return fail(LP_EINVAL, "too many horizontal nodes");
    HostAxis hx, hy, hz;
    int rc;
    if ((rc = build_axis(g->lon, g->nx, "lon", hx)) || (rc = build_axis(g->lat, g->ny, "lat", hy)))
        return rc;
    if (g->nz >= 2 && (rc = build_axis(g->depth, g->nz, "depth", hz)))
        return rc;

    lp_fieldset *fs = new lp_fieldset();
    auto bail = [&](int code) {
        fieldset_destroy(fs);
        return code;
    };
    (void)hipGetDevice(&fs->device);
    fs->nx = g->nx;
    fs->ny = g->ny;
    fs->nz = g->nz;
    fs->is3d = g->nz >= 2;
    fs->nzl = fs->is3d ? g->nz : 1;
    fs->mesh = g->mesh;
    fs->dtype = g->dtype;
    fs->capacity = g->capacity;
    fs->period = g->time_period;
    if ((rc = upload_axis(hx, fs->dx_, fs->g.ax)) || (rc = upload_axis(hy, fs->dy_, fs->g.ay)))
        return bail(rc);
    if (fs->is3d && (rc = upload_axis(hz, fs->dz_, fs->g.az)))
        return bail(rc);
    fs->g.spherical = g->mesh == LP_MESH_SPHERICAL;
    if (fs->g.spherical) {
        double tallest = 0.0;
        for (int j = 0; j + 1 < g->ny; ++j)
            tallest = std::max(tallest, g->lat[j + 1] - g->lat[j]);
        if (tallest <= 5.0) {  // cos(lat) from per-node tables plus a short series
            if ((rc = dalloc(&fs->dcoslat, (size_t)g->ny)) ||
                (rc = dalloc(&fs->dsinlat, (size_t)g->ny)))
                return bail(rc);
            if (lp::launch_lat_tables(fs->g.ay.c, g->ny, fs->dcoslat, fs->dsinlat, nullptr) !=
                    hipSuccess ||
                hipDeviceSynchronize() != hipSuccess)
                return bail(fail(LP_EDEVICE, "latitude table kernel failed"));
            fs->g.coslat = fs->dcoslat;
            fs->g.sinlat = fs->dsinlat;
            // truncation of the series below a quarter ulp for the tallest cell
            fs->g.cos_terms = tallest <= 0.3 ? 2 : (tallest <= 1.5 ? 3 : 4);
        }
    }
    if (g->land) {
        std::vector<uint8_t> cell((size_t)(g->ny - 1) * (g->nx - 1));
        const size_t nx = g->nx;
        for (int j = 0; j + 1 < g->ny; ++j)
            for (int i = 0; i + 1 < g->nx; ++i)
                cell[(size_t)j * (nx - 1) + i] =
                    (g->land[j * nx + i] && g->land[j * nx + i + 1] && g->land[(j + 1) * nx + i] &&
                     g->land[(j + 1) * nx + i + 1])
                        ? 1
                        : 0;
        if ((rc = dalloc(&fs->dland, cell.size())))
            return bail(rc);
        if (hipMemcpy(fs->dland, cell.data(), cell.size(), hipMemcpyHostToDevice) != hipSuccess)
            return bail(fail(LP_EDEVICE, "land mask upload failed"));
        fs->g.landcell = fs->dland;
        if ((rc = dalloc(&fs->dlandnode, (size_t)g->nx * g->ny)))
            return bail(rc);
        if (hipMemcpy(fs->dlandnode, g->land, (size_t)g->nx * g->ny, hipMemcpyHostToDevice) !=
            hipSuccess)
            return bail(fail(LP_EDEVICE, "land mask upload failed"));
    }
    fs->slot_bytes = node_bytes(fs->dtype, fs->is3d) * fs->plane() * fs->nzl;
    fs->slot_bytes = (fs->slot_bytes + 255) & ~(size_t)255;
    if ((rc = dalloc(&fs->dslots, fs->slot_bytes * fs->capacity)))
        return bail(rc);
    if ((rc = dalloc(&fs->dscales, (size_t)fs->capacity * fs->nzl * 3)) ||
        (rc = dalloc(&fs->dtmp, (size_t)fs->nzl * 3)))
        return bail(rc);
    if (hipStreamCreateWithFlags(&fs->up, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(LP_EDEVICE, "stream creation failed"));
    fs->ready.resize(fs->capacity);
    fs->release.resize(fs->capacity);
    for (int s = 0; s < fs->capacity; ++s) {
        if (hipEventCreateWithFlags(&fs->ready[s], hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&fs->release[s], hipEventDisableTiming) != hipSuccess)
            return bail(fail(LP_EDEVICE, "event creation failed"));
    }
    fs->slot_t.assign(fs->capacity, 0.0);
    fs->slot_seq.assign(fs->capacity, -1);
    fs->tracer_seq.assign(fs->capacity, -1);
    *out = fs;
    return LP_OK;
}

extern "C" void fieldset_destroy(lp_fieldset *fs)
{
    if (!fs)
        return;
    if (fs->up)
        (void)hipStreamSynchronize(fs->up);
    free_axis(fs->dx_);
    free_axis(fs->dy_);
    free_axis(fs->dz_);
    dfree(fs->dland);
    dfree(fs->dlandnode);
    dfree(fs->dcoslat);
    dfree(fs->dsinlat);
    dfree(fs->dslots);
    dfree(fs->dscales);
    dfree(fs->dtracer);
    dfree(fs->dtmp);
    dfree(fs->dstage);
    dfree(fs->dstage64);
    if (fs->hpin)
        (void)hipHostFree(fs->hpin);
    for (auto e : fs->pin_ev)
        if (e) (void)hipEventDestroy(e);
    if (fs->src_done)
        (void)hipEventDestroy(fs->src_done);
    for (auto e : fs->ready)
        if (e) (void)hipEventDestroy(e);
    for (auto e : fs->release)
        if (e) (void)hipEventDestroy(e);
    if (fs->up)
        (void)hipStreamDestroy(fs->up);
    delete fs;
}

namespace {

constexpr size_t kPinChunk = (size_t)256 << 20;  // bytes per pinned staging chunk

// memcpy on several host threads (large copies only; one thread below 32 MiB)
void parallel_copy(char *dst, const char *src, size_t len)
{
    const size_t per = (size_t)16 << 20;
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t nt = std::min<size_t>(std::min<size_t>(8, hw), std::max<size_t>(1, len / per));
    if (nt <= 1) {
        std::memcpy(dst, src, len);
        return;
    }
    std::vector<std::thread> th;
    const size_t step = (len + nt - 1) / nt;
    for (size_t t = 1; t < nt; ++t) {
        const size_t a = t * step, b = std::min(len, a + step);
        if (a < b)
            th.emplace_back([=] { std::memcpy(dst + a, src + a, b - a); });
    }
    std::memcpy(dst, src, std::min(len, step));
    for (auto &x : th)
        x.join();
}

// Host arrays src[0..nvar) of `bytes` each into consecutive device staging at dst, on
// the field set's upload stream, through two pinned chunks: a chunk is refilled by
// the host only after its previous host-to-device copy has finished, so the host
// copy of one chunk overlaps the DMA of the other.  Returns once the last chunk is
// queued; the host arrays are not read after that, the DMAs run on.
int upload_from_host(lp_fieldset *fs, const void *const *src, int nvar, size_t bytes, char *dst)
{
    if (!fs->hpin) {
        const size_t chunk = std::min(kPinChunk, (bytes + 4095) & ~(size_t)4095);
        if (hipHostMalloc((void **)&fs->hpin, 2 * chunk, hipHostMallocDefault) != hipSuccess) {
            fs->hpin = nullptr;
            (void)hipGetLastError();
            return fail(LP_ENOMEM, "pinned staging of %zu bytes failed", 2 * chunk);
        }
        fs->pin_chunk = chunk;
        for (auto &e : fs->pin_ev)
            if (!e)
                HIPCHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    }
    const size_t chunk = fs->pin_chunk;
    int k = fs->pin_next;
    for (int q = 0; q < nvar; ++q)
        for (size_t off = 0; off < bytes; off += chunk) {
            const size_t len = std::min(chunk, bytes - off);
            if (fs->pin_pending[k]) {  // its previous DMA must have read the chunk
                HIPCHECK(hipEventSynchronize(fs->pin_ev[k]));
                fs->pin_pending[k] = false;
            }
            char *buf = fs->hpin + (size_t)k * chunk;
            parallel_copy(buf, (const char *)src[q] + off, len);
            HIPCHECK(hipMemcpyAsync(dst + (size_t)q * bytes + off, buf, len,
                                    hipMemcpyHostToDevice, fs->up));
            HIPCHECK(hipEventRecord(fs->pin_ev[k], fs->up));
            fs->pin_pending[k] = true;
            k ^= 1;
        }
    fs->pin_next = k;
    return LP_OK;
}

}  // namespace

static int push_common(lp_fieldset *fs, double t, const void *U, const void *V, const void *W,
                       bool device_src, bool f64, void *stream)
{
    if (!fs || !U || !V || (fs->is3d && !W))
        return fail(LP_EINVAL, "null field pointer");
    if (f64 && fs->dtype != LP_F64)
        return fail(LP_EINVAL, "double snapshots need LP_F64 storage");
    if (!std::isfinite(t))
        return fail(LP_EINVAL, "snapshot time is not finite");
    if (fs->npushed > 0 && !(t > fs->last_t))
        return fail(LP_EINVAL, "snapshot times must increase (%g after %g)", t, fs->last_t);
    if (fs->period > 0.0) {
        if (fs->npushed >= fs->capacity)
            return fail(LP_ESTATE, "a periodic field set keeps every snapshot resident: "
                                   "capacity %d is full", fs->capacity);
        if (fs->npushed > 0 && !(t < fs->first_t + fs->period))
            return fail(LP_EINVAL, "snapshot time beyond one period");
    }
    const int slot = (int)(fs->npushed % fs->capacity);
    const size_t nvals = fs->plane() * fs->nzl;
    const int nvar = fs->is3d ? 3 : 2;
    int rc;
    // float arrays in device memory are converted where they are; everything else goes
    // through the device staging buffer
    const bool direct = device_src && !f64;
    if (f64) {
        if (!fs->dstage64 && (rc = dalloc(&fs->dstage64, nvals * 3)))
            return rc;
    } else if (!direct && !fs->dstage && (rc = dalloc(&fs->dstage, nvals * 3))) {
        return rc;
    }
    if (stream) {
        hipEvent_t ev;
        HIPCHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIPCHECK(hipEventRecord(ev, (hipStream_t)stream));
        HIPCHECK(hipStreamWaitEvent(fs->up, ev, 0));
        HIPCHECK(hipEventDestroy(ev));
    }
    // kernels that still read the slot must finish before it is overwritten
    HIPCHECK(hipStreamWaitEvent(fs->up, fs->release[slot], 0));
    const void *src[3] = {U, V, W};
    const size_t esz = f64 ? sizeof(double) : sizeof(float);
    char *dst = f64 ? (char *)fs->dstage64 : (char *)fs->dstage;
    if (device_src && !direct) {
        for (int q = 0; q < nvar; ++q)
            HIPCHECK(hipMemcpyAsync(dst + (size_t)q * nvals * esz, src[q], nvals * esz,
                                    hipMemcpyDeviceToDevice, fs->up));
    } else if (!device_src && (rc = upload_from_host(fs, src, nvar, nvals * esz, dst))) {
        return rc;
    }
    char *slotp = fs->dslots + (size_t)slot * fs->slot_bytes;
    float *scales = fs->dscales + (size_t)slot * fs->nzl * 3;
    const float *fsrc = direct ? (const float *)U : fs->dstage;
    const float *fv = direct ? (const float *)V : fs->dstage + nvals;
    const float *fw = direct ? (const float *)W : (fs->is3d ? fs->dstage + 2 * nvals : nullptr);
    hipError_t e;
    if (f64)
        e = lp::launch_convert_snapshot(fs->dtype, fs->is3d, nullptr, nullptr, nullptr,
                                        fs->dstage64, fs->dstage64 + nvals,
                                        fs->is3d ? fs->dstage64 + 2 * nvals : nullptr,
                                        fs->plane(), fs->nzl, slotp, scales, fs->dtmp, fs->up);
    else
        e = lp::launch_convert_snapshot(fs->dtype, fs->is3d, fsrc, fv, fs->is3d ? fw : nullptr,
                                        nullptr, nullptr, nullptr, fs->plane(), fs->nzl, slotp,
                                        scales, fs->dtmp, fs->up);
    HIPCHECK(e);
    HIPCHECK(hipEventRecord(fs->ready[slot], fs->up));
    if (device_src && stream) {
        // work the caller queues on `stream` later may reuse the source arrays: it runs
        // after the upload stream has read them (the copy, or the conversion itself)
        HIPCHECK(hipStreamWaitEvent((hipStream_t)stream, fs->ready[slot], 0));
    }
    if (fs->npushed == 0)
        fs->first_t = t;
    fs->slot_t[slot] = t;
    fs->slot_seq[slot] = fs->npushed;
    fs->npushed++;
    fs->last_t = t;
    return LP_OK;
}

extern "C" int fieldset_push_snapshot(lp_fieldset *fs, double t, const float *U, const float *V,
                                      const float *W, void *stream)
{
    return push_common(fs, t, U, V, W, false, false, stream);
}

extern "C" int fieldset_push_snapshot_f64(lp_fieldset *fs, double t, const double *U,
                                          const double *V, const double *W, void *stream)
{
    return push_common(fs, t, U, V, W, false, true, stream);
}

extern "C" int fieldset_push_snapshot_device(lp_fieldset *fs, double t, const float *dU,
                                             const float *dV, const float *dW, void *stream)
{
    return push_common(fs, t, dU, dV, dW, true, false, stream);
}

static int push_tracer(lp_fieldset *fs, double t, const float *T, bool device_src, void *stream)
{
    if (!fs || !T)
        return fail(LP_EINVAL, "null argument");
    int slot = -1;
    for (int s = 0; s < fs->capacity; ++s)
        if (fs->slot_seq[s] >= 0 && fs->slot_t[s] == t)
            slot = s;
    if (slot < 0)
        return fail(LP_ESTATE, "no resident snapshot has time %.17g", t);
    const size_t nvals = fs->plane() * fs->nzl;
    int rc;
    if (!fs->dtracer && (rc = dalloc(&fs->dtracer, nvals * (size_t)fs->capacity)))
        return rc;
    if (stream) {
        hipEvent_t ev;
        HIPCHECK(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        HIPCHECK(hipEventRecord(ev, (hipStream_t)stream));
        HIPCHECK(hipStreamWaitEvent(fs->up, ev, 0));
        HIPCHECK(hipEventDestroy(ev));
    }
    HIPCHECK(hipStreamWaitEvent(fs->up, fs->release[slot], 0));
    HIPCHECK(hipMemcpyAsync(fs->dtracer + (size_t)slot * nvals, T, nvals * sizeof(float),
                            device_src ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                            fs->up));
    // kernels that read this slot wait for `ready`, which now covers the tracer too
    HIPCHECK(hipEventRecord(fs->ready[slot], fs->up));
    if (!device_src)
        HIPCHECK(hipStreamSynchronize(fs->up));
    fs->tracer_seq[slot] = fs->slot_seq[slot];
    return LP_OK;
}

extern "C" int fieldset_push_tracer(lp_fieldset *fs, double t, const float *T, void *stream)
{
    return push_tracer(fs, t, T, false, stream);
}

extern "C" int fieldset_push_tracer_device(lp_fieldset *fs, double t, const float *dT,
                                          void *stream)
{
    return push_tracer(fs, t, dT, true, stream);
}

namespace {

struct Resident {
    double t;
    int slot;
};

std::vector<Resident> resident(const lp_fieldset *fs)
{
    std::vector<Resident> r;
    for (int s = 0; s < fs->capacity; ++s)
        if (fs->slot_seq[s] >= 0)
            r.push_back({fs->slot_t[s], s});
    std::sort(r.begin(), r.end(), [](const Resident &a, const Resident &b) { return a.t < b.t; });
    return r;
}

// Bracket of time t among the resident snapshots: linear weight tau between
// slot sa (earlier) and sb (later).
int bracket(const lp_fieldset *fs, const std::vector<Resident> &r, double t, TimeEntry &e)
{
    const int m = (int)r.size();
    if (m == 0)
        return fail(LP_ETIME, "no snapshot has been pushed");
    if (m == 1 && fs->npushed == 1) {  // steady field
        e.tau = 0.0;
        e.sa = e.sb = r[0].slot;
        return LP_OK;
    }
    if (fs->period > 0.0) {
        const double T0 = r[0].t;
        double q = std::fmod(t - T0, fs->period);
        if (q < 0.0)
            q += fs->period;
        const double tp = T0 + q;
        int s = 0;
        for (int k = 0; k < m; ++k)
            if (r[k].t <= tp)
                s = k;
        const double tn = (s + 1 < m) ? r[s + 1].t : T0 + fs->period;
        e.sa = r[s].slot;
        e.sb = (s + 1 < m) ? r[s + 1].slot : r[0].slot;
        e.tau = (tp - r[s].t) / (tn - r[s].t);
        return LP_OK;
    }
    if (!(t >= r[0].t && t <= r[m - 1].t) || m < 2)
        return fail(LP_ETIME, "time %.17g is not covered by the resident snapshots [%.17g, %.17g]",
                    t, r[0].t, r[m - 1].t);
    int s = 0;
    for (int k = 0; k + 1 < m; ++k)
        if (r[k].t <= t)
            s = k;
    e.sa = r[s].slot;
    e.sb = r[s + 1].slot;
    e.tau = (t - r[s].t) / (r[s + 1].t - r[s].t);
    return LP_OK;
}

}  // namespace

extern "C" int fieldset_get_snapshot(lp_fieldset *fs, double t, float *U, float *V, float *W)
{
    if (!fs || !U || !V)
        return fail(LP_EINVAL, "null argument");
    int slot = -1;
    for (int s = 0; s < fs->capacity; ++s)
        if (fs->slot_seq[s] >= 0 && fs->slot_t[s] == t)
            slot = s;
    if (slot < 0)
        return fail(LP_ETIME, "no resident snapshot at time %.17g", t);
    const size_t nvals = fs->plane() * fs->nzl;
    float *d = nullptr;
    int rc = dalloc(&d, nvals * 3);
    if (rc)
        return rc;
    HIPCHECK(hipStreamSynchronize(fs->up));
    hipError_t e = lp::launch_slot_values(fs->dtype, fs->is3d, fs->dslots + (size_t)slot * fs->slot_bytes,
                                          fs->dscales + (size_t)slot * fs->nzl * 3, fs->plane(),
                                          fs->nzl, d, d + nvals, fs->is3d ? d + 2 * nvals : nullptr,
                                          nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpy(U, d, nvals * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess) e = hipMemcpy(V, d + nvals, nvals * 4, hipMemcpyDeviceToHost);
    if (e == hipSuccess && W && fs->is3d) e = hipMemcpy(W, d + 2 * nvals, nvals * 4, hipMemcpyDeviceToHost);
    dfree(d);
    HIPCHECK(e);
    return LP_OK;
}

extern "C" int lp_philox_normals(uint32_t run_id, uint32_t seed, int64_t n, const uint32_t *pid,
                                 const uint32_t *step, uint32_t *words, double *normals)
{
    if (n < 0 || (n > 0 && (!pid || !step)))
        return fail(LP_EINVAL, "bad arguments");
    if (n == 0)
        return LP_OK;
    uint32_t *dp = nullptr, *dsn = nullptr, *dw = nullptr;
    double *dn = nullptr;
    int rc;
    if ((rc = dalloc(&dp, (size_t)n)) || (rc = dalloc(&dsn, (size_t)n)) ||
        (rc = dalloc(&dw, 4 * (size_t)n)) || (rc = dalloc(&dn, 2 * (size_t)n))) {
        dfree(dp); dfree(dsn); dfree(dw); dfree(dn);
        return rc;
    }
    hipError_t e = hipMemcpy(dp, pid, (size_t)n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(dsn, step, (size_t)n * 4, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = lp::launch_philox_normals(run_id, seed, n, dp, dsn, dw, dn, nullptr);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e == hipSuccess && words) e = hipMemcpy(words, dw, (size_t)n * 16, hipMemcpyDeviceToHost);
    if (e == hipSuccess && normals) e = hipMemcpy(normals, dn, (size_t)n * 16, hipMemcpyDeviceToHost);
    dfree(dp); dfree(dsn); dfree(dw); dfree(dn);
    HIPCHECK(e);
    return LP_OK;
}

extern "C" int fieldset_resident(const lp_fieldset *fs, int32_t *count, double *times)
{
    if (!fs || !count)
        return fail(LP_EINVAL, "null argument");
    auto r = resident(fs);
    *count = (int32_t)r.size();
    if (times)
        for (size_t k = 0; k < r.size(); ++k)
            times[k] = r[k].t;
    return LP_OK;
}

// ---------------------------------------------------------------- particle sets
extern "C" void pset_destroy(lp_pset *ps)
{
    if (!ps)
        return;
    (void)hipDeviceSynchronize();
    dfree(ps->dx);
    dfree(ps->dy);
    dfree(ps->dz);
    dfree(ps->dst);
    dfree(ps->dorder[0]);
    dfree(ps->dorder[1]);
    dfree(ps->dcount);
    dfree(ps->dkeys);
    dfree(ps->dhist);
    dfree(ps->dblk);
    dfree(ps->dpsteps);
    dfree(ps->dexp);
    dfree(ps->dtemp);
    dfree(ps->dage);
    dfree(ps->rtemp);
    dfree(ps->rage);
    dfree(ps->dqueues);
    dfree(ps->dres);
    dfree(ps->rx);
    dfree(ps->ry);
    dfree(ps->rz);
    dfree(ps->rst);
    dfree(ps->rci);
    dfree(ps->rcj);
    dfree(ps->rck);
    dfree(ps->dtab);
    if (ps->htab)
        (void)hipHostFree(ps->htab);
    if (ps->hcount)
        (void)hipHostFree(ps->hcount);
    if (ps->tab_ev)
        (void)hipEventDestroy(ps->tab_ev);
    if (ps->count_ev)
        (void)hipEventDestroy(ps->count_ev);
    for (auto &p : ps->prof) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    delete ps;
}

static int pset_create_common(lp_fieldset *fs, int64_t n, const double *lon, const double *lat,
                              const double *depth, double t0, int64_t step0, bool device_src,
                              hipStream_t stream, lp_pset **out)
{
    if (!fs || !out)
        return fail(LP_EINVAL, "null argument");
    *out = nullptr;
    if (n < 1 || n > 0x7FFFFFFFll)
        return fail(LP_EINVAL, "particle count %lld out of range [1, 2^31)", (long long)n);
    if (!lon || !lat || (fs->is3d && !depth))
        return fail(LP_EINVAL, "null position array");
    if (!std::isfinite(t0) || step0 < 0)
        return fail(LP_EINVAL, "bad start time or step");
    lp_pset *ps = new lp_pset();
    auto bail = [&](int code) {
        pset_destroy(ps);
        return code;
    };
    ps->fs = fs;
    ps->n = n;
    ps->t0 = t0;
    ps->step = step0;
    int rc;
    const size_t N = (size_t)n;
    if ((rc = dalloc(&ps->dx, N)) || (rc = dalloc(&ps->dy, N)) ||
        (fs->is3d && (rc = dalloc(&ps->dz, N))) || (rc = dalloc(&ps->dst, N)) ||
        (rc = dalloc(&ps->dorder[0], N)) || (rc = dalloc(&ps->dorder[1], N)) ||
        (rc = dalloc(&ps->dcount, 2)) || (rc = dalloc(&ps->dpsteps, 2 * lp::kCountWords)) ||
        (rc = dalloc(&ps->dexp, N)) || (rc = dalloc(&ps->dqueues, 8)) ||
        (rc = dalloc(&ps->dtemp, N)) || (rc = dalloc(&ps->dage, N)))
        return bail(rc);
    ps->nbins = lp::sort_bins(fs->g);
    if ((rc = dalloc(&ps->dkeys, N)) || (rc = dalloc(&ps->dhist, ps->nbins)) ||
        (rc = dalloc(&ps->dblk, lp::sort_blocksums(ps->nbins))))
        return bail(rc);
    if (hipHostMalloc((void **)&ps->hcount, sizeof(uint32_t), hipHostMallocDefault) != hipSuccess)
        return bail(fail(LP_ENOMEM, "pinned allocation failed"));
    if (hipEventCreateWithFlags(&ps->tab_ev, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&ps->count_ev, hipEventDisableTiming) != hipSuccess)
        return bail(fail(LP_EDEVICE, "event creation failed"));
    const hipMemcpyKind kind = device_src ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    auto cp = [&](double *dst, const double *src) {
        return hipMemcpyAsync(dst, src, N * sizeof(double), kind, stream);
    };
    if (cp(ps->dx, lon) != hipSuccess || cp(ps->dy, lat) != hipSuccess ||
        (fs->is3d && cp(ps->dz, depth) != hipSuccess))
        return bail(fail(LP_EDEVICE, "particle upload failed"));
    if (hipMemsetAsync(ps->dst, 0, N, stream) != hipSuccess ||
        hipMemsetAsync(ps->dpsteps, 0, 2 * lp::kCountWords * sizeof(unsigned long long),
                       stream) != hipSuccess ||
        hipMemsetAsync(ps->dexp, 0, N, stream) != hipSuccess ||
        hipMemsetAsync(ps->dtemp, 0xFF, N * sizeof(double), stream) != hipSuccess ||  // NaN
        hipMemsetAsync(ps->dage, 0, N * sizeof(double), stream) != hipSuccess ||
        lp::launch_iota(ps->dorder[0], N, stream) != hipSuccess ||
        lp::launch_fill_u32(ps->dcount, (uint32_t)n, 1, stream) != hipSuccess)
        return bail(fail(LP_EDEVICE, "particle set initialisation failed"));
    if (!device_src && hipStreamSynchronize(stream) != hipSuccess)
        return bail(fail(LP_EDEVICE, "particle upload failed"));
    ps->n_launch = (uint32_t)n;
    ps->last_stream = stream;
    *out = ps;
    return LP_OK;
}

extern "C" int pset_create(lp_fieldset *fs, int64_t n, const double *lon, const double *lat,
                           const double *depth, double t0, int64_t step0, lp_pset **out)
{
    return pset_create_common(fs, n, lon, lat, depth, t0, step0, false, nullptr, out);
}

extern "C" int pset_create_device(lp_fieldset *fs, int64_t n, const double *dlon,
                                  const double *dlat, const double *ddepth, double t0,
                                  int64_t step0, void *stream, lp_pset **out)
{
    return pset_create_common(fs, n, dlon, dlat, ddepth, t0, step0, true, (hipStream_t)stream,
                              out);
}

namespace {

int grow_records(lp_pset *ps, int64_t need)
{
    if (need <= ps->rec_cap && (!ps->behave_records || ps->rtemp))
        return LP_OK;
    int64_t cap = std::max<int64_t>(need, std::max<int64_t>(4, ps->rec_cap * 2));
    const size_t old = (size_t)(ps->nrec * ps->nper), tot = (size_t)(cap * ps->nper);
    const bool is3d = ps->fs->is3d;
    double *rx, *ry, *rz = nullptr;
    uint8_t *rst;
    int32_t *ci, *cj, *ck = nullptr;
    int rc;
    if ((rc = dalloc(&rx, tot)) || (rc = dalloc(&ry, tot)) || (is3d && (rc = dalloc(&rz, tot))) ||
        (rc = dalloc(&rst, tot)) || (rc = dalloc(&ci, tot)) || (rc = dalloc(&cj, tot)) ||
        (is3d && (rc = dalloc(&ck, tot))))
        return rc;
    if (old) {
        HIPCHECK(hipMemcpy(rx, ps->rx, old * 8, hipMemcpyDeviceToDevice));
        HIPCHECK(hipMemcpy(ry, ps->ry, old * 8, hipMemcpyDeviceToDevice));
        if (is3d)
            HIPCHECK(hipMemcpy(rz, ps->rz, old * 8, hipMemcpyDeviceToDevice));
        HIPCHECK(hipMemcpy(rst, ps->rst, old, hipMemcpyDeviceToDevice));
        HIPCHECK(hipMemcpy(ci, ps->rci, old * 4, hipMemcpyDeviceToDevice));
        HIPCHECK(hipMemcpy(cj, ps->rcj, old * 4, hipMemcpyDeviceToDevice));
        if (is3d)
            HIPCHECK(hipMemcpy(ck, ps->rck, old * 4, hipMemcpyDeviceToDevice));
    }
    dfree(ps->rx);
    dfree(ps->ry);
    dfree(ps->rz);
    dfree(ps->rst);
    dfree(ps->rci);
    dfree(ps->rcj);
    dfree(ps->rck);
    if (ps->behave_records) {
        double *rt = nullptr, *ra = nullptr;
        if ((rc = dalloc(&rt, tot)) || (rc = dalloc(&ra, tot))) {
            dfree(rt);
            return rc;
        }
        if (old && ps->rtemp) {
            HIPCHECK(hipMemcpy(rt, ps->rtemp, old * 8, hipMemcpyDeviceToDevice));
            HIPCHECK(hipMemcpy(ra, ps->rage, old * 8, hipMemcpyDeviceToDevice));
        } else if (old) {  // records taken before any worked-example kernel ran
            HIPCHECK(hipMemset(rt, 0xFF, old * 8));
            HIPCHECK(hipMemset(ra, 0, old * 8));
        }
        dfree(ps->rtemp);
        dfree(ps->rage);
        ps->rtemp = rt;
        ps->rage = ra;
    }
    ps->rx = rx;
    ps->ry = ry;
    ps->rz = rz;
    ps->rst = rst;
    ps->rci = ci;
    ps->rcj = cj;
    ps->rck = ck;
    ps->rec_cap = cap;
    return LP_OK;
}

int take_record(lp_pset *ps, hipStream_t s)
{
    lp::RecordParams R{};
    R.g = ps->fs->g;
    R.x = ps->dx;
    R.y = ps->dy;
    R.z = ps->dz;
    R.status = ps->dst;
    R.n = ps->n;
    R.stride = ps->stride;
    R.nper = ps->nper;
    const size_t off = (size_t)(ps->nrec * ps->nper);
    R.rx = ps->rx + off;
    R.ry = ps->ry + off;
    R.rz = ps->fs->is3d ? ps->rz + off : nullptr;
    R.rst = ps->rst + off;
    R.ci = ps->rci + off;
    R.cj = ps->rcj + off;
    R.ck = ps->fs->is3d ? ps->rck + off : nullptr;
    if (ps->rtemp) {
        R.temp = ps->dtemp;
        R.age = ps->dage;
        R.rtemp = ps->rtemp + off;
        R.rage = ps->rage + off;
    }
    HIPCHECK(lp::launch_record(R, s));
    ps->nrec++;
    return LP_OK;
}

}  // namespace

namespace {

// One execute call split into its output segments.
struct ExecPlan {
    int64_t nsteps = 0, per = 0;
    std::vector<std::pair<int64_t, int64_t>> segs;  // launches: (first step, steps)
    std::vector<char> seg_end;                      // the launch ends an output segment
    std::vector<char> used;                         // snapshot slots read
    lp::AdvectParams P{};                           // per-call part of the kernel arguments
    size_t toff = 0;                                // time-table offset of the next segment
    bool records = false;
};

// Validate, rebase the time origin, build and upload the stage-time table, order
// the stream after the snapshot uploads and take the first record.  Nothing is
// launched if a stage time is not covered (LP_ETIME) or an argument is bad.
int exec_prepare(lp_pset *ps, double runtime, double dt, double outputdt, const lp_exec_opts *o,
                 hipStream_t stream, bool allow_records, ExecPlan &plan)
{
    if (!ps || !o)
        return fail(LP_EINVAL, "null argument");
    lp_fieldset *fs = ps->fs;
    if (o->kernel != LP_KERNEL_RK4 && o->kernel != LP_KERNEL_EULER &&
        o->kernel != LP_KERNEL_RKF45)
        return fail(LP_EINVAL, "unknown kernel %d", o->kernel);
    const bool rkf = o->kernel == LP_KERNEL_RKF45;
    if (rkf && (!(o->rkf_tol > 0.0) || !std::isfinite(o->rkf_tol) || o->rkf_min_exp > 0 ||
                o->rkf_min_exp < -30 || o->rkf_max_exp < 0 || o->rkf_max_exp > 30))
        return fail(LP_EINVAL, "RKF45 needs rkf_tol > 0, rkf_min_exp in [-30, 0] and "
                               "rkf_max_exp in [0, 30]");
    if (rkf && o->Kh != 0.0)
        return fail(LP_EINVAL, "RKF45 takes no Brownian term (Kh must be 0)");
    if (!(o->sink_speed >= 0.0) || !std::isfinite(o->sink_speed) || !(o->maxage >= 0.0) ||
        !std::isfinite(o->maxage) || !std::isfinite(o->dwell_depth))
        return fail(LP_EINVAL, "sink_speed and maxage must be finite and >= 0");
    if (o->sink_speed > 0.0 && !fs->is3d)
        return fail(LP_EINVAL, "sinking needs a 3D field set");
    const bool behave = o->sample_tracer || o->maxage > 0.0 || o->sink_speed > 0.0;
    if (behave && rkf)
        return fail(LP_EINVAL, "the worked-example kernels run with RK4 or Euler, not RKF45");
    if (o->interp != LP_INTERP_LINEAR && o->interp != LP_INTERP_NEAREST)
        return fail(LP_EINVAL, "unknown interpolation %d", o->interp);
    if (o->recovery != LP_DELETE && o->recovery != LP_FREEZE)
        return fail(LP_EINVAL, "unknown recovery policy %d", o->recovery);
    if (dt == 0.0 || !std::isfinite(dt))
        return fail(LP_EINVAL, "dt must be nonzero and finite");
    const double adt = std::fabs(dt);
    if (!(runtime >= 0.0) || !std::isfinite(runtime) || !(outputdt >= 0.0))
        return fail(LP_EINVAL, "runtime and outputdt must be >= 0");
    if (!(o->Kh >= 0.0) || o->output_stride < 0 || o->sort_every < 0 || o->sort_steps < 0)
        return fail(LP_EINVAL, "bad options");
    if (rkf && o->sort_steps > 0)
        return fail(LP_EINVAL, "RKF45 runs a whole output interval per launch: sort_steps "
                               "must be 0");
    const int64_t nsteps = (int64_t)std::llround(runtime / adt);
    if (std::fabs((double)nsteps * adt - runtime) > 1e-9 * std::max(runtime, adt))
        return fail(LP_EINVAL, "dt %g does not divide runtime %g", dt, runtime);
    int64_t per = nsteps;
    if (outputdt > 0.0) {
        per = (int64_t)std::llround(outputdt / adt);
        if (per < 1 || std::fabs((double)per * adt - outputdt) > 1e-9 * std::max(outputdt, adt))
            return fail(LP_EINVAL, "dt %g does not divide outputdt %g", dt, outputdt);
    }
    if (nsteps > 0x3FFFFFFF || per > 0x3FFFFFFF)
        return fail(LP_EINVAL, "too many steps in one call");
    if (allow_records && o->output_stride > 0) {
        const int64_t nper = (ps->n + o->output_stride - 1) / o->output_stride;
        if (ps->stride && ps->stride != o->output_stride)
            return fail(LP_EINVAL, "output_stride changed between calls (%lld then %d)",
                        (long long)ps->stride, o->output_stride);
        ps->stride = o->output_stride;
        ps->nper = nper;
    }
    plan = ExecPlan();
    plan.nsteps = nsteps;
    plan.per = per;
    plan.records = allow_records && ps->stride > 0;
    if (nsteps == 0)
        return LP_OK;
    double t0 = ps->t0;
    if (ps->dt != 0.0 && dt != ps->dt)  // keep t = t0 + step * dt at the current step
        t0 = (ps->t0 + (double)ps->step * ps->dt) - (double)ps->step * dt;
    // one launch per output segment, or with sort_steps = K one per K steps of it
    const int64_t cut = o->sort_steps > 0 ? (int64_t)o->sort_steps : 0;
    for (int64_t a = 0; a < nsteps; a += per) {
        const int64_t len = std::min(per, nsteps - a);
        const int64_t piece = cut > 0 ? cut : len;
        for (int64_t c = 0; c < len; c += piece) {
            plan.segs.emplace_back(ps->step + a + c, std::min(piece, len - c));
            plan.seg_end.push_back(c + piece >= len ? 1 : 0);
        }
    }
    size_t ntab = 0;
    if (!rkf)
        for (auto &sg : plan.segs)
            ntab += 2 * (size_t)sg.second + 1;
    const auto res = resident(fs);
    plan.used.assign(fs->capacity, 0);
    if (rkf) {
        // every particle runs its own stage times inside [t_a, t_b]: check the ends
        // against the resident snapshots, keep them all, and make sure the floor
        // step moves the clock anywhere in that range
        const double ta = t0 + (double)ps->step * dt, tb = t0 + (double)(ps->step + nsteps) * dt;
        TimeEntry e;
        int rc;
        if ((rc = bracket(fs, res, ta, e)) || (rc = bracket(fs, res, tb, e)))
            return rc;
        const double tm = std::max(std::fabs(ta), std::fabs(tb));
        if (tm + std::ldexp(adt, o->rkf_min_exp) * 0.25 == tm)
            return fail(LP_EINVAL, "the RKF45 floor step |dt| 2^%d is too small for times "
                                   "near %g", o->rkf_min_exp, tm);
        if (res.size() > ps->res_cap) {
            dfree(ps->dres);
            ps->res_cap = 0;
            if ((rc = dalloc(&ps->dres, res.size())))
                return rc;
            ps->res_cap = res.size();
        }
        std::vector<lp::ResTime> rt(res.size());
        for (size_t q = 0; q < res.size(); ++q) {
            rt[q].t = res[q].t;
            rt[q].slot = res[q].slot;
            rt[q].pad = 0;
            plan.used[res[q].slot] = 1;
        }
        // the table is tiny; a synchronous upload keeps it valid for every launch
        HIPCHECK(hipMemcpy(ps->dres, rt.data(), rt.size() * sizeof(lp::ResTime),
                           hipMemcpyHostToDevice));
    }
    if (ps->tab_pending) {
        HIPCHECK(hipEventSynchronize(ps->tab_ev));
        ps->tab_pending = false;
    }
    if (ntab > 0 && ntab > ps->tab_cap) {
        dfree(ps->dtab);
        if (ps->htab)
            (void)hipHostFree(ps->htab);
        ps->htab = nullptr;
        ps->tab_cap = 0;
        int rc = dalloc(&ps->dtab, ntab);
        if (rc)
            return rc;
        if (hipHostMalloc((void **)&ps->htab, ntab * sizeof(TimeEntry), hipHostMallocDefault) !=
            hipSuccess)
            return fail(LP_ENOMEM, "pinned allocation of the time table failed");
        ps->tab_cap = ntab;
    }
    if (!rkf) {
        size_t q = 0;
        for (auto &sg : plan.segs) {
            for (int64_t h = 0; h <= 2 * sg.second; ++h) {
                const int64_t nn = sg.first + h / 2;
                const double t = (h & 1) ? t0 + ((double)nn + 0.5) * dt : t0 + (double)nn * dt;
                int rc = bracket(fs, res, t, ps->htab[q]);
                if (rc)
                    return rc;
                plan.used[ps->htab[q].sa] = plan.used[ps->htab[q].sb] = 1;
                ++q;
            }
        }
    }
    ps->t0 = t0;
    if (ntab > 0) {
        HIPCHECK(hipMemcpyAsync(ps->dtab, ps->htab, ntab * sizeof(TimeEntry),
                                hipMemcpyHostToDevice, stream));
        HIPCHECK(hipEventRecord(ps->tab_ev, stream));
        ps->tab_pending = true;
    }
    for (int s = 0; s < fs->capacity; ++s)
        if (plan.used[s])
            HIPCHECK(hipStreamWaitEvent(stream, fs->ready[s], 0));
    if (ps->count_pending && hipEventQuery(ps->count_ev) == hipSuccess) {
        ps->n_launch = std::min<uint32_t>(ps->n_launch, *ps->hcount);
        ps->count_pending = false;
    }
    if (behave && o->sample_tracer) {
        for (int s = 0; s < fs->capacity; ++s)
            if (plan.used[s] && fs->tracer_seq[s] != fs->slot_seq[s])
                return fail(LP_ESTATE, "the snapshot at time %.17g has no tracer",
                            fs->slot_t[s]);
    }
    ps->dt = dt;
    if (behave)
        ps->behave_records = true;
    if (plan.records) {
        int64_t nout = 0;
        for (char e : plan.seg_end)
            nout += e ? 1 : 0;
        int rc = grow_records(ps, ps->nrec + nout + 1);
        if (rc)
            return rc;
        if (ps->nrec == 0 && (rc = take_record(ps, stream)))
            return rc;
    }
    lp::AdvectParams &P = plan.P;
    P.g = fs->g;
    P.f.slots = fs->dslots;
    P.f.slot_bytes = fs->slot_bytes;
    P.f.scales = fs->dscales;
    P.f.nzl = fs->nzl;
    P.f.steady = (fs->npushed == 1) ? 1 : 0;
    P.dt = dt;
    P.hdt = 0.5 * dt;
    P.dt6 = dt * (1.0 / 6.0);
    P.policy = o->recovery == LP_DELETE ? 0 : 1;
    P.cache = o->stencil_cache ? 1 : 0;
    P.scheme = o->kernel == LP_KERNEL_EULER ? 1 : (rkf ? 2 : 0);
    P.nearest = o->interp == LP_INTERP_NEAREST ? 1 : 0;
    P.Kh = o->Kh;
    P.run_id = o->run_id;
    P.seed = o->seed;
    P.x = ps->dx;
    P.y = ps->dy;
    P.z = ps->dz;
    P.status = ps->dst;
    P.psteps = ps->dpsteps;
    P.prej = ps->dpsteps + lp::kCountWords;
    P.hexp = ps->dexp;
    P.queues = ps->dqueues;
    P.f.tracer = fs->dtracer;
    P.behave = behave ? 1 : 0;
    P.sample = o->sample_tracer ? 1 : 0;
    P.sink_speed = o->sink_speed;
    P.dwell_depth = o->dwell_depth;
    P.maxage = o->maxage;
    P.temp = ps->dtemp;
    P.age = ps->dage;
    if (rkf) {
        P.res = ps->dres;
        P.nres = (int32_t)res.size();
        P.period = fs->period;
        P.inv_period = fs->period > 0.0 ? 1.0 / fs->period : 0.0;
        P.tol = o->rkf_tol;
        P.emin = o->rkf_min_exp;
        P.emax = o->rkf_max_exp;
        // attempts per particle and segment: at most one non-cut accepted step per
        // floor step of the segment, one cut step, one retry per accepted step plus
        // the initial descent to the floor
        const double floor_steps = std::ceil((double)per / std::ldexp(1.0, o->rkf_min_exp));
        const double bound = 2.0 * (floor_steps + 2.0) + (o->rkf_max_exp - o->rkf_min_exp) + 8.0;
        P.max_iter = bound > 2.0e9 ? 2000000000 : (int32_t)bound;
    }
    return LP_OK;
}

// Sort if due and fill the per-segment kernel arguments of segment k.
int exec_segment_pre(lp_pset *ps, const lp_exec_opts *o, ExecPlan &plan, size_t k,
                     hipStream_t stream)
{
    lp_fieldset *fs = ps->fs;
    if (o->sort_steps > 0 || (o->sort_every > 0 && ps->segs_since_sort >= o->sort_every)) {
        HIPCHECK(lp::launch_sort(fs->g, ps->dx, ps->dy, ps->dz, ps->dst, ps->dorder[ps->cur],
                                 ps->dcount + ps->cur, ps->n_launch, ps->dkeys, ps->dhist,
                                 ps->nbins, ps->dblk, ps->dorder[1 - ps->cur],
                                 ps->dcount + (1 - ps->cur), stream));
        ps->cur = 1 - ps->cur;
        ps->segs_since_sort = 0;
    }
    const auto &sg = plan.segs[k];
    plan.P.tab = ps->dtab + plan.toff;
    plan.P.step0 = sg.first;
    plan.P.nsteps = (int32_t)sg.second;
    plan.P.order = ps->dorder[ps->cur];
    plan.P.n_active = ps->dcount + ps->cur;
    plan.P.t_start = ps->t0 + (double)sg.first * ps->dt;
    plan.P.t_end = ps->t0 + (double)(sg.first + sg.second) * ps->dt;
    return LP_OK;
}

// Compact the active list and take the output record after segment k.
int exec_segment_post(lp_pset *ps, ExecPlan &plan, size_t k, hipStream_t stream)
{
    HIPCHECK(lp::launch_compact(ps->dorder[ps->cur], ps->dcount + ps->cur, ps->dst,
                                ps->dorder[1 - ps->cur], ps->dcount + (1 - ps->cur),
                                ps->n_launch, stream));
    ps->cur = 1 - ps->cur;
    if (plan.seg_end[k]) {
        ps->segs_since_sort++;
        if (plan.records) {
            int rc = take_record(ps, stream);
            if (rc)
                return rc;
        }
    }
    plan.toff += 2 * (size_t)plan.segs[k].second + 1;
    return LP_OK;
}

int exec_finish(lp_pset *ps, ExecPlan &plan, hipStream_t stream)
{
    lp_fieldset *fs = ps->fs;
    // release[s] must cover every reader of slot s, also readers on other streams
    // (two particle sets may share one field set): chain the earlier readers in
    // before recording, so that a push waits for all of them
    for (int s = 0; s < fs->capacity; ++s)
        if (plan.used[s]) {
            HIPCHECK(hipStreamWaitEvent(stream, fs->release[s], 0));
            HIPCHECK(hipEventRecord(fs->release[s], stream));
        }
    HIPCHECK(hipMemcpyAsync(ps->hcount, ps->dcount + ps->cur, sizeof(uint32_t),
                            hipMemcpyDeviceToHost, stream));
    HIPCHECK(hipEventRecord(ps->count_ev, stream));
    ps->count_pending = true;
    ps->step += plan.nsteps;
    ps->last_stream = stream;
    return LP_OK;
}

}  // namespace

extern "C" int pset_execute(lp_pset *ps, double runtime, double dt, double outputdt,
                            const lp_exec_opts *o, void *stream_)
{
    hipStream_t stream = (hipStream_t)stream_;
    ExecPlan plan;
    int rc = exec_prepare(ps, runtime, dt, outputdt, o, stream, true, plan);
    if (rc || plan.nsteps == 0)
        return rc;
    for (size_t k = 0; k < plan.segs.size(); ++k) {
        if ((rc = exec_segment_pre(ps, o, plan, k, stream)))
            return rc;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (o->profile) {
            HIPCHECK(hipEventCreate(&e0));
            HIPCHECK(hipEventCreate(&e1));
            HIPCHECK(hipEventRecord(e0, stream));
        }
        if (plan.P.scheme == 2)
            HIPCHECK(lp::launch_rkf45(ps->fs->dtype, ps->fs->is3d, plan.P, ps->n_launch, stream));
        else
            HIPCHECK(lp::launch_advect(ps->fs->dtype, ps->fs->is3d, plan.P, ps->n_launch,
                                       stream));
        if (o->profile) {
            HIPCHECK(hipEventRecord(e1, stream));
            ps->prof.emplace_back(e0, e1);
        }
        if ((rc = exec_segment_post(ps, plan, k, stream)))
            return rc;
    }
    return exec_finish(ps, plan, stream);
}

namespace {

// Device descriptors of a batched launch, reused from call to call once the
// previous launch that read them has completed.
struct BatchScratch {
    lp::AdvectParams *druns = nullptr, *hruns = nullptr;
    uint32_t *dcstart = nullptr, *hcstart = nullptr, *dqueues = nullptr;
    size_t cap_runs = 0;
    hipEvent_t done = nullptr;
    bool pending = false;
    // graph mode: the stream segments are captured on, and the executable graph of
    // the last captured segment (updated in place while the topology stays the same)
    hipStream_t cap = nullptr;
    hipGraphExec_t exec = nullptr;
    int64_t instantiated = 0, updated = 0;
};
thread_local BatchScratch g_batch;

// End a capture that failed part-way, dropping what was captured.
void abandon_capture(hipStream_t cs)
{
    hipGraph_t g = nullptr;
    (void)hipStreamEndCapture(cs, &g);
    if (g)
        (void)hipGraphDestroy(g);
    (void)hipGetLastError();
}

// Turn the captured graph of one segment into the executable graph: update the
// previous one in place when the topology matches, else instantiate anew.
int graph_from_capture(BatchScratch &b, hipGraph_t g)
{
    if (b.exec) {
        hipGraphNode_t err_node = nullptr;
        hipGraphExecUpdateResult res = hipGraphExecUpdateError;
        if (hipGraphExecUpdate(b.exec, g, &err_node, &res) == hipSuccess &&
            res == hipGraphExecUpdateSuccess) {
            b.updated++;
            return LP_OK;
        }
        (void)hipGetLastError();
        (void)hipGraphExecDestroy(b.exec);
        b.exec = nullptr;
    }
    HIPCHECK(hipGraphInstantiate(&b.exec, g, nullptr, nullptr, 0));
    b.instantiated++;
    return LP_OK;
}

int batch_reserve(size_t nruns)
{
    BatchScratch &b = g_batch;
    if (b.pending) {
        HIPCHECK(hipEventSynchronize(b.done));
        b.pending = false;
    }
    if (!b.done)
        HIPCHECK(hipEventCreateWithFlags(&b.done, hipEventDisableTiming));
    if (!b.dqueues) {
        int rc = dalloc(&b.dqueues, 8);
        if (rc)
            return rc;
    }
    if (nruns <= b.cap_runs)
        return LP_OK;
    dfree(b.druns);
    dfree(b.dcstart);
    if (b.hruns) (void)hipHostFree(b.hruns);
    if (b.hcstart) (void)hipHostFree(b.hcstart);
    b.hruns = nullptr;
    b.hcstart = nullptr;
    b.cap_runs = 0;
    int rc;
    if ((rc = dalloc(&b.druns, nruns)) || (rc = dalloc(&b.dcstart, nruns + 1)))
        return rc;
    if (hipHostMalloc((void **)&b.hruns, nruns * sizeof(lp::AdvectParams), hipHostMallocDefault) !=
            hipSuccess ||
        hipHostMalloc((void **)&b.hcstart, (nruns + 1) * sizeof(uint32_t), hipHostMallocDefault) !=
            hipSuccess)
        return fail(LP_ENOMEM, "pinned allocation of batch descriptors failed");
    b.cap_runs = nruns;
    return LP_OK;
}

int execute_batch(lp_pset **ps, int32_t nruns, double runtime, double dt, double outputdt,
                  const lp_exec_opts *opts, hipStream_t stream, int block, bool allow_records,
                  double *kernel_ms)
{
    if (!ps || !opts || nruns < 1)
        return fail(LP_EINVAL, "null argument or no runs");
    if (block != 64 && block != 128 && block != 256 && block != 512)
        return fail(LP_EINVAL, "batch block size must be 64, 128, 256 or 512");
    const lp_fieldset *f0 = ps[0] ? ps[0]->fs : nullptr;
    if (!f0)
        return fail(LP_EINVAL, "null particle set");
    for (int r = 0; r < nruns; ++r) {
        if (!ps[r])
            return fail(LP_EINVAL, "null particle set %d", r);
        const lp_fieldset *f = ps[r]->fs;
        if (f->is3d || f->dtype != f0->dtype || f->g.spherical != f0->g.spherical ||
            (f->npushed == 1) != (f0->npushed == 1))
            return fail(LP_EINVAL, "batched runs must be 2D with one storage type, one mesh kind "
                                   "and all steady or all time-varying (run %d differs)", r);
        if (opts[r].stencil_cache != opts[0].stencil_cache || opts[r].graph != opts[0].graph ||
            opts[r].sort_steps != opts[0].sort_steps)
            return fail(LP_EINVAL, "batched runs share the stencil_cache, graph and sort_steps "
                                   "settings");
        if (opts[r].kernel == LP_KERNEL_RKF45)
            return fail(LP_EINVAL, "the batched launch takes RK4 or Euler, not RKF45 (run %d)", r);
        if (opts[r].interp != LP_INTERP_LINEAR)
            return fail(LP_EINVAL, "the batched launch interpolates linearly only (run %d)", r);
        if (opts[r].sample_tracer || opts[r].maxage > 0.0 || opts[r].sink_speed > 0.0)
            return fail(LP_EINVAL, "the batched launch runs no worked-example kernels (run %d)",
                        r);
        for (int q = 0; q < r; ++q)
            if (ps[q] == ps[r])
                return fail(LP_EINVAL, "particle set %d appears twice", r);
    }
    std::vector<ExecPlan> plans(nruns);
    for (int r = 0; r < nruns; ++r) {
        int rc = exec_prepare(ps[r], runtime, dt, outputdt, &opts[r], stream, allow_records,
                              plans[r]);
        if (rc)
            return rc;
    }
    if (plans[0].nsteps == 0)
        return LP_OK;
    const size_t nseg = plans[0].segs.size();
    const bool use_graph = opts[0].graph != 0;
    for (size_t k = 0; k < nseg; ++k) {
        int rc = batch_reserve((size_t)nruns);
        if (rc)
            return rc;
        BatchScratch &b = g_batch;
        // graph mode: the segment's launches are recorded on the capture stream and
        // run as one graph on `stream`; otherwise they go to `stream` directly
        hipEvent_t e0 = nullptr, e1 = nullptr;
        const bool prof = opts[0].profile || kernel_ms;
        if (prof) {  // graph mode times the whole segment's graph
            HIPCHECK(hipEventCreate(&e0));
            HIPCHECK(hipEventCreate(&e1));
        }
        hipStream_t cs = stream;
        if (use_graph) {
            if (!b.cap)
                HIPCHECK(hipStreamCreateWithFlags(&b.cap, hipStreamNonBlocking));
            cs = b.cap;
            HIPCHECK(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
        }
        auto bail = [&](int code) {
            if (use_graph)
                abandon_capture(cs);
            return code;
        };
        uint32_t total = 0;
        for (int r = 0; r < nruns; ++r) {
            if ((rc = exec_segment_pre(ps[r], &opts[r], plans[r], k, cs)))
                return bail(rc);
            b.hruns[r] = plans[r].P;
            b.hcstart[r] = total;
            total += (ps[r]->n_launch + block - 1) / block;
        }
        b.hcstart[nruns] = total;
        hipError_t he = hipMemcpyAsync(b.druns, b.hruns, nruns * sizeof(lp::AdvectParams),
                                       hipMemcpyHostToDevice, cs);
        if (he == hipSuccess)
            he = hipMemcpyAsync(b.dcstart, b.hcstart, (nruns + 1) * sizeof(uint32_t),
                                hipMemcpyHostToDevice, cs);
        if (he != hipSuccess)
            return bail(fail(LP_EDEVICE, "batch descriptor upload failed: %s",
                             hipGetErrorString(he)));
        if (prof && !use_graph)
            HIPCHECK(hipEventRecord(e0, stream));
        int met = 0;
        bool brown = false;
        if (f0->g.spherical) {
            met = 3;  // every grid takes the 2-term latitude series
            for (int r = 0; r < nruns; ++r) {
                if (!ps[r]->fs->g.coslat) {
                    met = 2;  // some grid has cells too tall for the latitude series
                    break;
                }
                if (ps[r]->fs->g.cos_terms != 2)
                    met = 1;
            }
        }
        for (int r = 0; r < nruns; ++r)
            brown = brown || opts[r].Kh > 0.0;
        he = lp::launch_advect_batch(f0->dtype, f0->npushed == 1, met, brown, b.druns,
                                     b.dcstart, nruns, total, b.dqueues, block, cs, nullptr);
        if (he != hipSuccess)
            return bail(fail(LP_EDEVICE, "batched launch failed: %s", hipGetErrorString(he)));
        if (prof && !use_graph)
            HIPCHECK(hipEventRecord(e1, stream));
        if (!use_graph) {
            HIPCHECK(hipEventRecord(b.done, stream));
            b.pending = true;
        }
        for (int r = 0; r < nruns; ++r)
            if ((rc = exec_segment_post(ps[r], plans[r], k, cs)))
                return bail(rc);
        if (use_graph) {
            hipGraph_t g = nullptr;
            HIPCHECK(hipStreamEndCapture(cs, &g));
            rc = graph_from_capture(b, g);
            (void)hipGraphDestroy(g);
            if (rc)
                return rc;
            if (prof)
                HIPCHECK(hipEventRecord(e0, stream));
            HIPCHECK(hipGraphLaunch(b.exec, stream));
            if (prof)
                HIPCHECK(hipEventRecord(e1, stream));
            // the descriptors in pinned memory are read when the graph runs
            HIPCHECK(hipEventRecord(b.done, stream));
            b.pending = true;
        }
        if (prof) {
            if (kernel_ms) {
                HIPCHECK(hipEventSynchronize(e1));
                float ms = 0.f;
                HIPCHECK(hipEventElapsedTime(&ms, e0, e1));
                *kernel_ms += ms;
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
            } else {
                ps[0]->prof.emplace_back(e0, e1);
            }
        }
    }
    for (int r = 0; r < nruns; ++r) {
        int rc = exec_finish(ps[r], plans[r], stream);
        if (rc)
            return rc;
    }
    return LP_OK;
}

}  // namespace

extern "C" int pset_execute_batch(lp_pset **ps, int32_t nruns, double runtime, double dt,
                                  double outputdt, const lp_exec_opts *opts, int32_t block,
                                  void *stream)
{
    return execute_batch(ps, nruns, runtime, dt, outputdt, opts, (hipStream_t)stream,
                         block ? block : 256, true, nullptr);
}

namespace {

// The particle-step and retry counters of a set, each summed over its slots.
int read_counters(lp_pset *ps, unsigned long long sums[2])
{
    std::vector<unsigned long long> c(2 * (size_t)lp::kCountWords);
    HIPCHECK(hipMemcpy(c.data(), ps->dpsteps, c.size() * 8, hipMemcpyDeviceToHost));
    sums[0] = sums[1] = 0;
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < lp::kCountSlots; ++i)
            sums[k] += c[(size_t)k * lp::kCountWords + (size_t)i * lp::kCountStride];
    return LP_OK;
}

// Copy of the mutable state of a particle set, for autotuning trials.
struct Snapshot {
    double *x = nullptr, *y = nullptr, *z = nullptr;
    uint8_t *st = nullptr;
    uint32_t *order = nullptr, count = 0;
    unsigned long long psteps = 0;
    int cur = 0, segs_since_sort = 0;
    uint32_t n_launch = 0;
    int64_t step = 0, stride = 0;
    double t0 = 0.0, dt = 0.0;
};

int save_state(lp_pset *ps, Snapshot &s)
{
    const size_t N = (size_t)ps->n;
    int rc;
    if ((rc = dalloc(&s.x, N)) || (rc = dalloc(&s.y, N)) || (ps->dz && (rc = dalloc(&s.z, N))) ||
        (rc = dalloc(&s.st, N)) || (rc = dalloc(&s.order, N)))
        return rc;
    HIPCHECK(hipDeviceSynchronize());
    HIPCHECK(hipMemcpy(s.x, ps->dx, N * 8, hipMemcpyDeviceToDevice));
    HIPCHECK(hipMemcpy(s.y, ps->dy, N * 8, hipMemcpyDeviceToDevice));
    if (ps->dz) HIPCHECK(hipMemcpy(s.z, ps->dz, N * 8, hipMemcpyDeviceToDevice));
    HIPCHECK(hipMemcpy(s.st, ps->dst, N, hipMemcpyDeviceToDevice));
    HIPCHECK(hipMemcpy(s.order, ps->dorder[ps->cur], N * 4, hipMemcpyDeviceToDevice));
    HIPCHECK(hipMemcpy(&s.count, ps->dcount + ps->cur, 4, hipMemcpyDeviceToHost));
    unsigned long long sums[2];
    if ((rc = read_counters(ps, sums)))
        return rc;
    s.psteps = sums[0];
    s.cur = ps->cur;
    s.segs_since_sort = ps->segs_since_sort;
    s.n_launch = ps->n_launch;
    s.step = ps->step;
    s.stride = ps->stride;
    s.t0 = ps->t0;
    s.dt = ps->dt;
    return LP_OK;
}

int restore_state(lp_pset *ps, Snapshot &s)
{
    const size_t N = (size_t)ps->n;
    HIPCHECK(hipDeviceSynchronize());
    ps->cur = s.cur;
    HIPCHECK(hipMemcpy(ps->dx, s.x, N * 8, hipMemcpyDeviceToDevice));
    HIPCHECK(hipMemcpy(ps->dy, s.y, N * 8, hipMemcpyDeviceToDevice));
    if (ps->dz) HIPCHECK(hipMemcpy(ps->dz, s.z, N * 8, hipMemcpyDeviceToDevice));
    HIPCHECK(hipMemcpy(ps->dst, s.st, N, hipMemcpyDeviceToDevice));
    HIPCHECK(hipMemcpy(ps->dorder[ps->cur], s.order, N * 4, hipMemcpyDeviceToDevice));
    HIPCHECK(hipMemcpy(ps->dcount + ps->cur, &s.count, 4, hipMemcpyHostToDevice));
    {
        std::vector<unsigned long long> c(2 * (size_t)lp::kCountWords, 0ull);
        c[0] = s.psteps;
        HIPCHECK(hipMemcpy(ps->dpsteps, c.data(), c.size() * 8, hipMemcpyHostToDevice));
    }
    ps->segs_since_sort = s.segs_since_sort;
    ps->n_launch = s.n_launch;
    ps->step = s.step;
    ps->stride = s.stride;
    ps->t0 = s.t0;
    ps->dt = s.dt;
    ps->count_pending = false;
    return LP_OK;
}

void free_state(Snapshot &s)
{
    dfree(s.x);
    dfree(s.y);
    dfree(s.z);
    dfree(s.st);
    dfree(s.order);
}

std::string tune_key(lp_pset **ps, int nruns)
{
    double nodes = 0.0, parts = 0.0;
    for (int r = 0; r < nruns; ++r) {
        nodes += (double)ps[r]->fs->plane();
        parts += (double)ps[r]->n;
    }
    const int g = (int)std::lround(std::log2(std::max(1.0, nodes / nruns)));
    const int n = (int)std::lround(std::log2(std::max(1.0, parts)));
    static const char *dt[] = {"f64", "f32", "bf16", "f16s"};
    char buf[96];
    snprintf(buf, sizeof buf, "%s:%s:2d:runs%d:g%d:n%d", dt[ps[0]->fs->dtype],
             ps[0]->fs->g.spherical ? "sph" : "flat", nruns, g, n);
    return buf;
}

// The cache is a JSON object with one entry per line:
//   "key": {"block": B, "stencil_cache": C, "sort_every": S, "sort_steps": K, "ms": T},
// (entries in an older format without "sort_steps" do not parse and are tuned again)
bool cache_lookup(const char *path, const std::string &key, lp_tune *t)
{
    if (!path)
        return false;
    FILE *f = fopen(path, "r");
    if (!f)
        return false;
    char line[512];
    bool found = false;
    const std::string pat = "\"" + key + "\"";
    while (fgets(line, sizeof line, f)) {
        const char *p = strstr(line, pat.c_str());
        if (!p)
            continue;
        lp_tune r{};
        if (sscanf(p + pat.size(), " : {\"block\": %d, \"stencil_cache\": %d, \"sort_every\": %d, "
                                   "\"sort_steps\": %d, \"ms\": %lf}", &r.block,
                   &r.stencil_cache, &r.sort_every, &r.sort_steps, &r.ms) == 5) {
            *t = r;
            found = true;
        }
    }
    fclose(f);
    return found;
}

void cache_store(const char *path, const std::string &key, const lp_tune &t)
{
    if (!path)
        return;
    std::vector<std::string> lines;
    if (FILE *f = fopen(path, "r")) {
        char line[512];
        const std::string pat = "\"" + key + "\"";
        while (fgets(line, sizeof line, f)) {
            std::string l(line);
            while (!l.empty() && (l.back() == '\n' || l.back() == ','))
                l.pop_back();
            if (l.find("\": {") != std::string::npos && l.find(pat) == std::string::npos)
                lines.push_back(l);
        }
        fclose(f);
    }
    char buf[512];
    snprintf(buf, sizeof buf,
             "  \"%s\": {\"block\": %d, \"stencil_cache\": %d, \"sort_every\": %d, "
             "\"sort_steps\": %d, \"ms\": %.4f}",
             key.c_str(), t.block, t.stencil_cache, t.sort_every, t.sort_steps, t.ms);
    lines.push_back(buf);
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f)
        return;
    fprintf(f, "{\n");
    for (size_t k = 0; k < lines.size(); ++k)
        fprintf(f, "%s%s\n", lines[k].c_str(), k + 1 < lines.size() ? "," : "");
    fprintf(f, "}\n");
    fclose(f);
    rename(tmp.c_str(), path);
}

}  // namespace

extern "C" int pset_autotune_batch(lp_pset **ps, int32_t nruns, double dt, int32_t trial_steps,
                                   const lp_exec_opts *opts, const char *cache_path,
                                   lp_tune *best)
{
    if (!ps || !opts || !best || nruns < 1 || trial_steps < 1 || !(dt > 0.0))
        return fail(LP_EINVAL, "bad autotune arguments");
    const std::string key = tune_key(ps, nruns);
    if (cache_lookup(cache_path, key, best))
        return LP_OK;
    std::vector<Snapshot> saved(nruns);
    for (int r = 0; r < nruns; ++r) {
        int rc = save_state(ps[r], saved[r]);
        if (rc) {
            for (auto &s : saved) free_state(s);
            return rc;
        }
    }
    std::vector<lp_exec_opts> o(opts, opts + nruns);
    lp_tune b{};
    b.ms = 1e300;
    int rc = LP_OK;
    hipEvent_t t0 = nullptr, t1 = nullptr;
    if (hipEventCreate(&t0) != hipSuccess || hipEventCreate(&t1) != hipSuccess) {
        if (t0) (void)hipEventDestroy(t0);
        for (auto &sv : saved) free_state(sv);
        return fail(LP_EDEVICE, "event creation failed");
    }
    const int blocks[] = {128, 256, 512};
    // sort cadence ladder: never, once per output segment, every 64, 16 and 4 steps
    struct Cadence {
        int every, steps;
    };
    const Cadence ladder[] = {{0, 0}, {1, 0}, {0, 64}, {0, 16}, {0, 4}};
    // the trial spans at least two of the longest cadence's launches
    const int steps = std::max(trial_steps, 128);
    for (int cache = 1; cache >= 0 && rc == LP_OK; --cache)
        for (const Cadence &cad : ladder) {
            if (rc != LP_OK)
                break;
            for (int blk : blocks) {
                for (auto &x : o) {
                    x.stencil_cache = cache;
                    x.sort_every = cad.every;
                    x.sort_steps = cad.steps;
                    x.output_stride = 0;
                    x.profile = 0;
                    x.graph = 0;
                }
                // the trial is one output segment, timed whole on the device: the sorts
                // in it and the per-run preparation count, not the kernel alone
                for (int r = 0; r < nruns; ++r)
                    ps[r]->segs_since_sort = cad.every ? 1 << 30 : 0;
                float fms = 0.f;
                if (hipEventRecord(t0, nullptr) != hipSuccess) {
                    rc = fail(LP_EDEVICE, "event record failed");
                    break;
                }
                rc = execute_batch(ps, nruns, steps * dt, dt, 0.0, o.data(), nullptr, blk,
                                   false, nullptr);
                if (rc == LP_OK && (hipEventRecord(t1, nullptr) != hipSuccess ||
                                    hipEventSynchronize(t1) != hipSuccess ||
                                    hipEventElapsedTime(&fms, t0, t1) != hipSuccess))
                    rc = fail(LP_EDEVICE, "trial timing failed");
                const double ms = fms;
                for (int r = 0; r < nruns && rc == LP_OK; ++r)
                    rc = restore_state(ps[r], saved[r]);
                if (rc)
                    break;
                if (ms < b.ms) {
                    b.ms = ms;
                    b.block = blk;
                    b.stencil_cache = cache;
                    b.sort_every = cad.every;
                    b.sort_steps = cad.steps;
                }
            }
        }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    for (auto &s : saved)
        free_state(s);
    if (rc)
        return rc;
    *best = b;
    cache_store(cache_path, key, b);
    return LP_OK;
}

extern "C" int pset_status(lp_pset *ps, lp_counts *c, uint8_t *status)
{
    if (!ps || !c)
        return fail(LP_EINVAL, "null argument");
    HIPCHECK(hipStreamSynchronize(ps->last_stream));
    std::vector<uint8_t> st((size_t)ps->n);
    HIPCHECK(hipMemcpy(st.data(), ps->dst, st.size(), hipMemcpyDeviceToHost));
    unsigned long long steps[2] = {0, 0};
    if (int rc = read_counters(ps, steps))
        return rc;
    lp_counts r{};
    r.n = ps->n;
    for (uint8_t s : st) {
        if (s == 0) r.active++;
        if (s & LP_ST_OOB) r.oob++;
        if (s & LP_ST_LAND) r.land++;
        if (s & LP_ST_DELETED) r.deleted++;
    }
    r.particle_steps = (int64_t)steps[0];
    r.rejected_steps = (int64_t)steps[1];
    r.step = ps->step;
    r.time = ps->t0 + (double)ps->step * (ps->dt != 0.0 ? ps->dt : 0.0);
    *c = r;
    if (status)
        std::memcpy(status, st.data(), st.size());
    return LP_OK;
}

extern "C" int pset_get_behaviour(lp_pset *ps, double *temp, double *age)
{
    if (!ps)
        return fail(LP_EINVAL, "null argument");
    HIPCHECK(hipStreamSynchronize(ps->last_stream));
    const size_t N = (size_t)ps->n;
    if (temp) HIPCHECK(hipMemcpy(temp, ps->dtemp, N * 8, hipMemcpyDeviceToHost));
    if (age) HIPCHECK(hipMemcpy(age, ps->dage, N * 8, hipMemcpyDeviceToHost));
    return LP_OK;
}

extern "C" int pset_records_behaviour(lp_pset *ps, double *temp, double *age)
{
    if (!ps)
        return fail(LP_EINVAL, "null argument");
    if (!ps->behave_records)
        return fail(LP_ESTATE, "no execute with a worked-example kernel has run");
    HIPCHECK(hipStreamSynchronize(ps->last_stream));
    const size_t T = (size_t)(ps->nrec * ps->nper);
    if (T == 0 || !ps->rtemp)
        return LP_OK;
    if (temp) HIPCHECK(hipMemcpy(temp, ps->rtemp, T * 8, hipMemcpyDeviceToHost));
    if (age) HIPCHECK(hipMemcpy(age, ps->rage, T * 8, hipMemcpyDeviceToHost));
    return LP_OK;
}

extern "C" int pset_get_step_exponents(lp_pset *ps, int8_t *e)
{
    if (!ps || !e)
        return fail(LP_EINVAL, "null argument");
    HIPCHECK(hipStreamSynchronize(ps->last_stream));
    HIPCHECK(hipMemcpy(e, ps->dexp, (size_t)ps->n, hipMemcpyDeviceToHost));
    return LP_OK;
}

extern "C" int pset_get(lp_pset *ps, double *lon, double *lat, double *depth, int32_t *ci,
                        int32_t *cj, int32_t *ck)
{
    if (!ps)
        return fail(LP_EINVAL, "null argument");
    HIPCHECK(hipStreamSynchronize(ps->last_stream));
    const size_t N = (size_t)ps->n;
    if (lon) HIPCHECK(hipMemcpy(lon, ps->dx, N * 8, hipMemcpyDeviceToHost));
    if (lat) HIPCHECK(hipMemcpy(lat, ps->dy, N * 8, hipMemcpyDeviceToHost));
    if (depth && ps->fs->is3d) HIPCHECK(hipMemcpy(depth, ps->dz, N * 8, hipMemcpyDeviceToHost));
    if (ci || cj || ck) {
        int32_t *d = nullptr;
        int rc = dalloc(&d, 3 * N);
        if (rc)
            return rc;
        lp::RecordParams R{};
        R.g = ps->fs->g;
        R.x = ps->dx;
        R.y = ps->dy;
        R.z = ps->dz;
        R.status = ps->dst;
        R.n = ps->n;
        R.stride = 1;
        R.nper = ps->n;
        R.ci = d;
        R.cj = d + N;
        R.ck = d + 2 * N;
        hipError_t e = lp::launch_record(R, nullptr);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e == hipSuccess && ci) e = hipMemcpy(ci, d, N * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess && cj) e = hipMemcpy(cj, d + N, N * 4, hipMemcpyDeviceToHost);
        if (e == hipSuccess && ck) e = hipMemcpy(ck, d + 2 * N, N * 4, hipMemcpyDeviceToHost);
        dfree(d);
        HIPCHECK(e);
    }
    return LP_OK;
}

// ---------------------------------------------------------------- allocation-free query
// pset_get_noalloc: pset_get whose cell-index query writes into a fixed device array
// instead of a buffer allocated per call.  The array holds three int32 indices for up
// to LP_NOALLOC_MAX_PARTICLES particles; every GPU the library runs on holds its own
// copy until the process ends.  In host code `scratch` names a host-side stand-in,
// not a device address: the address on each device comes from hipGetSymbolAddress,
// taken once per device with that device current, and only that address is used.
static __device__ __align__(256) int32_t scratch[(size_t)LP_NOALLOC_MAX_PARTICLES * 3];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
int32_t *g_scratch_dev[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up on the first call).
int scratch_on_current_device(int32_t **out)
{
    int dev = -1;
    HIPCHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices)
        return fail(LP_EDEVICE, "device %d is beyond the %d devices the scratch table covers",
                    dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_dev[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(LP_EDEVICE, "hipGetSymbolAddress of the scratch array failed on device "
                                    "%d: %s", dev, hipGetErrorString(e));
        }
        g_scratch_dev[dev] = (int32_t *)p;
    }
    *out = g_scratch_dev[dev];
    return LP_OK;
}

}  // namespace

extern "C" int pset_get_noalloc(lp_pset *ps, double *lon, double *lat, double *depth,
                                int32_t *ci, int32_t *cj, int32_t *ck)
{
    if (!ps)
        return fail(LP_EINVAL, "null argument");
    if (ps->n > (int64_t)LP_NOALLOC_MAX_PARTICLES)
        return fail(LP_EINVAL, "pset_get_noalloc takes sets of at most %d particles (this one "
                               "has %lld); use pset_get", LP_NOALLOC_MAX_PARTICLES,
                    (long long)ps->n);
    const hipStream_t s = ps->last_stream;
    HIPCHECK(hipStreamSynchronize(s));
    const size_t N = (size_t)ps->n;
    if (lon) HIPCHECK(hipMemcpy(lon, ps->dx, N * 8, hipMemcpyDeviceToHost));
    if (lat) HIPCHECK(hipMemcpy(lat, ps->dy, N * 8, hipMemcpyDeviceToHost));
    if (depth && ps->fs->is3d) HIPCHECK(hipMemcpy(depth, ps->dz, N * 8, hipMemcpyDeviceToHost));
    if (!(ci || cj || ck))
        return LP_OK;
    int32_t *d = nullptr;
    int rc = scratch_on_current_device(&d);
    if (rc)
        return rc;
    // every index the copies below read is written by this launch: nothing needs clearing
    lp::RecordParams R{};
    R.g = ps->fs->g;
    R.x = ps->dx;
    R.y = ps->dy;
    R.z = ps->dz;
    R.status = ps->dst;
    R.n = ps->n;
    R.stride = 1;
    R.nper = ps->n;
    R.ci = d;
    R.cj = d + N;
    R.ck = d + 2 * N;
    HIPCHECK(lp::launch_record(R, s));
    HIPCHECK(hipStreamSynchronize(s));
    if (ci) HIPCHECK(hipMemcpy(ci, d, N * 4, hipMemcpyDeviceToHost));
    if (cj) HIPCHECK(hipMemcpy(cj, d + N, N * 4, hipMemcpyDeviceToHost));
    if (ck) HIPCHECK(hipMemcpy(ck, d + 2 * N, N * 4, hipMemcpyDeviceToHost));
    return LP_OK;
}

extern "C" int pset_records(lp_pset *ps, int64_t *nrec, int64_t *nper, double *lon, double *lat,
                            double *depth, uint8_t *status, int32_t *ci, int32_t *cj,
                            int32_t *ck)
{
    if (!ps || !nrec || !nper)
        return fail(LP_EINVAL, "null argument");
    *nrec = ps->nrec;
    *nper = ps->nper;
    if (!(lon || lat || depth || status || ci || cj || ck))
        return LP_OK;
    HIPCHECK(hipStreamSynchronize(ps->last_stream));
    const size_t T = (size_t)(ps->nrec * ps->nper);
    if (T == 0)
        return LP_OK;
    if (lon) HIPCHECK(hipMemcpy(lon, ps->rx, T * 8, hipMemcpyDeviceToHost));
    if (lat) HIPCHECK(hipMemcpy(lat, ps->ry, T * 8, hipMemcpyDeviceToHost));
    if (depth && ps->rz) HIPCHECK(hipMemcpy(depth, ps->rz, T * 8, hipMemcpyDeviceToHost));
    if (status) HIPCHECK(hipMemcpy(status, ps->rst, T, hipMemcpyDeviceToHost));
    if (ci) HIPCHECK(hipMemcpy(ci, ps->rci, T * 4, hipMemcpyDeviceToHost));
    if (cj) HIPCHECK(hipMemcpy(cj, ps->rcj, T * 4, hipMemcpyDeviceToHost));
    if (ck && ps->rck) HIPCHECK(hipMemcpy(ck, ps->rck, T * 4, hipMemcpyDeviceToHost));
    return LP_OK;
}

extern "C" int pset_timing(lp_pset *ps, double *kernel_ms, int64_t *launches)
{
    if (!ps || !kernel_ms || !launches)
        return fail(LP_EINVAL, "null argument");
    double tot = 0.0;
    for (auto &p : ps->prof) {
        HIPCHECK(hipEventSynchronize(p.second));
        float ms = 0.f;
        HIPCHECK(hipEventElapsedTime(&ms, p.first, p.second));
        tot += ms;
    }
    *kernel_ms = tot;
    *launches = (int64_t)ps->prof.size();
    for (auto &p : ps->prof) {
        (void)hipEventDestroy(p.first);
        (void)hipEventDestroy(p.second);
    }
    ps->prof.clear();
    return LP_OK;
}

extern "C" const char *lp_last_error(void) { return g_err.c_str(); }

extern "C" const char *lp_version(void) { return "lp-mi355x 0.1 (gfx950)"; }

// ---------------------------------------------------------------- internal helpers
// Reset a particle set to n <= capacity particles at device positions (x, y), time
// t0 and step 0, with every particle active; used for the surrogate's training
// rounds so one set serves every round.
int lp_pset_reset_device(lp_pset *ps, int64_t n, const double *x, const double *y, double t0,
                         hipStream_t stream)
{
    if (!ps || n < 1 || n > ps->n)
        return fail(LP_EINVAL, "bad reset");
    HIPCHECK(hipMemcpyAsync(ps->dx, x, (size_t)n * 8, hipMemcpyDeviceToDevice, stream));
    HIPCHECK(hipMemcpyAsync(ps->dy, y, (size_t)n * 8, hipMemcpyDeviceToDevice, stream));
    HIPCHECK(hipMemsetAsync(ps->dst, 0, (size_t)ps->n, stream));
    if (n < ps->n)  // the unused tail is never advanced
        HIPCHECK(hipMemsetAsync(ps->dst + n, LP_ST_DELETED, (size_t)(ps->n - n), stream));
    HIPCHECK(hipMemsetAsync(ps->dpsteps, 0,
                            2 * lp::kCountWords * sizeof(unsigned long long), stream));
    HIPCHECK(hipMemsetAsync(ps->dexp, 0, (size_t)ps->n, stream));
    HIPCHECK(hipMemsetAsync(ps->dtemp, 0xFF, (size_t)ps->n * sizeof(double), stream));
    HIPCHECK(hipMemsetAsync(ps->dage, 0, (size_t)ps->n * sizeof(double), stream));
    HIPCHECK(lp::launch_iota(ps->dorder[0], (size_t)n, stream));
    HIPCHECK(lp::launch_fill_u32(ps->dcount, (uint32_t)n, 1, stream));
    ps->cur = 0;
    ps->n_launch = (uint32_t)n;
    ps->count_pending = false;
    ps->t0 = t0;
    ps->dt = 0.0;
    ps->step = 0;
    ps->segs_since_sort = 1 << 30;
    ps->last_stream = stream;
    return LP_OK;
}

void lp_set_error(const char *msg) { g_err = msg; }

int lp_time_entry(const lp_fieldset *fs, double t, lp::TimeEntry *e)
{
    return bracket(fs, resident(fs), t, *e);
}
