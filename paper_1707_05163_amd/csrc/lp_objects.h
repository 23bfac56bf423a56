// lp_objects.h -- host-side objects behind the opaque handles of the C ABI
// (internal to the library).
#pragma once

#include <utility>
#include <vector>

#include "../../include/lp.h"
#include "lp_internal.h"

// device arrays of one grid axis
struct DevAxis {
    double *c = nullptr, *rw = nullptr;
    int32_t *guess = nullptr;
};

struct lp_fieldset {
    int device = 0;
    int nx = 0, ny = 0, nz = 0, nzl = 1;
    bool is3d = false;
    int mesh = 0, dtype = 0, capacity = 0;
    double period = 0.0;
    DevAxis dx_, dy_, dz_;
    lp::GridDev g{};
    uint8_t *dland = nullptr;      // land cells
    uint8_t *dlandnode = nullptr;  // land nodes (seeding in all-ocean cells)
    double *dcoslat = nullptr, *dsinlat = nullptr;
    char *dslots = nullptr;
    size_t slot_bytes = 0;
    float *dscales = nullptr;
    float *dtracer = nullptr;       // tracer slots (allocated at the first tracer push)
    std::vector<int64_t> tracer_seq;// push index whose tracer each slot holds, -1 = none
    float *dtmp = nullptr;
    float *dstage = nullptr;
    double *dstage64 = nullptr;
    // pinned host staging of pushes from host memory: two chunks of pin_chunk bytes,
    // each with the event of its last host-to-device copy
    char *hpin = nullptr;
    size_t pin_chunk = 0;
    hipEvent_t pin_ev[2] = {nullptr, nullptr};
    bool pin_pending[2] = {false, false};
    int pin_next = 0;
    hipEvent_t src_done = nullptr;  // device-source pushes: the source has been read
    hipStream_t up = nullptr;
    std::vector<hipEvent_t> ready, release;
    std::vector<double> slot_t;
    std::vector<int64_t> slot_seq;  // push index held by each slot, -1 = empty
    int64_t npushed = 0;
    double first_t = 0.0, last_t = 0.0;

    size_t plane() const { return (size_t)nx * (size_t)ny; }
};

struct lp_pset {
    lp_fieldset *fs = nullptr;
    int64_t n = 0;
    double *dx = nullptr, *dy = nullptr, *dz = nullptr;
    uint8_t *dst = nullptr;
    uint32_t *dorder[2] = {nullptr, nullptr};
    uint32_t *dcount = nullptr;  // [2]
    int cur = 0;
    uint32_t n_launch = 0;       // host upper bound of the active count
    uint32_t *hcount = nullptr;  // pinned copy of the device count
    hipEvent_t count_ev = nullptr;
    bool count_pending = false;
    uint32_t *dkeys = nullptr, *dhist = nullptr, *dblk = nullptr;
    uint32_t nbins = 0;
    unsigned long long *dpsteps = nullptr;  // [0] particle-steps, [1] RKF45 retries
    int8_t *dexp = nullptr;                  // RKF45 step exponents
    double *dtemp = nullptr, *dage = nullptr;// worked-example tracer sample and age
    bool behave_records = false;             // records carry temp and age
    double *rtemp = nullptr, *rage = nullptr;
    uint32_t *dqueues = nullptr;             // RKF45 work queues (8)
    lp::ResTime *dres = nullptr;             // resident-snapshot table of RKF45 launches
    size_t res_cap = 0;
    double t0 = 0.0, dt = 0.0;
    int64_t step = 0;
    // output records (record-major)
    int64_t stride = 0, nper = 0, nrec = 0, rec_cap = 0;
    double *rx = nullptr, *ry = nullptr, *rz = nullptr;
    uint8_t *rst = nullptr;
    int32_t *rci = nullptr, *rcj = nullptr, *rck = nullptr;
    // time table
    lp::TimeEntry *dtab = nullptr, *htab = nullptr;
    size_t tab_cap = 0;
    hipEvent_t tab_ev = nullptr;
    bool tab_pending = false;
    // profiling
    std::vector<std::pair<hipEvent_t, hipEvent_t>> prof;
    int segs_since_sort = 1 << 30;
    hipStream_t last_stream = nullptr;
};


int lp_pset_reset_device(lp_pset *ps, int64_t n, const double *x, const double *y, double t0,
                         hipStream_t stream);
void lp_set_error(const char *msg);
// bracketing resident snapshots of time t (LP_ETIME if not covered)
int lp_time_entry(const lp_fieldset *fs, double t, lp::TimeEntry *e);
