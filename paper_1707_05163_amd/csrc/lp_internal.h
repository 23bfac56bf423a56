// lp_internal.h -- device-side parameter blocks and launcher declarations shared by
// the library's translation units (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lp {

constexpr double kMetresPerDegree = 111120.0;  // 1852 m per arc minute
constexpr double kDegToRad = 0.017453292519943295;
constexpr int kTile = 16;        // horizontal cells per tile side (sort key)
constexpr int kGuessBins = 4096; // bins of the cell-guess table of a non-uniform axis
// The particle-step and retry counters are spread over kCountSlots slots, one 128-byte
// line apart (kCountWords 64-bit words per counter); a wave adds to the slot of its
// block and readers sum the slots.  A single counter would take one device-wide atomic
// per wave on one address, and those serialise: they alone made a launch of a few
// steps over millions of particles last most of a millisecond.
constexpr int kCountSlots = 64, kCountStride = 16, kCountWords = kCountSlots * kCountStride;
constexpr int kBlock = 256;      // threads per block of the advection kernels

enum Store : int { kF64 = 0, kF32 = 1, kBF16 = 2, kF16S = 3 };

// One axis of a rectilinear grid.
struct AxisDev {
    const double *c;         // n coordinates
    const double *rw;        // n-1 inverse cell widths 1/(c[i+1]-c[i])
    const int32_t *guess;    // kGuessBins entries (non-uniform axes) or null
    double lo, hi;           // c[0], c[n-1]
    double ginv;             // bins (or cells, if uniform) per unit coordinate
    int32_t n;
    int32_t uniform;         // 1: (x-lo)*ginv is the cell to within one
};

struct GridDev {
    AxisDev ax, ay, az;      // az.n == 0 in 2D
    const uint8_t *landcell; // (ny-1)*(nx-1) cells, 1 = four land corners; or null
    const double *coslat;    // cos and sin of each latitude node (spherical meshes whose
    const double *sinlat;    // cells are at most 5 degrees tall), else null
    int32_t spherical;
    int32_t cos_terms;       // terms of the cos / sin series across one cell (2, 3 or 4,
                             // from the tallest cell: 0.3, 1.5 or 5 degrees)
};

// Bracketing snapshots and weight of one stage time.
struct TimeEntry {
    double tau;
    int32_t sa, sb;          // slot indices
};

// One resident snapshot: its time and slot, in increasing time order.
struct ResTime {
    double t;
    int32_t slot, pad;
};

struct FieldDev {
    const void *slots;       // capacity slots, each slot_bytes long
    size_t slot_bytes;
    const float *scales;     // LP_F16_SCALED: [slot][level][var] power-of-two scales
    int32_t nzl;             // levels per slot (1 in 2D)
    int32_t steady;          // single snapshot: no time interpolation
    const float *tracer;     // scalar tracer, [slot][level][ny][nx] floats, or null
};

struct AdvectParams {
    GridDev g;
    FieldDev f;
    const TimeEntry *tab;    // 2*nsteps+1 entries: t_n, t_n+dt/2, t_n+dt, ...
    double dt;
    double hdt;              // dt / 2
    double dt6;              // dt * (1 / 6), RK4's weight unit
    int64_t step0;           // step index (from t0) of the first step of the launch
    int32_t nsteps;
    int32_t policy;          // 0 delete, 1 freeze
    int32_t cache;           // 1: stencil cache kernels
    int32_t scheme;          // 0 RK4, 1 Euler forward
    int32_t nearest;         // 1: nearest-neighbour in space
    uint32_t zero;           // always 0 (an offset the compiler cannot fold)
    double Kh;
    uint32_t run_id, seed;
    double *x, *y, *z;       // particle state, id order
    uint8_t *status;
    const uint32_t *order;   // active ids, processing order
    const uint32_t *n_active;// device count of `order`
    unsigned long long *psteps;  // kCountWords words (see kCountSlots)
    // adaptive RKF45 (scheme 2): each lane brackets its own stage times
    const ResTime *res;      // resident snapshots by time
    int32_t nres;
    int32_t emin, emax;      // step exponent range, step = |dt| 2^e
    int32_t max_iter;        // attempts per particle and launch (a bound never reached)
    double period;           // > 0: periodic snapshots
    double inv_period;       // 1 / period (a quotient estimate only)
    double t_start, t_end;   // the launch carries every particle from t_start to t_end
    double tol;              // error tolerance per step, metres
    int8_t *hexp;            // per-particle step exponents, id order
    uint32_t *queues;        // 8 work-queue counters of the persistent launch
    unsigned long long *prej;// attempts retried at half the step (kCountWords words)
    // the worked example's kernels ahead of each step's advection (gather kernels)
    int32_t behave;          // 1: any of them is on
    int32_t sample;          // sample the tracer into temp
    double sink_speed;       // m/s, 0 = off
    double dwell_depth;      // m
    double maxage;           // s, 0 = off
    double *temp, *age;      // per particle, id order
};

struct RecordParams {
    GridDev g;
    const double *x, *y, *z;
    const uint8_t *status;
    int64_t n, stride, nper;
    double *rx, *ry, *rz;
    uint8_t *rst;
    int32_t *ci, *cj, *ck;
    const double *temp, *age;   // worked-example variables (or null)
    double *rtemp, *rage;
};

// GEMM of the surrogate network: C[M x N] = sum_k A(i, k) B(k, j) on bf16 operands
// with FP32 accumulation, A(i, k) = A[i*sai + k*sak], B(k, j) = B[k*sbk + j*sbj].
enum : int { kEpiHidden = 0, kEpiOut = 1, kEpiBackData = 2, kEpiAccum = 3 };
struct GemmArgs {
    const uint16_t *A, *B;
    int64_t M, N, K, kchunk;   // M % 32 == 0, N % 32 == 0 (% 128 if N >= 128), K % 16 == 0
    int64_t sai, sak, sbk, sbj;
    const float *bias;         // hidden / output: per column
    float *Z;                  // hidden: FP32 pre-activation out (may be null)
    uint16_t *H;               // hidden: bf16 GELU(z) out; back-data: bf16 dz out
    int64_t ldc;               // row stride of Z, H, Zin, dZ
    float *Y;                  // output: FP32 out; accumulate: FP32 += C
    int64_t ldy;
    int32_t nvalid;            // output: columns actually stored
    const float *Zin;          // back-data: pre-activation of the layer below
    float *dZ;                 // back-data: FP32 dz out
};

// Inference of the surrogate network 64 -> 256 x 4 -> 2 in one kernel: X [rows][64]
// bf16 features, WT[l] bf16 [pad_out][fan_in], bias[l] FP32 [pad_out], Y [rows][2].
struct MlpFusedArgs {
    const uint16_t *X;
    int64_t rows;            // multiple of 32
    const uint16_t *WT[5];
    const float *bias[5];
    float *Y;
};

// launchers (return hipError_t of the launch)
hipError_t launch_advect(int store, bool is3d, const AdvectParams &p, uint32_t n_launch,
                         hipStream_t s);
hipError_t launch_rkf45(int store, bool is3d, const AdvectParams &p, uint32_t n_launch,
                        hipStream_t s);
hipError_t launch_record(const RecordParams &p, hipStream_t s);
// batched launch: met 0 flat, 1 spherical with latitude tables, 2 spherical without,
// 3 spherical with latitude tables and the 2-term series in every run;
// brown: some run has a Brownian term
hipError_t launch_advect_batch(int store, bool steady, int met, bool brown,
                               const AdvectParams *runs, const uint32_t *cstart, int nruns,
                               uint32_t total, uint32_t *queues, int block, hipStream_t s,
                               int *grid_out);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, size_t n, hipStream_t s);
hipError_t launch_iota(uint32_t *p, size_t n, hipStream_t s);
hipError_t launch_compact(const uint32_t *order_in, const uint32_t *n_in, const uint8_t *status,
                          uint32_t *order_out, uint32_t *n_out, uint32_t n_launch,
                          hipStream_t s);
hipError_t launch_sort(const GridDev &g, const double *x, const double *y, const double *z,
                       const uint8_t *status, const uint32_t *order_in, const uint32_t *n_in,
                       uint32_t n_launch, uint32_t *keys, uint32_t *hist, uint32_t nbins,
                       uint32_t *blocksums, uint32_t *order_out, uint32_t *n_out,
                       hipStream_t s, bool cells = false);
// bins of the sort's key: tiles (times levels in 3D), or with `cells` the cells of the
// tiles, kTile x kTile bins a tile (2D only; ignored in 3D)
uint32_t sort_bins(const GridDev &g, bool cells = false);
size_t sort_blocksums(uint32_t nbins);
hipError_t launch_convert_snapshot(int store, bool is3d, const float *U, const float *V,
                                   const float *W, const double *U64, const double *V64,
                                   const double *W64, size_t plane, int nzl, void *slot,
                                   float *scales, float *tmp, hipStream_t s);
hipError_t launch_philox_normals(uint32_t run_id, uint32_t seed, int64_t n, const uint32_t *pid,
                                 const uint32_t *step, uint32_t *words, double *normals,
                                 hipStream_t s);
hipError_t launch_slot_values(int store, bool is3d, const void *slot, const float *scales,
                              size_t plane, int nzl, float *U, float *V, float *W, hipStream_t s);
hipError_t launch_lat_tables(const double *lat, int ny, double *coslat, double *sinlat,
                              hipStream_t s);
hipError_t launch_gemm(int epi, const GemmArgs &g, hipStream_t s);
hipError_t launch_mlp_fused(const MlpFusedArgs &a, hipStream_t s);
hipError_t launch_loss_grad(const float *Y, const float *T, int64_t B, int ldy, float *dZ,
                            uint16_t *dZq, float *loss, hipStream_t s);
hipError_t launch_colsum(const float *dZ, int64_t B, int N, float *db, hipStream_t s);
hipError_t launch_adam(float *W, const float *G, float *m, float *v, int K, int N, int nvalid,
                       float lr, float b1, float b2, float eps, int t, uint16_t *Wb, uint16_t *WT,
                       hipStream_t s);
hipError_t launch_fill_f32(float *p, float v, int64_t n, hipStream_t s);
hipError_t launch_to_bf16(const float *x, int64_t n, uint16_t *y, hipStream_t s);
hipError_t launch_level_absmax(const float *F, size_t plane, int nzl, float *out,
                               hipStream_t s);

}  // namespace lp
