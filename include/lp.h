/*
 * lp.h -- C ABI of the MI355X Lagrangian particle advection library.
 *
 * The interface follows the statement of the problem in Lange & van Sebille,
 * "Parcels v0.9" (GMD 2017):
 *   - a FieldSet of gridded Fields with time snapshots on a rectilinear grid
 *     (Sect. 2.4; read three time slices at a time and advanced, Sect. 3.1 and
 *     Sect. 3.4);
 *   - a ParticleSet created from longitude / latitude (/ depth) arrays
 *     (Sect. 2.1, Sect. 3.2);
 *   - pset.execute(kernel, runtime, dt, output interval, recovery), the dynamic
 *     update loop of Sect. 2.2 and Sect. 3.4, with per-particle error states
 *     mapped to a recovery action (Sect. 2.1.2);
 *   - the AdvectionRK4 / AdvectionRK4_3D kernels (Sect. 2.1.1, Sect. 3.3), with
 *     linear interpolation in space and time (Sect. 2.3, Sect. 2.4) and the
 *     m/s -> degree/s conversion on spherical meshes (Sect. 4.2.2).
 *
 * Conventions for every call:
 *   - return value: LP_OK (0) or a negative LP_E* code; lp_last_error() then
 *     returns a message (thread-local, valid until the next failing call on the
 *     same thread).  Per-particle problems are never return codes: they are
 *     status bits (LP_ST_*), as the paper maps particle errors to recovery
 *     kernels.
 *   - host arrays are owned by the caller and only read (or written) during the
 *     call; "_device" variants take device pointers on the library's GPU, which
 *     the caller keeps valid until the stream reaches the copy.
 *   - the library owns every device buffer it allocates; *_destroy frees them.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls that return data to the host synchronise that stream.
 *   - all positions are FP64; longitudes/latitudes in degrees on a spherical
 *     mesh, metres on a flat mesh; depth in metres, positive downward.
 */
#ifndef LP_H
#define LP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define LP_OK 0
#define LP_EINVAL (-1)  /* bad argument: sizes, non-monotone axes, dt not dividing */
#define LP_ENOMEM (-2)  /* device or pinned host allocation failed */
#define LP_EDEVICE (-3) /* a HIP runtime call failed */
#define LP_ETIME (-4)   /* a needed time is not covered by the resident snapshots */
#define LP_ESTATE (-5)  /* call not allowed in the current state */

/* mesh */
#define LP_MESH_FLAT 0
#define LP_MESH_SPHERICAL 1

/* device storage type of the field snapshots */
#define LP_F64 0        /* double values, FP64 interpolation */
#define LP_F32 1        /* float values, FP64 interpolation */
#define LP_BF16 2       /* bfloat16 (round-to-nearest-even), FP32 interpolation */
#define LP_F16_SCALED 3 /* float16 times a power-of-two scale per (variable,
                           level, snapshot), FP32 interpolation */

/* recovery policy on a particle error */
#define LP_DELETE 0 /* error bit plus LP_ST_DELETED; the particle is removed */
#define LP_FREEZE 1 /* error bit only; the particle stays where it was */

/* particle status bits */
#define LP_ST_OOB 1u     /* a stage point or the end point left the grid */
#define LP_ST_LAND 2u    /* the end point fell in a cell with four land corners */
#define LP_ST_DELETED 4u /* removed by the DELETE policy */
#define LP_ST_AGED 8u    /* reached maxage (with LP_ST_DELETED); see lp_exec_opts */

/* integrators (Sect. 2.1.1) */
#define LP_KERNEL_RK4 0   /* classical fourth-order Runge-Kutta, the default */
#define LP_KERNEL_EULER 1 /* Euler forward: one slope per step */
#define LP_KERNEL_RKF45 2 /* adaptive Runge-Kutta-Fehlberg 4(5), per-particle step;
                             see lp_exec_opts.rkf_tol */

/* spatial interpolation (Sect. 2.3); time is always linear */
#define LP_INTERP_LINEAR 0  /* bilinear / trilinear */
#define LP_INTERP_NEAREST 1 /* value of the nearest node (a half-way point goes up) */

/* ------------------------------------------------------------------ FieldSet */
typedef struct lp_fieldset lp_fieldset;

typedef struct {
    int32_t nx, ny;     /* horizontal nodes (>= 2 each) */
    int32_t nz;         /* 0: two-dimensional (U, V); >= 2: levels (U, V, W) */
    const double *lon;  /* nx strictly increasing (degrees or metres) */
    const double *lat;  /* ny strictly increasing */
    const double *depth;/* nz strictly increasing, NULL when nz == 0 */
    int32_t mesh;       /* LP_MESH_FLAT or LP_MESH_SPHERICAL */
    int32_t dtype;      /* LP_F64, LP_F32, LP_BF16 or LP_F16_SCALED */
    int32_t capacity;   /* device snapshot slots (>= 1); 3 keeps two resident
                           snapshots plus one being uploaded (Sect. 3.1) */
    double time_period; /* > 0: snapshots repeat with this period; every snapshot
                           of the period must then stay resident */
    const uint8_t *land;/* ny*nx node mask (1 = land), or NULL */
} lp_grid_desc;

/* Create a field set on the current device.  Copies the axes and the mask. */
int fieldset_create(const lp_grid_desc *g, lp_fieldset **out);

/* Push the snapshot at time t (advancetime, Sect. 3.4): U, V (and W when
 * nz >= 2) are host float arrays [max(nz,1)][ny][nx], i fastest, in m/s (W
 * positive downward).  Times must increase from push to push.  When all slots
 * are full the oldest snapshot is replaced, after the kernels that read it have
 * finished.  The arrays go to the device through two pinned staging chunks of
 * the library's (up to 256 MiB each, allocated at the first push): host threads
 * fill one chunk while the other is copied to the device on the field set's own
 * upload stream, which then converts the snapshot to the storage type.  The call
 * returns once the last chunk is queued, without waiting for the device copies;
 * a later pset_execute waits for them.  The host arrays may be reused when the
 * call returns.  LP_ENOMEM if the pinned staging cannot be allocated.  The upload
 * starts after the work queued on `stream` before the call; with stream NULL it
 * waits for nothing but the readers of the slot it replaces, so it can overlap
 * kernels already queued (the next time slice loads while the current one is
 * advected). */
int fieldset_push_snapshot(lp_fieldset *fs, double t, const float *U, const float *V,
                           const float *W, void *stream);
/* Same with double host arrays (LP_F64 storage keeps them exact). */
int fieldset_push_snapshot_f64(lp_fieldset *fs, double t, const double *U, const double *V,
                               const double *W, void *stream);
/* Same with float arrays already in device memory: they are converted into the
 * slot where they are, without a copy.  Work the caller queues on `stream` after
 * this call runs after the arrays have been read, so they may then be freed or
 * overwritten in stream order; with stream NULL the caller keeps them until the
 * next pset_execute that reads the slot has been queued and has completed. */
int fieldset_push_snapshot_device(lp_fieldset *fs, double t, const float *dU, const float *dV,
                                  const float *dW, void *stream);
/* A scalar tracer (the temperature of the worked example, Sect. 3.1 and
 * Sect. 3.3) for the resident snapshot at time t: a host float array laid out like
 * U ([max(nz,1)][ny][nx]), interpolated like the velocity.  The tracer belongs to that snapshot: when
 * a later push takes its slot, the slot has no tracer until this is called again.
 * LP_ESTATE if no resident snapshot has time t.  Synchronises the upload. */
int fieldset_push_tracer(lp_fieldset *fs, double t, const float *T, void *stream);
/* Same with a device array (copied in order on `stream`). */
int fieldset_push_tracer_device(lp_fieldset *fs, double t, const float *dT, void *stream);
/* Values held for the resident snapshot at time t, as float [max(nz,1)][ny][nx]
 * arrays (bfloat16 and scaled float16 values are returned exactly, as floats);
 * W may be NULL in 2D.  LP_ETIME if no resident snapshot has time t.  Syncs. */
int fieldset_get_snapshot(lp_fieldset *fs, double t, float *U, float *V, float *W);
/* Number of snapshots currently resident and their times (times may be NULL). */
int fieldset_resident(const lp_fieldset *fs, int32_t *count, double *times);
void fieldset_destroy(lp_fieldset *fs);

/* ---------------------------------------------------------------- ParticleSet */
typedef struct lp_pset lp_pset;

/* Create n particles from host arrays (depth NULL in 2D).  Particle p has id p.
 * Time is t0 + k*dt after k steps; step0 is the number of steps already taken
 * from t0 (so a set can be resumed exactly from pset_get output) and is also
 * the step index that keys the Brownian random numbers. */
int pset_create(lp_fieldset *fs, int64_t n, const double *lon, const double *lat,
                const double *depth, double t0, int64_t step0, lp_pset **out);
/* Same with device arrays (copied into the set's own buffers on `stream`). */
int pset_create_device(lp_fieldset *fs, int64_t n, const double *dlon, const double *dlat,
                       const double *ddepth, double t0, int64_t step0, void *stream,
                       lp_pset **out);

typedef struct {
    int32_t kernel;       /* LP_KERNEL_RK4, LP_KERNEL_EULER or LP_KERNEL_RKF45 */
    int32_t recovery;     /* LP_DELETE or LP_FREEZE */
    double Kh;            /* > 0: add a Brownian displacement sqrt(2 Kh |dt|) N(0,1)
                             metres per horizontal component after each step's RK4
                             end point X* (Sect. 4.2.7); on a spherical mesh the
                             metres become degrees with the metric at lat(X*) */
    uint32_t run_id, seed;/* Philox4x32-10 key (run_id, seed); counter (id, step) */
    int32_t output_stride;/* record every k-th particle id at each output time;
                             0 = no records */
    int32_t sort_every;   /* re-sort particles by grid tile every k output
                             segments (0 = never) */
    int32_t profile;      /* 1: time each advection launch with HIP events */
    int32_t stencil_cache;/* 1: each lane keeps its cell's stencil (as interpolation
                             coefficients, in registers and LDS) and reloads it only
                             when it changes cell or snapshot pair; 0: gather the
                             stencil at every stage (same results up to rounding) */
    int32_t interp;       /* LP_INTERP_LINEAR or LP_INTERP_NEAREST */
    /* LP_KERNEL_RKF45 (the adaptive scheme named in Sect. 2.1.1; the control
     * rule is this library's reading): each particle steps by |dt| 2^e with its
     * own integer exponent e in [rkf_min_exp, rkf_max_exp] (e starts at 0 and is
     * kept from call to call).  An attempt takes the six Fehlberg slopes; the
     * fourth-order solution advances the particle and the fifth-minus-fourth
     * difference, as a length in metres, is its error.  An error above rkf_tol
     * retries the step at e - 1 (unless e is already the minimum); an accepted
     * error at most rkf_tol / 32 raises e by one for the next step (up to the
     * maximum).  The last step of each output interval is cut short to land on
     * the output time and leaves e unchanged.  Needs Kh = 0; the batched launch
     * and the autotuner do not take it.  In 2D, stencil_cache = 1 runs the six
     * stages on the stencil cache (same results up to rounding); the gather form
     * (stencil_cache = 0) is the faster one at RKF45's long steps. */
    double rkf_tol;       /* > 0, metres per step */
    int32_t rkf_min_exp;  /* in [-30, 0]; |dt| 2^min must still move the clock */
    int32_t rkf_max_exp;  /* in [0, 30] */
    /* The worked example's custom kernels (Sect. 3.3), run in this order before
     * the advection of each step (the paper prints their code only as figures;
     * this is the library's reading).  Sinking (3D, sink_speed > 0): a particle
     * deeper than dwell_depth moves by sink_speed * dt, not past dwell_depth (so a
     * time-backward run raises it back to where it lived).  Age (maxage > 0): a
     * particle at or above dwell_depth (any particle when sinking is off) ages by
     * |dt|; on the step its age reaches maxage it gets LP_ST_AGED | LP_ST_DELETED
     * and does not move.  Sample (sample_tracer = 1): the particle's temp becomes
     * the tracer at its position and the step's start time.  While a sinking
     * particle is at its dwelling depth the advection is horizontal only.  Any of
     * these needs LP_KERNEL_RK4 or LP_KERNEL_EULER.  With stencil_cache = 1 they run
     * in the cached 3D kernel for FP32/FP64 fields without a Brownian term, else in
     * the gather kernel (same results up to rounding). */
    double sink_speed;    /* m/s, >= 0 (0 = off) */
    double dwell_depth;   /* m */
    double maxage;        /* s, >= 0 (0 = off) */
    int32_t sample_tracer;/* 1: sample the field set's tracer every step */
    int32_t graph;        /* pset_execute_batch only (every run the same): 1 = each output
                             segment's launches (sorts, descriptor upload, the batched
                             advection, compactions, records) are captured into a HIP
                             graph and launched as one; the executable graph is made at
                             the first segment and updated in place for the later ones
                             (made anew when a segment's launches differ, e.g. a sort);
                             same results as 0, bit for bit */
    int32_t sort_steps;   /* > 0: re-sort every sort_steps steps instead: each output
                             segment is advanced in launches of at most sort_steps steps,
                             each after a sort (sort_every is then ignored); not with
                             RKF45.  Results do not depend on the sort cadence */
} lp_exec_opts;

/* Advance every active particle by runtime/|dt| steps of dt, taking an output
 * record every outputdt (0 = only at the end).  |dt| must divide runtime and
 * outputdt (both >= 0).  A negative dt runs backward in time (the time-backward
 * mode of Sect. 2.2); time is t0 + step * dt, re-based when dt changes so that
 * the current time is kept.  The first execute of a set also records the start.
 * Asynchronous on `stream`; returns LP_ETIME before launching anything if a
 * stage time is not covered by the resident snapshots. */
int pset_execute(lp_pset *ps, double runtime, double dt, double outputdt,
                 const lp_exec_opts *opts, void *stream);

typedef struct {
    int64_t n, active, oob, land, deleted;
    int64_t particle_steps; /* (particle, step) pairs that started active; with
                               RKF45 the attempts that were not retried */
    double time;            /* current time */
    int64_t step;           /* steps of dt taken since t0 */
    int64_t rejected_steps; /* RKF45 attempts retried at half the step */
} lp_counts;

/* Run many independent particle sets (each with its own field set: grid size,
 * snapshots and particle count may all differ) through one persistent launch per
 * output segment.  Same result per set as calling pset_execute on each with its
 * own opts[r] (which must agree on stencil_cache, use RK4 or Euler and linear
 * interpolation); the field sets must all be 2D with one storage type, one mesh
 * kind, and all steady or all time-varying.  The
 * active particles of all sets are cut into chunks of `block` (64, 128, 256 or
 * 512; 0 = 256) particles, handed out through per-XCD atomic work queues. */
int pset_execute_batch(lp_pset **ps, int32_t nruns, double runtime, double dt, double outputdt,
                       const lp_exec_opts *opts, int32_t block, void *stream);

typedef struct {
    int32_t block, stencil_cache, sort_every, sort_steps; /* chosen launch shape */
    double ms;                                /* device time of the winning trial */
} lp_tune;

/* Autotuner for pset_execute_batch: times every combination of block size (128,
 * 256, 512), stencil cache (on, off) and sort cadence (never, once per output
 * segment, every 64, 16 or 4 steps) over max(trial_steps, 128) steps of dt from
 * the current state (the whole trial segment on the device: its sorts and
 * preparation included, not the kernel alone), restores the state after each
 * trial, and returns the fastest.  The choice is cached in the JSON file at
 * cache_path (NULL = no cache) under a key made of the storage type, mesh, run
 * count and the log2 of the mean grid size and of the particle count; a cached
 * entry is returned without trials.  Synchronises. */
int pset_autotune_batch(lp_pset **ps, int32_t nruns, double dt, int32_t trial_steps,
                        const lp_exec_opts *opts, const char *cache_path, lp_tune *best);

/* The particles' error states (Sect. 2.1.2: an error type such as out-of-bounds,
 * mapped to a recovery action; the worked example deletes particles that leave
 * the domain, Sect. 3.4): counts of active, out-of-bounds, land and deleted
 * particles, the particle-steps taken and the set's time and step, and, if
 * status != NULL, the n status bytes (LP_ST_* bits) in id order.  Synchronises
 * the stream of the last execute. */
int pset_status(lp_pset *ps, lp_counts *c, uint8_t *status);
/* The particles' state variables lon, lat (and depth) (Sect. 2.1.2: particle.lon,
 * particle.lat; Sect. 3.2) and the grid cell of each position (-1 outside the
 * grid), in id order whatever order the device processed them in; any output
 * pointer may be NULL.  Synchronises. */
int pset_get(lp_pset *ps, double *lon, double *lat, double *depth, int32_t *ci, int32_t *cj,
             int32_t *ck);
/* The particles' sampled tracer (NaN before the first sample) and age in seconds,
 * id order; either pointer may be NULL.  Synchronises. */
int pset_get_behaviour(lp_pset *ps, double *temp, double *age);
/* The tracer and age of every output record (record-major, like pset_records);
 * records taken before the first execute with a worked-example kernel hold NaN
 * and 0.  LP_ESTATE if no such execute has run.  Synchronises. */
int pset_records_behaviour(lp_pset *ps, double *temp, double *age);
/* The n RKF45 step exponents e (step |dt| 2^e) in id order.  Synchronises. */
int pset_get_step_exponents(lp_pset *ps, int8_t *e);
/* Allocation-free pset_get, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same outputs as pset_get, bit for bit, but the cell-index query writes into
 * a fixed device array of 3 x LP_NOALLOC_MAX_PARTICLES int32 (24 MiB) instead of a
 * buffer allocated per call.  Each GPU holds its own copy of that array from the
 * first call on it until the process ends.  Sets with more than
 * LP_NOALLOC_MAX_PARTICLES particles get LP_EINVAL.  Calls no hipMalloc or
 * hipFree.  Every call on one GPU shares that GPU's array: calls that overlap on
 * one GPU (from several host threads) race, and the caller must serialise them.
 * Synchronises the stream of the set's last execute. */
#define LP_NOALLOC_MAX_PARTICLES (1 << 21)
int pset_get_noalloc(lp_pset *ps, double *lon, double *lat, double *depth, int32_t *ci,
                     int32_t *cj, int32_t *ck);
/* Output records, taken at every output interval of an execute (Sect. 2.2 and
 * Sect. 3.4: the execute call's output interval; Sect. 3.5: positions stored on
 * the fly, one long vector per variable): *nrec records of *nper =
 * ceil(n / output_stride) particles (ids 0, k, 2k, ...), record-major, each with
 * position, status and cell indices.  Call with NULL arrays to get the sizes.
 * Synchronises. */
int pset_records(lp_pset *ps, int64_t *nrec, int64_t *nper, double *lon, double *lat,
                 double *depth, uint8_t *status, int32_t *ci, int32_t *cj, int32_t *ck);
/* Sum and count of the timed advection launches since the last call (needs
 * opts.profile = 1).  Synchronises. */
int pset_timing(lp_pset *ps, double *kernel_ms, int64_t *launches);
void pset_destroy(lp_pset *ps);

/* The random numbers of the Brownian term (Sect. 4.2.7), computed on the device by
 * the same code the advection kernels use: for each i < n, Philox4x32-10 (Salmon
 * et al., SC'11) with key (run_id, seed) and counter (pid[i], step[i], 0, 0) gives
 * words[4i..4i+3]; uniforms u1 = top 53 bits of (w0:w1) * 2^-53 + 2^-54 and u2 from
 * (w2:w3); Box-Muller gives normals[2i] = r cos(2 pi u2), normals[2i+1] =
 * r sin(2 pi u2), r = sqrt(-2 ln u1).  Host arrays; words or normals may be NULL.
 * Synchronises. */
int lp_philox_normals(uint32_t run_id, uint32_t seed, int64_t n, const uint32_t *pid,
                      const uint32_t *step, uint32_t *words, double *normals);

/* ------------------------------------------------------------ flow-map surrogate
 * A learned stand-in for a fixed number of RK4 steps: a fully connected network
 * 64 -> 256 -> 256 -> 256 -> 256 -> 2 with tanh-form GELU after each hidden layer,
 * bfloat16 weights and activations, FP32 accumulation on the matrix cores, FP32
 * master weights and Adam.  Parameters travel as one float array, layer by layer:
 * W_l (fan_in x fan_out, row-major) then b_l (fan_out). */
typedef struct lp_model lp_model;
int64_t surrogate_param_count(void);
/* He-normal initialisation (std sqrt(2 / fan_in)) from `seed`, zero biases. */
int surrogate_create(uint32_t seed, lp_model **out);
int surrogate_get_params(lp_model *m, float *params);
int surrogate_set_params(lp_model *m, const float *params);
/* Network output for B host rows X [B x 64] (rounded to bf16) -> Y [B x 2]. */
int surrogate_forward(lp_model *m, int64_t B, const float *X, float *Y);
/* Gradients (parameter layout) of L = (1/2B) sum (y - t)^2 over a batch of B rows
 * (B a multiple of 128), without updating; loss may be NULL. */
int surrogate_gradients(lp_model *m, int64_t B, const float *X, const float *T, float *grads,
                        float *loss);
/* One Adam step (b1 0.9, b2 0.999, eps 1e-8) on that batch; loss may be NULL. */
int surrogate_train_step(lp_model *m, int64_t B, const float *X, const float *T, double lr,
                         float *loss);
void surrogate_destroy(lp_model *m);

typedef struct {
    int64_t n_segments;         /* training segments to generate with RK4 */
    int32_t steps_per_segment;  /* fine RK4 steps per segment (24) */
    double dt;                  /* fine RK4 step (300 s) */
    int32_t round_size;         /* segments per generation round; a round starts all
                                   its particles at one time on the dt grid */
    int32_t batch;              /* training batch, a multiple of 128 */
    int64_t iterations;         /* Adam steps */
    double lr;                  /* initial learning rate, cosine-decayed to lr / 20 */
    uint32_t seed;
} lp_surrogate_cfg;

typedef struct {
    int64_t segments_kept, segments_dropped, iterations;
    double first_loss, final_loss; /* mean batch loss of the first / last 100 steps */
    double gen_ms, train_ms;
} lp_train_stats;

/* Train the network on the field set (2D; all snapshots resident).  Data: segments
 * of steps_per_segment RK4 steps of dt started uniformly inside cells whose four
 * corners are ocean, at start times uniform on the dt grid over the snapshot period
 * (or span); segments that leave the grid or reach land are dropped.  Features are
 * gathered from the snapshots on the fly; target: the segment displacement in
 * metres east and north.  Everything runs on the device.  Synchronises. */
int surrogate_train(lp_fieldset *fs, lp_model *m, const lp_surrogate_cfg *cfg,
                    lp_train_stats *st, void *stream);

typedef struct {
    int64_t segments, evaluated, accepted, fallback;
    double mlp_ms, coarse_ms, fine_ms, total_ms;
    double sort_ms; /* cell sorts of the active list and reordering of the state (every 12
                       segments) */
} lp_surrogate_stats;

/* Advance a 2D particle set by runtime in segments of steps_per_segment steps of dt,
 * taking the network's displacement where it agrees with RK4 over the segment in
 * two steps to within residual_m metres and ends inside the grid off land, and
 * re-integrating every other particle with the fine RK4 steps (plain RK4 is the
 * fallback and the arbiter).  Synchronises. */
int pset_execute_surrogate(lp_pset *ps, lp_model *m, double runtime, double dt,
                           int32_t steps_per_segment, double residual_m,
                           lp_surrogate_stats *st, void *stream);

/* The two steps of the surrogate around the network, on their own (the same kernels
 * that pset_execute_surrogate and surrogate_train run).
 *
 * surrogate_features: the network's input rows for n positions (x, y) at time t on a
 * 2D field set, as the bfloat16 values the network reads, returned as floats
 * X[n][64]: [0..3] lon/180, lat/90, sin and cos of 2 pi (t - T0) / P (T0 the first
 * resident snapshot, P the period, or the span of the resident snapshots); [4..53]
 * U, V (m/s) at the 5 x 5 nodes around the nearest node (j - 2 .. j + 2 outer, i - 2
 * .. i + 2 inner, U then V; indices clamped to the grid), each linear in time
 * between the snapshots bracketing t; [54..55] the position's offset from that node
 * in cell widths; [56..57] U, V bilinear at the position and linear in time;
 * [58..59] the cell's width and height in metres / 30 km; [60..63] zero.  Positions
 * outside the grid are clamped to it.  LP_ETIME if t is not covered.  Synchronises.
 *
 * surrogate_check: the residual check of the inference for n candidate segments
 * starting at (x0, y0): the network's output Y[i][2] (east and north displacement
 * in units of 7200 m) is accepted, accept[i] = 1 and (x1, y1) = its end point,
 * when the coarse estimate ended in the grid (coarse_status[i] == 0), the distance
 * in metres between the network's displacement and the coarse one (xc - x0,
 * yc - y0; converted to metres with the metric at y0 on a spherical mesh) is at
 * most residual_m, and the end point is inside the grid and not in a land cell;
 * otherwise accept[i] = 0 and (x1, y1) = (x0, y0).  Synchronises. */
int surrogate_features(lp_fieldset *fs, int64_t n, const double *x, const double *y, double t,
                       float *X);
int surrogate_check(lp_fieldset *fs, int64_t n, const double *x0, const double *y0,
                    const double *xc, const double *yc, const uint8_t *coarse_status,
                    const float *Y, double residual_m, uint8_t *accept, double *x1, double *y1);

const char *lp_last_error(void);
/* Library version string. */
const char *lp_version(void);

#ifdef __cplusplus
}
#endif

#endif /* LP_H */
