"""FieldSet / ParticleSet wrappers over the C ABI, named after the paper's API
(Sect. 2.1, Sect. 3).  Argument marshalling only: every step of the advection
runs in the HIP library.  Host arrays are numpy; device arrays are torch CUDA
tensors (torch provides device memory and the stream handle)."""

from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np

from . import _lib as L

SEED = 0x17070516
_DTYPES = {"f64": L.LP_F64, "f32": L.LP_F32, "bf16": L.LP_BF16, "f16s": L.LP_F16_SCALED}
_MESH = {"flat": L.LP_MESH_FLAT, "spherical": L.LP_MESH_SPHERICAL}
_RECOVERY = {"delete": L.LP_DELETE, "freeze": L.LP_FREEZE}
_KERNEL = {"rk4": L.LP_KERNEL_RK4, "euler": L.LP_KERNEL_EULER, "rkf45": L.LP_KERNEL_RKF45}
# RKF45 step control: tolerance per step (m), exponent range of the step |dt| 2^e
RKF_TOL, RKF_MIN_EXP, RKF_MAX_EXP = 1.0, -6, 4
_INTERP = {"linear": L.LP_INTERP_LINEAR, "nearest": L.LP_INTERP_NEAREST}


def _is_torch(a) -> bool:
    return type(a).__module__.startswith("torch")


def _stream(stream):
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return C.c_void_p(torch.cuda.current_stream().cuda_stream)
        except ImportError:
            pass
        return None
    if hasattr(stream, "cuda_stream"):
        return C.c_void_p(stream.cuda_stream)
    return C.c_void_p(int(stream))


def _host(a, dtype):
    return None if a is None else np.ascontiguousarray(a, dtype=dtype)


def _ptr(a):
    if a is None:
        return None
    if _is_torch(a):
        return C.c_void_p(a.data_ptr())
    return C.c_void_p(a.ctypes.data)


class FieldSet:
    """Velocity snapshots on a rectilinear lon/lat(/depth) grid held in a ring of
    ``capacity`` device slots."""

    def __init__(self, lon, lat, depth=None, mesh: str = "flat", dtype: str = "f32",
                 capacity: int = 3, time_period: float = 0.0, land=None):
        self._keep = [_host(lon, np.float64), _host(lat, np.float64), _host(depth, np.float64),
                      _host(land, np.uint8)]
        lo, la, de, ld = self._keep
        self.nx, self.ny = lo.size, la.size
        self.nz = 0 if de is None else de.size
        self.dtype = dtype
        self.mesh = mesh
        g = L.lp_grid_desc(self.nx, self.ny, self.nz, lo.ctypes.data, la.ctypes.data,
                           None if de is None else de.ctypes.data, _MESH[mesh], _DTYPES[dtype],
                           int(capacity), float(time_period),
                           None if ld is None else ld.ctypes.data)
        h = C.c_void_p()
        L.check(L.lib.fieldset_create(C.byref(g), C.byref(h)))
        self._h = h

    @classmethod
    def from_workload(cls, w, dtype: str = "f32", capacity: Optional[int] = None,
                      push: bool = True, time_period: Optional[float] = None):
        g = w.grid
        cap = w.fields.nt if capacity is None else capacity
        period = w.fields.period if time_period is None else time_period
        fs = cls(g.lon, g.lat, g.depth, "spherical" if g.spherical else "flat", dtype, cap,
                 period, g.land)
        if push:
            for s in range(min(cap, w.fields.nt)):
                fs.push_snapshot(w.fields.times[s], *w.fields.snapshot(s))
                if w.fields.has_tracer:
                    fs.push_tracer(w.fields.times[s], w.fields.tracer_snapshot(s))
        return fs

    @property
    def handle(self):
        return self._h

    def push_snapshot(self, t: float, U, V, W=None, stream=None):
        """advancetime: upload the snapshot at time t into the next ring slot.  The
        upload follows the work queued on `stream` (default: torch's current stream);
        stream=0 orders it after nothing, for sources that are already complete."""
        if _is_torch(U):
            L.check(L.lib.fieldset_push_snapshot_device(self._h, float(t), _ptr(U), _ptr(V),
                                                        _ptr(W), _stream(stream)))
            return
        if self.dtype == "f64" and np.asarray(U).dtype == np.float64:
            u, v, w = _host(U, np.float64), _host(V, np.float64), _host(W, np.float64)
            L.check(L.lib.fieldset_push_snapshot_f64(self._h, float(t), _ptr(u), _ptr(v),
                                                     _ptr(w), _stream(stream)))
            return
        u, v, w = _host(U, np.float32), _host(V, np.float32), _host(W, np.float32)
        L.check(L.lib.fieldset_push_snapshot(self._h, float(t), _ptr(u), _ptr(v), _ptr(w),
                                             _stream(stream)))

    advancetime = push_snapshot

    def push_tracer(self, t: float, T, stream=None):
        """The scalar tracer (e.g. temperature) of the resident snapshot at time t."""
        if _is_torch(T):
            L.check(L.lib.fieldset_push_tracer_device(self._h, float(t), _ptr(T),
                                                      _stream(stream)))
            return
        L.check(L.lib.fieldset_push_tracer(self._h, float(t), _ptr(_host(T, np.float32)),
                                           _stream(stream)))

    def get_snapshot(self, t: float):
        """Values held on the device for the snapshot at time t (exact, as float32)."""
        shape = (self.ny, self.nx) if self.nz == 0 else (self.nz, self.ny, self.nx)
        U, V = np.empty(shape, np.float32), np.empty(shape, np.float32)
        W = np.empty(shape, np.float32) if self.nz else None
        L.check(L.lib.fieldset_get_snapshot(self._h, float(t), _ptr(U), _ptr(V), _ptr(W)))
        return U, V, W

    def resident(self):
        n = C.c_int32()
        t = np.zeros(1024)
        L.check(L.lib.fieldset_resident(self._h, C.byref(n), t.ctypes.data))
        return t[: n.value].copy()

    def close(self):
        if getattr(self, "_h", None):
            L.lib.fieldset_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def philox_normals(run_id: int, seed: int, pid, step):
    """Philox4x32-10 words and Box-Muller normals computed on the device."""
    pid = np.ascontiguousarray(pid, np.uint32)
    step = np.ascontiguousarray(step, np.uint32)
    n = pid.size
    words = np.empty((n, 4), np.uint32)
    normals = np.empty((n, 2), np.float64)
    L.check(L.lib.lp_philox_normals(int(run_id), int(seed) & 0xFFFFFFFF, n, _ptr(pid),
                                    _ptr(step), _ptr(words), _ptr(normals)))
    return words, normals


class ParticleSet:
    """Particles with FP64 positions; particle p has id p."""

    def __init__(self, fieldset: FieldSet, lon, lat, depth=None, t0: float = 0.0,
                 step0: int = 0, stream=None):
        self.fieldset = fieldset
        h = C.c_void_p()
        if _is_torch(lon):
            self.n = int(lon.numel())
            L.check(L.lib.pset_create_device(fieldset.handle, self.n, _ptr(lon), _ptr(lat),
                                             _ptr(depth), float(t0), int(step0),
                                             _stream(stream), C.byref(h)))
        else:
            lo, la, de = _host(lon, np.float64), _host(lat, np.float64), _host(depth, np.float64)
            self.n = int(lo.size)
            L.check(L.lib.pset_create(fieldset.handle, self.n, _ptr(lo), _ptr(la), _ptr(de),
                                      float(t0), int(step0), C.byref(h)))
        self._h = h
        self.is3d = fieldset.nz > 0
        self._time = float(t0)       # the set's time, tracked for record times
        self._rec_times = []         # time of each output record
        self._stride = 0

    @staticmethod
    def opts(recovery: str = "delete", Kh: float = 0.0, run_id: int = 0, seed: int = SEED,
             output_stride: int = 0, sort_every: int = 1, profile: bool = False,
             stencil_cache: bool = True, kernel: str = "rk4", interp: str = "linear",
             tol: float = RKF_TOL, min_exp: int = RKF_MIN_EXP, max_exp: int = RKF_MAX_EXP,
             sink_speed: float = 0.0, dwell_depth: float = 0.0, maxage: float = 0.0,
             sample: bool = False, graph: bool = False, sort_steps: int = 0):
        return L.lp_exec_opts(_KERNEL[kernel], _RECOVERY[recovery], float(Kh), int(run_id),
                              int(seed) & 0xFFFFFFFF, int(output_stride), int(sort_every),
                              int(bool(profile)), int(bool(stencil_cache)), _INTERP[interp],
                              float(tol), int(min_exp), int(max_exp), float(sink_speed),
                              float(dwell_depth), float(maxage), int(bool(sample)),
                              int(bool(graph)), int(sort_steps))

    def execute(self, runtime: float, dt: float, outputdt: float = 0.0,
                recovery: str = "delete", Kh: float = 0.0, run_id: int = 0, seed: int = SEED,
                output_stride: int = 0, sort_every: int = 1, profile: bool = False,
                stencil_cache: bool = True, kernel: str = "rk4", interp: str = "linear",
                tol: float = RKF_TOL, min_exp: int = RKF_MIN_EXP, max_exp: int = RKF_MAX_EXP,
                sink_speed: float = 0.0, dwell_depth: float = 0.0, maxage: float = 0.0,
                sample: bool = False, sort_steps: int = 0, stream=None):
        """The update loop: runtime/|dt| steps of dt (negative dt runs backward).  With
        kernel="rkf45" each particle steps adaptively by |dt| 2^e, e in
        [min_exp, max_exp], to within `tol` metres per step."""
        o = self.opts(recovery, Kh, run_id, seed, output_stride, sort_every, profile,
                      stencil_cache, kernel, interp, tol, min_exp, max_exp, sink_speed,
                      dwell_depth, maxage, sample, sort_steps=sort_steps)
        L.check(L.lib.pset_execute(self._h, float(runtime), float(dt), float(outputdt),
                                   C.byref(o), _stream(stream)))
        if runtime > 0:
            if output_stride > 0:
                from .particlefile import record_times
                self._stride = int(output_stride)
                self._rec_times.extend(record_times(self._time, float(runtime),
                                                    float(outputdt), float(dt),
                                                    first=not self._rec_times))
            self._time += float(runtime) if dt > 0 else -float(runtime)

    def write_trajectories(self, path: str, **kw) -> int:
        """Write the output records as a CF-1.6 indexed-ragged trajectory file
        (particlefile.write_indexed); returns the number of observations."""
        from .particlefile import write_indexed
        recs = self.records()
        if recs["lon"].shape[0] != len(self._rec_times):
            raise RuntimeError("records were taken outside ParticleSet.execute; "
                               "use particlefile.write_indexed with their times")
        ids = np.arange(0, self.n, max(self._stride, 1))
        return write_indexed(path, recs, self._rec_times, ids,
                             spherical=self.fieldset.mesh == "spherical", **kw)

    def status(self):
        c = L.lp_counts()
        st = np.empty(self.n, np.uint8)
        L.check(L.lib.pset_status(self._h, C.byref(c), st.ctypes.data))
        counts = {k: getattr(c, k) for k, _ in L.lp_counts._fields_}
        return counts, st

    def behaviour(self):
        """Sampled tracer (NaN before the first sample) and age in seconds, id order."""
        temp, age = np.empty(self.n), np.empty(self.n)
        L.check(L.lib.pset_get_behaviour(self._h, temp.ctypes.data, age.ctypes.data))
        return temp, age

    def step_exponents(self):
        """RKF45 step exponents e (step |dt| 2^e), id order."""
        e = np.empty(self.n, np.int8)
        L.check(L.lib.pset_get_step_exponents(self._h, e.ctypes.data))
        return e

    def get(self):
        n = self.n
        out = dict(lon=np.empty(n), lat=np.empty(n), ci=np.empty(n, np.int32),
                   cj=np.empty(n, np.int32))
        if self.is3d:
            out["depth"] = np.empty(n)
            out["ck"] = np.empty(n, np.int32)
        L.check(L.lib.pset_get(self._h, _ptr(out["lon"]), _ptr(out["lat"]),
                               _ptr(out.get("depth")), _ptr(out["ci"]), _ptr(out["cj"]),
                               _ptr(out.get("ck"))))
        return out

    def records(self):
        nrec, nper = C.c_int64(), C.c_int64()
        L.check(L.lib.pset_records(self._h, C.byref(nrec), C.byref(nper), None, None, None,
                                   None, None, None, None))
        shape = (nrec.value, nper.value)
        out = dict(lon=np.empty(shape), lat=np.empty(shape), status=np.empty(shape, np.uint8),
                   ci=np.empty(shape, np.int32), cj=np.empty(shape, np.int32))
        if self.is3d:
            out["depth"] = np.empty(shape)
            out["ck"] = np.empty(shape, np.int32)
        L.check(L.lib.pset_records(self._h, C.byref(nrec), C.byref(nper), _ptr(out["lon"]),
                                   _ptr(out["lat"]), _ptr(out.get("depth")),
                                   _ptr(out["status"]), _ptr(out["ci"]), _ptr(out["cj"]),
                                   _ptr(out.get("ck"))))
        temp, age = np.empty(shape), np.empty(shape)
        if L.lib.pset_records_behaviour(self._h, _ptr(temp), _ptr(age)) == 0:
            out["temp"] = temp
            out["age"] = age
        return out

    def execute_surrogate(self, model: "Surrogate", runtime: float, dt: float = 300.0,
                          steps_per_segment: int = 24, residual_m: float = 50.0, stream=None):
        """Advance with the network where it passes the residual check, RK4 elsewhere."""
        st = L.lp_surrogate_stats()
        L.check(L.lib.pset_execute_surrogate(self._h, model.handle, float(runtime), float(dt),
                                             int(steps_per_segment), float(residual_m),
                                             C.byref(st), _stream(stream)))
        return {k: getattr(st, k) for k, _ in L.lp_surrogate_stats._fields_}

    def timing(self):
        ms, k = C.c_double(), C.c_int64()
        L.check(L.lib.pset_timing(self._h, C.byref(ms), C.byref(k)))
        return ms.value, k.value

    def close(self):
        if getattr(self, "_h", None):
            L.lib.pset_destroy(self._h)
            self._h = None

    @property
    def handle(self):
        return self._h

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def execute_batch(psets, runtime: float, dt: float, outputdt: float = 0.0, opts=None,
                  block: int = 256, stream=None):
    """One persistent launch per output segment for many independent particle sets;
    ``opts`` is a list of ParticleSet.opts(...) (one per set)."""
    n = len(psets)
    hs = (C.c_void_p * n)(*[p.handle for p in psets])
    oa = (L.lp_exec_opts * n)(*(opts if opts is not None else [ParticleSet.opts()] * n))
    L.check(L.lib.pset_execute_batch(hs, n, float(runtime), float(dt), float(outputdt), oa,
                                     int(block), _stream(stream)))


def autotune_batch(psets, dt: float, trial_steps: int, opts=None, cache_path=None):
    """Time the batched launch shapes on the current state (restored afterwards) and
    return the fastest as a dict; cached in the JSON file ``cache_path``."""
    n = len(psets)
    hs = (C.c_void_p * n)(*[p.handle for p in psets])
    oa = (L.lp_exec_opts * n)(*(opts if opts is not None else [ParticleSet.opts()] * n))
    t = L.lp_tune()
    L.check(L.lib.pset_autotune_batch(hs, n, float(dt), int(trial_steps), oa,
                                      None if cache_path is None else str(cache_path).encode(),
                                      C.byref(t)))
    return dict(block=t.block, stencil_cache=t.stencil_cache, sort_every=t.sort_every,
                sort_steps=t.sort_steps, ms=t.ms)


SIZES = (64, 256, 256, 256, 256, 2)


class Surrogate:
    """The flow-map network on the device (weights, optimiser state, kernels)."""

    def __init__(self, seed: int = 0):
        h = C.c_void_p()
        L.check(L.lib.surrogate_create(int(seed) & 0xFFFFFFFF, C.byref(h)))
        self._h = h

    @property
    def handle(self):
        return self._h

    @staticmethod
    def param_count() -> int:
        return int(L.lib.surrogate_param_count())

    def get_params(self):
        """List of (W, b) per layer, float32, W shaped (fan_in, fan_out)."""
        flat = np.empty(self.param_count(), np.float32)
        L.check(L.lib.surrogate_get_params(self._h, flat.ctypes.data))
        return _unflatten(flat)

    def set_params(self, layers):
        flat = np.concatenate([np.concatenate([np.asarray(W, np.float32).ravel(),
                                               np.asarray(b, np.float32).ravel()])
                               for W, b in layers]).astype(np.float32)
        L.check(L.lib.surrogate_set_params(self._h, flat.ctypes.data))

    def forward(self, X):
        X = np.ascontiguousarray(X, np.float32)
        Y = np.empty((X.shape[0], 2), np.float32)
        L.check(L.lib.surrogate_forward(self._h, X.shape[0], X.ctypes.data, Y.ctypes.data))
        return Y

    def gradients(self, X, T):
        X = np.ascontiguousarray(X, np.float32)
        T = np.ascontiguousarray(T, np.float32)
        g = np.empty(self.param_count(), np.float32)
        loss = np.zeros(1, np.float32)
        L.check(L.lib.surrogate_gradients(self._h, X.shape[0], X.ctypes.data, T.ctypes.data,
                                          g.ctypes.data, loss.ctypes.data))
        return _unflatten(g), float(loss[0])

    def train_step(self, X, T, lr: float):
        X = np.ascontiguousarray(X, np.float32)
        T = np.ascontiguousarray(T, np.float32)
        loss = np.zeros(1, np.float32)
        L.check(L.lib.surrogate_train_step(self._h, X.shape[0], X.ctypes.data, T.ctypes.data,
                                           float(lr), loss.ctypes.data))
        return float(loss[0])

    def train(self, fieldset: "FieldSet", n_segments: int, iterations: int,
              steps_per_segment: int = 24, dt: float = 300.0, round_size: int = 100_000,
              batch: int = 4096, lr: float = 1e-3, seed: int = 1, stream=None):
        """Generate RK4 segments on the field set and train on them (all on device)."""
        cfg = L.lp_surrogate_cfg(int(n_segments), int(steps_per_segment), float(dt),
                                 int(round_size), int(batch), int(iterations), float(lr),
                                 int(seed) & 0xFFFFFFFF)
        st = L.lp_train_stats()
        L.check(L.lib.surrogate_train(fieldset.handle, self._h, C.byref(cfg), C.byref(st),
                                      _stream(stream)))
        return {k: getattr(st, k) for k, _ in L.lp_train_stats._fields_}

    def close(self):
        if getattr(self, "_h", None):
            L.lib.surrogate_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _unflatten(flat):
    out, q = [], 0
    for a, b in zip(SIZES[:-1], SIZES[1:]):
        W = flat[q:q + a * b].reshape(a, b)
        q += a * b
        bb = flat[q:q + b]
        q += b
        out.append((W.copy(), bb.copy()))
    return out


def surrogate_features(fieldset: FieldSet, x, y, t: float):
    """The surrogate network's input rows [n x 64] at positions (x, y) and time t, as
    the bfloat16 values the network reads (see surrogate_features in lp.h)."""
    x = np.ascontiguousarray(x, np.float64)
    y = np.ascontiguousarray(y, np.float64)
    X = np.empty((x.size, 64), np.float32)
    L.check(L.lib.surrogate_features(fieldset.handle, x.size, _ptr(x), _ptr(y), float(t),
                                     _ptr(X)))
    return X


def surrogate_check(fieldset: FieldSet, x0, y0, xc, yc, coarse_status, Y, residual_m: float):
    """The surrogate's residual check on n candidate segments: (accept, x1, y1)."""
    x0, y0, xc, yc = (np.ascontiguousarray(a, np.float64) for a in (x0, y0, xc, yc))
    st = np.ascontiguousarray(coarse_status, np.uint8)
    Y = np.ascontiguousarray(Y, np.float32)
    n = x0.size
    acc = np.empty(n, np.uint8)
    x1, y1 = np.empty(n), np.empty(n)
    L.check(L.lib.surrogate_check(fieldset.handle, n, _ptr(x0), _ptr(y0), _ptr(xc), _ptr(yc),
                                  _ptr(st), _ptr(Y), float(residual_m), _ptr(acc), _ptr(x1),
                                  _ptr(y1)))
    return acc.astype(bool), x1, y1
