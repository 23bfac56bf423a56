"""Python access to the FP64 oracle (``lp_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline leg
of the benchmark may import this module; the product library never does, and it
shares no code with the HIP path.  Inputs come from the ``synthetic`` package.

The run driver below follows the execute statement of the paper (Sect. 2.2,
Sect. 3.4): advance every particle from the start time in steps of dt and take
an output record at every output interval, each record holding the position,
the status and the cell indices of that position.
"""

from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "lp_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

ST_OOB = 1
ST_LAND = 2
ST_DELETED = 4
ST_AGED = 8
POLICY_DELETE = 0
POLICY_FREEZE = 1
# Philox key word used with the run id: (run_id, SEED)
SEED = 0x17070516


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, FP64, no contraction, OpenMP)."""
    if force or not os.path.exists(LIB):
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
               "-fPIC", "-shared", "-o", LIB + ".tmp", SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class _FS(C.Structure):
    _fields_ = [("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
                ("X", C.c_void_p), ("Y", C.c_void_p), ("Z", C.c_void_p),
                ("spherical", C.c_int), ("nt", C.c_int), ("T", C.c_void_p),
                ("period", C.c_double), ("stored_f32", C.c_int),
                ("U", C.c_void_p), ("V", C.c_void_p), ("W", C.c_void_p),
                ("land", C.c_void_p), ("tracer", C.c_void_p), ("tracer_f32", C.c_int)]


class _OPT(C.Structure):
    _fields_ = [("policy", C.c_int), ("Kh", C.c_double),
                ("run_id", C.c_uint32), ("seed", C.c_uint32),
                ("scheme", C.c_int), ("nearest", C.c_int),
                ("tol", C.c_double), ("emin", C.c_int), ("emax", C.c_int),
                ("sink_speed", C.c_double), ("dwell_depth", C.c_double),
                ("maxage", C.c_double), ("sample", C.c_int)]


SCHEME_RK4 = 0
SCHEME_EULER = 1
SCHEME_RKF45 = 2
# RKF45 step control defaults: tolerance per step (m) and exponent range of |dt| 2^e
RKF_TOL = 1.0
RKF_EMIN = -6
RKF_EMAX = 4


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build()
        L = C.CDLL(LIB)
        P = C.c_void_p
        L.or_locate.argtypes = [C.c_double, P, C.c_int, C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.or_locate.restype = C.c_int
        L.or_sample.argtypes = [C.POINTER(_FS), C.c_double, C.c_double, C.c_double, C.c_double, P]
        L.or_sample.restype = C.c_int
        L.or_sample_nearest.argtypes = L.or_sample.argtypes
        L.or_sample_nearest.restype = C.c_int
        L.or_sample_tracer.argtypes = [C.POINTER(_FS), C.c_double, C.c_double, C.c_double,
                                       C.c_double, C.POINTER(C.c_double)]
        L.or_sample_tracer.restype = C.c_int
        L.or_time_bracket.argtypes = [C.POINTER(_FS), C.c_double, C.POINTER(C.c_int),
                                      C.POINTER(C.c_int), C.POINTER(C.c_double)]
        L.or_time_bracket.restype = C.c_int
        L.or_philox4x32_10.argtypes = [P, P, P]
        L.or_philox4x32_10.restype = None
        L.or_normals.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_uint32, P]
        L.or_normals.restype = None
        L.or_advance.argtypes = [C.POINTER(_FS), C.c_int64, P, P, P, P, P, C.c_double,
                                 C.c_double, C.c_int64, C.c_int64, C.POINTER(_OPT),
                                 C.POINTER(C.c_int64), C.c_int, P, P]
        L.or_advance.restype = C.c_int
        L.or_rkf45_attempt.argtypes = [C.POINTER(_FS), C.c_int, C.c_double, C.c_double, P, P,
                                       P, P]
        L.or_rkf45_attempt.restype = C.c_int
        L.or_metres.argtypes = [C.POINTER(_FS), C.c_double, P]
        L.or_metres.restype = C.c_double
        L.or_advance_rkf45.argtypes = [C.POINTER(_FS), C.c_int64, P, P, P, P, P, C.c_double,
                                       C.c_double, C.c_double, C.POINTER(_OPT),
                                       C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.c_int]
        L.or_advance_rkf45.restype = C.c_int
        L.or_cell_indices.argtypes = [C.POINTER(_FS), C.c_int64, P, P, P, P, P, P]
        L.or_cell_indices.restype = None
        L.or_max_threads.argtypes = []
        L.or_max_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data


class OracleFieldSet:
    """Field set view for the oracle.  Holds references to the arrays it points at.

    U, V, W carry a leading time axis: [nt, ny, nx] or [nt, nz, ny, nx], float32
    or float64 (read as FP64)."""

    def __init__(self, lon, lat, depth, times, U, V, W=None, spherical=False,
                 period=0.0, land=None, tracer=None):
        self.lon = np.ascontiguousarray(lon, np.float64)
        self.lat = np.ascontiguousarray(lat, np.float64)
        self.depth = None if depth is None else np.ascontiguousarray(depth, np.float64)
        self.times = np.ascontiguousarray(np.atleast_1d(times), np.float64)
        f32 = U.dtype == np.float32
        dt_ = np.float32 if f32 else np.float64
        self.U = np.ascontiguousarray(U, dt_)
        self.V = np.ascontiguousarray(V, dt_)
        self.W = None if W is None else np.ascontiguousarray(W, dt_)
        self.land = None if land is None else np.ascontiguousarray(land, np.uint8)
        self.tracer = None if tracer is None else np.ascontiguousarray(
            tracer, np.float32 if np.asarray(tracer).dtype == np.float32 else np.float64)
        nz = 0 if self.depth is None else self.depth.size
        if self.depth is not None and self.W is None:
            raise ValueError("3D field set needs W")
        self.s = _FS(self.lon.size, self.lat.size, nz, _ptr(self.lon), _ptr(self.lat),
                     _ptr(self.depth), int(bool(spherical)), self.times.size, _ptr(self.times),
                     float(period), int(f32), _ptr(self.U), _ptr(self.V), _ptr(self.W),
                     _ptr(self.land), _ptr(self.tracer),
                     int(self.tracer is not None and self.tracer.dtype == np.float32))

    @property
    def is3d(self):
        return self.depth is not None

    @classmethod
    def from_workload(cls, w):
        U, V, W = w.fields.materialise()
        return cls(w.grid.lon, w.grid.lat, w.grid.depth, w.fields.times, U, V, W,
                   spherical=w.grid.spherical, period=w.fields.period, land=w.grid.land,
                   tracer=w.fields.materialise_tracer())

    # -- single-point primitives used by the pins
    def sample(self, x, y, z, t, nearest=False):
        out = np.zeros(3)
        f = lib().or_sample_nearest if nearest else lib().or_sample
        rc = f(C.byref(self.s), x, y, z, t, out.ctypes.data)
        return rc, out

    def rkf45_attempt(self, t, h, p, nearest=False):
        """One RKF45 attempt: (rc, fourth-order end point, fifth-order end point,
        error estimate) from position p = (x, y, z) at time t with signed step h."""
        p = np.ascontiguousarray(p, np.float64)
        p4, p5, err = np.zeros(3), np.zeros(3), np.zeros(3)
        rc = lib().or_rkf45_attempt(C.byref(self.s), int(bool(nearest)), float(t), float(h),
                                    p.ctypes.data, p4.ctypes.data, p5.ctypes.data,
                                    err.ctypes.data)
        return rc, p4, p5, err

    def metres(self, y, e):
        e = np.ascontiguousarray(e, np.float64)
        return lib().or_metres(C.byref(self.s), float(y), e.ctypes.data)

    def sample_tracer(self, x, y, z, t):
        v = C.c_double()
        rc = lib().or_sample_tracer(C.byref(self.s), x, y, z, t, C.byref(v))
        return rc, v.value

    def time_bracket(self, t):
        s0, s1, tau = C.c_int(), C.c_int(), C.c_double()
        rc = lib().or_time_bracket(C.byref(self.s), t, C.byref(s0), C.byref(s1), C.byref(tau))
        return rc, s0.value, s1.value, tau.value

    def cell_indices(self, x, y, z=None):
        x = np.ascontiguousarray(x, np.float64)
        y = np.ascontiguousarray(y, np.float64)
        z = None if z is None else np.ascontiguousarray(z, np.float64)
        n = x.size
        ci = np.empty(n, np.int32)
        cj = np.empty(n, np.int32)
        ck = np.empty(n, np.int32)
        lib().or_cell_indices(C.byref(self.s), n, _ptr(x), _ptr(y), _ptr(z),
                              _ptr(ci), _ptr(cj), _ptr(ck))
        return ci, cj, ck


def locate(x: float, X: np.ndarray):
    X = np.ascontiguousarray(X, np.float64)
    i, f = C.c_int(), C.c_double()
    rc = lib().or_locate(float(x), X.ctypes.data, X.size, C.byref(i), C.byref(f))
    return (None, None) if rc else (i.value, f.value)


def philox4x32_10(ctr, key):
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    lib().or_philox4x32_10(c.ctypes.data, k.ctypes.data, out.ctypes.data)
    return out


def normals(run_id, seed, pid, step):
    out = np.zeros(2)
    lib().or_normals(run_id, seed, pid, step, out.ctypes.data)
    return out


@dataclass
class State:
    x: np.ndarray
    y: np.ndarray
    z: Optional[np.ndarray]
    status: np.ndarray
    pid: np.ndarray
    t_org: float
    step: int
    psteps: int = 0
    dt: Optional[float] = None  # dt of the previous advance (time origin bookkeeping)
    exps: Optional[np.ndarray] = None  # RKF45 step exponents (int8), step = |dt| 2^e
    rejected: int = 0                  # RKF45 attempts retried for accuracy
    temp: Optional[np.ndarray] = None  # sampled tracer (NaN before the first sample)
    age: Optional[np.ndarray] = None   # seconds lived at the dwelling depth


def make_state(x, y, z=None, pid=None, t_org=0.0, step=0) -> State:
    x = np.array(x, np.float64, copy=True)
    y = np.array(y, np.float64, copy=True)
    z = None if z is None else np.array(z, np.float64, copy=True)
    pid = np.arange(x.size, dtype=np.uint32) if pid is None else np.ascontiguousarray(pid, np.uint32)
    return State(x, y, z, np.zeros(x.size, np.uint8), pid, float(t_org), int(step),
                 exps=np.zeros(x.size, np.int8), temp=np.full(x.size, np.nan),
                 age=np.zeros(x.size))


def advance(fs: OracleFieldSet, st: State, dt: float, nsteps: int, Kh: float = 0.0,
            run_id: int = 0, seed: int = SEED, policy: int = POLICY_DELETE,
            nthreads: int = 0, scheme: int = SCHEME_RK4, nearest: bool = False,
            tol: float = RKF_TOL, emin: int = RKF_EMIN, emax: int = RKF_EMAX,
            sink_speed: float = 0.0, dwell_depth: float = 0.0, maxage: float = 0.0,
            sample: bool = False) -> int:
    """Advance ``st`` in place by ``nsteps`` steps of ``dt`` (negative dt runs
    backward in time); returns the oracle's return code (0, or -4 if a needed time
    lies outside the snapshots).  With RKF45 the call is one output interval: every
    particle goes from t_org + step dt to t_org + (step + nsteps) dt in adaptive
    steps |dt| 2^e."""
    if fs.is3d and st.z is None:
        raise ValueError("3D field set needs depths")
    opt = _OPT(int(policy), float(Kh), int(run_id) & 0xFFFFFFFF, int(seed) & 0xFFFFFFFF,
               int(scheme), int(bool(nearest)), float(tol), int(emin), int(emax),
               float(sink_speed), float(dwell_depth), float(maxage), int(bool(sample)))
    # time is t_org + step * dt; a change of dt keeps the current time
    if st.dt is not None and dt != st.dt:
        st.t_org = (st.t_org + st.step * st.dt) - st.step * dt
    ps = C.c_int64(0)
    if scheme == SCHEME_RKF45:
        if Kh != 0.0:
            raise ValueError("RKF45 takes no Brownian term")
        if st.exps is None:
            st.exps = np.zeros(st.x.size, np.int8)
        t_s = st.t_org + st.step * dt
        t_e = st.t_org + (st.step + int(nsteps)) * dt
        rj = C.c_int64(0)
        rc = lib().or_advance_rkf45(C.byref(fs.s), st.x.size, _ptr(st.x), _ptr(st.y),
                                    _ptr(st.z if fs.is3d else None), _ptr(st.status),
                                    _ptr(st.exps), t_s, t_e, float(dt), C.byref(opt),
                                    C.byref(ps), C.byref(rj), int(nthreads))
        if rc == 0:
            st.step += int(nsteps)
            st.psteps += ps.value
            st.rejected += rj.value
            st.dt = float(dt)
        return rc
    rc = lib().or_advance(C.byref(fs.s), st.x.size, _ptr(st.x), _ptr(st.y),
                          _ptr(st.z if fs.is3d else None), _ptr(st.status), _ptr(st.pid),
                          st.t_org, float(dt), st.step, int(nsteps), C.byref(opt),
                          C.byref(ps), int(nthreads), _ptr(st.temp), _ptr(st.age))
    if rc == 0:
        st.step += int(nsteps)
        st.psteps += ps.value
        st.dt = float(dt)
    return rc


def record(fs: OracleFieldSet, st: State) -> dict:
    ci, cj, ck = fs.cell_indices(st.x, st.y, st.z if fs.is3d else None)
    r = dict(lon=st.x.copy(), lat=st.y.copy(), status=st.status.copy(), ci=ci, cj=cj,
             temp=st.temp.copy(), age=st.age.copy())
    if fs.is3d:
        r["depth"] = st.z.copy()
        r["ck"] = ck
    return r


def run(fs: OracleFieldSet, st: State, dt: float, runtime: float, outputdt: float,
        Kh: float = 0.0, run_id: int = 0, policy: int = POLICY_DELETE,
        nthreads: int = 0, first_record: bool = True, scheme: int = SCHEME_RK4,
        nearest: bool = False, tol: float = RKF_TOL, emin: int = RKF_EMIN,
        emax: int = RKF_EMAX, sink_speed: float = 0.0, dwell_depth: float = 0.0,
        maxage: float = 0.0, sample: bool = False):
    """Execute for ``runtime`` with records every ``outputdt``; returns the list of
    records (the first taken at the start time when ``first_record``).  A negative
    dt runs backward in time (runtime and outputdt stay positive)."""
    adt = abs(dt)
    nsteps = int(round(runtime / adt))
    per = int(round(outputdt / adt)) if outputdt > 0 else nsteps
    if nsteps * adt != runtime or (outputdt > 0 and per * adt != outputdt):
        raise ValueError("dt must divide runtime and outputdt")
    recs = [record(fs, st)] if first_record else []
    done = 0
    while done < nsteps:
        k = min(per, nsteps - done)
        rc = advance(fs, st, dt, k, Kh=Kh, run_id=run_id, policy=policy, nthreads=nthreads,
                     scheme=scheme, nearest=nearest, tol=tol, emin=emin, emax=emax,
                     sink_speed=sink_speed, dwell_depth=dwell_depth, maxage=maxage,
                     sample=sample)
        if rc != 0:
            raise RuntimeError(f"oracle advance failed: {rc}")
        done += k
        recs.append(record(fs, st))
    return recs


def max_threads() -> int:
    return lib().or_max_threads()
