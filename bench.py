#!/usr/bin/env python3
"""Benchmark of the RK4 advection hot path on one MI355X.

Workload (default): the 3D field on the global 0.1 degree grid with 50 stretched
depth levels (3600 x 1800 x 50), 11 daily float32 U, V, W snapshots built in HBM
and streamed through a three-slot ring (two resident, one being converted: the
paper's execute-one-day-then-advancetime loop), 10,000,000 particles, RK4_3D with
dt = 600 s for 10 days (1440 steps), daily records of every 100th particle.  One
benchmark step is that whole 10-day run (snapshot pushes, advection, compaction
and records) with the source snapshots and start positions already in HBM.

Prints one JSON line: particle-steps/s, the roofline of the dominant kernel
(algorithmic FP64 flops per launch over the launch time measured with HIP events
on the launch stream, against the FP64 vector peak; with the stencil cache the
kernel is bound by instruction issue, not by HBM), the algorithmic-byte rate and
reuse factor beside it, the counted HBM bytes and VALU issue rate from the
recorded rocprofv3 counters while the kernel source matches them, the error in km
of each output time against the FP64 oracle, and the FP64 oracle timed on the
host cores (all cores and one) on a bounded sample of the same workload.
Other workloads: --config cfg1 | cfg3 | cfg4 | foram.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DAY_S = 86400.0
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector (FMA = 2 flops)
# Vector instruction issue: 256 CUs x 4 SIMDs, each issuing one wave64 VALU
# instruction every 4 cycles at 2.4 GHz (a wave64 FP64 FMA is 128 flops, so this is
# the FP64 peak counted in instructions: 78.6e12 / 128).
VALU_ISSUE_PEAK = 1024 * 2.4e9 / 4.0

# Algorithmic cost of one 2D spherical RK4 particle-step with linear time
# interpolation (see the design notes): bytes of the four-corner stencil of U, V
# at two snapshots in float32, and FP64 flops of the method (cos excluded,
# a division counted as one flop).
STENCIL_BYTES_2D_F32 = 4 * 2 * 2 * 4     # 64 B
STATE_BYTES_2D = 8 + 8 + 8 + 8 + 4 + 1 + 1  # lon, lat read + write, order id, status r/w
FLOPS_2D_STEP = 230
FLOPS_3D_STEP = 567
FLOPS_BROWNIAN = 9  # sqrt(2 Kh dt), two kicks, -2 ln u1 scaling, 2 pi u2 (transcendentals excluded)
# One RKF45 attempt in 2D: six stages of 51 flops (as in RK4), 80 for the stage
# positions (15 tableau terms x 2 flops x 2 coordinates + 5 x 4 for p + h s), 62
# for the fourth-order and error combinations, the end point, the error length and
# the six stage times; stencil bytes: six stages x 64 B.
FLOPS_RKF45_ATTEMPT_2D = 448
STENCIL_BYTES_RKF45_2D_F32 = 6 * 64
STATE_BYTES_RKF45_2D = STATE_BYTES_2D + 2  # plus the step exponent read and written

# Counter record of the dominant kernel, from rocprofv3 --pmc passes (one counter set
# per run) over each mode's default workload: FETCH_SIZE and WRITE_SIZE in KiB per
# dispatch (FETCH_SIZE counts half the bytes that a conversion kernel of known size
# reads, so it is scaled by 2.0; WRITE_SIZE matches a fill of known size, factor 1.0),
# the L2 hits and misses, and the wave-level VALU and SALU instruction counts.  The
# figures belong to the kernel source they were taken on: they are reported only
# while the digest of advect.hip's code (comments and whitespace dropped) equals the
# one recorded here, and come from the summary named in COUNTER_SOURCE.
FETCH_SCALE, WRITE_SCALE = 2.0, 1.0
COUNTER_SOURCE = "profiles/counters_k_advect2d_cfg1_k_advect3d_cfg2.md"
COUNTERS = {
    "advect_sha256": "07a8e58413fc66a254fc93aeedf8de7f10067d808f557bdb13fd324019b54e0c",
    "cfg1": (185046.8, 64867.8),    # (FETCH_SIZE KiB, WRITE_SIZE KiB) per launch of k_advect2d
    "cfg2": (7774787.2, 246243.9),  # the same for k_advect3d
    # (TCC_HIT_sum, TCC_MISS_sum) per launch: L2 requests of the same kernels
    "cfg1_l2": (3889879.5, 4499888.4),
    "cfg2_l2": (71593672.8, 126480295.3),
    # (SQ_INSTS_VALU, SQ_INSTS_SALU) wave instructions per launch
    "cfg1_sq": (8.45743e+08, 4.75763e+08),
    "cfg2_sq": (8.06692e+09, 3.03271e+09),
}


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=3)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--config", default="cfg2",
                   choices=["cfg1", "cfg2", "cfg3", "cfg4", "foram"],
                   help="workload (default cfg2: 3D, 10M particles, 3600x1800x50, 10 days)")
    p.add_argument("--particles", type=int, default=None,
                   help="particle count (default: the workload's own: cfg1 1M, cfg2 10M, "
                        "cfg4 4M, foram 1M)")
    p.add_argument("--days", type=int, default=None,
                   help="simulated days (default: cfg1 30, cfg2 10, cfg4 30)")
    p.add_argument("--dtype", default="f32", choices=["f32", "bf16", "f16s"])
    p.add_argument("--output-stride", type=int, default=1)
    p.add_argument("--sort-every", type=int, default=None,
                   help="re-sort by grid tile every k output segments, 0 never (default: the "
                        "measured best for the cached RK4 kernels, 10 on cfg1 and 0 on cfg2 and "
                        "foram, whose 3D kernel runs faster on the generators' random order "
                        "than on the tile order; 1 elsewhere)")
    p.add_argument("--cpu-baseline", type=int, default=1)
    p.add_argument("--cpu-sample-stride", type=int, default=10,
                   help="cfg1: the oracle's CPU timing follows every k-th particle for the "
                        "whole run (about 10 s on 16 cores at k = 10)")
    p.add_argument("--cpu-1thread-stride", type=int, default=16,
                   help="the one-thread oracle timing follows every k-th particle of the "
                        "all-core sample")
    p.add_argument("--train-segments", type=int, default=50_000_000)
    p.add_argument("--train-iters", type=int, default=12_000)
    p.add_argument("--residual-m", default="50",
                   help="comma-separated residual thresholds in metres (cfg4)")
    p.add_argument("--stencil-cache", type=int, default=None,
                   help="1: stencil cache kernels (default for RK4); 0: gather at "
                        "every stage (default for RKF45, whose long steps leave the cell often)")
    p.add_argument("--kernel", default="rk4", choices=["rk4", "rkf45"],
                   help="cfg1: the integrator (rkf45: adaptive steps |dt| 2^e)")
    p.add_argument("--rkf-tol", type=float, default=1e-3, help="RKF45 tolerance, m per step")
    p.add_argument("--rkf-min-exp", type=int, default=-6)
    p.add_argument("--rkf-max-exp", type=int, default=5)
    p.add_argument("--kh", type=float, default=0.0,
                   help="cfg1: Brownian diffusivity in m^2/s (0: plain RK4, the benchmark)")
    p.add_argument("--calibrate-copy", type=float, default=0.0,
                   help="first copy this many GB device-to-device (a plain copy kernel of "
                        "known size, to scale hardware byte counters)")
    p.add_argument("--error-stride", type=int, default=100,
                   help="cfg2: records and the oracle's error report on ids = 0 mod this "
                        "(0 = no records, no error report)")
    p.add_argument("--graph", type=int, default=1,
                   help="cfg3: 1 = each output segment of the batched run is captured into a "
                        "HIP graph and launched as one (0: direct launches)")
    p.add_argument("--error-report", type=int, default=1,
                   help="cfg2: 0 = take the records but skip the oracle's error report")
    p.add_argument("--host-stream", type=int, default=0,
                   help="cfg2: 1 = push every snapshot from pinned host memory (PCIe) "
                        "instead of from HBM, and report the end-to-end rate")
    a = p.parse_args()
    if a.sort_every is None:
        cached_rk4 = a.kernel == "rk4" and a.stencil_cache != 0
        a.sort_every = SORT_EVERY.get(a.config, 1) if cached_rk4 else 1
    return a


# default sort cadence of the cached RK4 runs (output segments between sorts, 0 never)
SORT_EVERY = {"cfg1": 10, "cfg2": 0, "foram": 0}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_oracle(fs, w, ids, nsteps, threads):
    """The FP64 oracle, as it stands, advancing the particles `ids` of workload w by
    nsteps steps on `threads` host threads; returns (particle-steps, seconds, state)."""
    from oracle import oracle as O
    z = None if w.depth0 is None else w.depth0[ids]
    st = O.make_state(w.lon0[ids], w.lat0[ids], z, pid=ids.astype(np.uint32), t_org=w.t0)
    t = time.perf_counter()
    rc = O.advance(fs, st, w.dt, nsteps, nthreads=threads)
    el = time.perf_counter() - t
    assert rc == 0
    return st.psteps, el, st


def cpu_baseline(w, stride: int, stride1: int, nsteps=None, fs=None):
    """The FP64 oracle on every `stride`-th particle of the workload for the whole run
    on all host cores, and on every (stride * stride1)-th particle on one core."""
    from oracle import oracle as O
    fs = fs or O.OracleFieldSet.from_workload(w)
    nsteps = w.nsteps if nsteps is None else nsteps
    threads = O.max_threads()
    ids = np.arange(0, w.n, stride)
    ps_all, el_all, _ = time_oracle(fs, w, ids, nsteps, threads)
    ids1 = np.arange(0, w.n, stride * stride1)
    ps_1, el_1, _ = time_oracle(fs, w, ids1, nsteps, 1)
    return dict(value=ps_all / el_all, unit="particle-steps/s", cores=threads, kind="oracle",
                sample=f"every {stride}th particle ({ids.size}) for the full {nsteps} steps: "
                       f"{ps_all} particle-steps in {el_all:.2f} s on {threads} threads; one "
                       f"thread: every {stride * stride1}th particle ({ids1.size}), {ps_1} "
                       f"particle-steps in {el_1:.2f} s",
                value_1thread=ps_1 / el_1, cpu_model=cpu_model(), nproc=os.cpu_count())


def _advect_digest():
    """sha256 of advect.hip's code: `//` comments and whitespace are dropped first, so
    that an edit to the comments alone keeps the counter record."""
    import hashlib
    import re
    src = os.path.join(ROOT, "paper_1707_05163_amd", "csrc", "advect.hip")
    with open(src, encoding="utf-8") as f:
        text = f.read()
    code = re.sub(r"//[^\n]*", "", text)
    code = re.sub(r"\s+", " ", code).strip()
    return hashlib.sha256(code.encode()).hexdigest()


def _counters_valid(mode, default_workload):
    return (default_workload and mode in COUNTERS
            and COUNTERS["advect_sha256"] == _advect_digest())


def measured_traffic(mode, default_workload):
    """HBM bytes per launch of the dominant kernel from the recorded counter passes,
    or None (other workload, or the kernel source changed since they were taken)."""
    if not _counters_valid(mode, default_workload):
        return None
    fetch_kib, write_kib = COUNTERS[mode]
    return (fetch_kib * FETCH_SCALE + write_kib * WRITE_SCALE) * 1024.0


def measured_counters(mode, default_workload, steps_per_launch, avg_launch_s):
    """The counter record of the dominant kernel (HBM bytes per launch, L2 hit rate, L2
    requests per particle-step, VALU and SALU issue against the issue peak, the
    latter over the live launch time), or None as for measured_traffic."""
    t = measured_traffic(mode, default_workload)
    l2 = COUNTERS.get(mode + "_l2")
    sq = COUNTERS.get(mode + "_sq")
    if t is None or l2 is None or sq is None:
        return None
    hit, miss = l2
    valu, salu = sq
    return {"source": COUNTER_SOURCE, "hbm_bytes_per_launch": round(t),
            "hbm_frac": round(t / avg_launch_s / 1e9 / HBM_PEAK_GBS, 4),
            "l2_hit_rate": round(hit / (hit + miss), 4),
            "l2_requests_per_particle_step": round((hit + miss) / steps_per_launch, 5),
            "valu_per_particle_step": round(valu * 64 / steps_per_launch, 1),
            "salu_per_particle_step": round(salu * 64 / steps_per_launch, 1),
            "valu_issue_frac": round(valu / avg_launch_s / VALU_ISSUE_PEAK, 4),
            "salu_issue_frac": round(salu / avg_launch_s / VALU_ISSUE_PEAK, 4)}


def roofline(steps_per_launch, avg_launch_s, bytes_per_step, flops_per_step,
             traffic_bytes=None):
    """Roofline of the dominant kernel and the algorithmic-byte figures beside it.

    `roofline`: the method's algorithmic FP64 flops per launch over the HIP-event
    launch time, against the FP64 vector peak ("alu": with the per-lane stencil cache
    the kernels are bound by instruction issue and latency, not by HBM); `traffic`
    is the counted HBM bytes per launch over the same time, in GB/s, when a counter
    record matches the source.  `alg_bytes`: the method's stencil and state bytes per
    launch over the launch time against the HBM peak; above 1 it counts reuse of one
    stencil across many steps, which `reuse_factor` (algorithmic over counted bytes)
    states."""
    hbm_ach = steps_per_launch * bytes_per_step / avg_launch_s / 1e9
    alu_ach = steps_per_launch * flops_per_step / avg_launch_s / 1e12
    traffic = None if traffic_bytes is None else round(traffic_bytes / avg_launch_s / 1e9, 2)
    roof = {"bound": "alu", "achieved": round(alu_ach, 3), "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": round(alu_ach / FP64_VECTOR_PEAK_TFLOPS, 4),
            "traffic": traffic, "traffic_unit": "GB/s (counted HBM bytes, counter record)",
            "flops_per_particle_step": flops_per_step}
    alg = {"achieved": round(hbm_ach, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "alg_bytes_frac": round(hbm_ach / HBM_PEAK_GBS, 4),
           "bytes_per_particle_step": round(bytes_per_step, 3),
           "reuse_factor": None if traffic_bytes is None else
           round(steps_per_launch * bytes_per_step / traffic_bytes, 2)}
    return roof, alg


def great_circle_km(lon1, lat1, lon2, lat2):
    R = 111120.0 * 180.0 / np.pi / 1000.0
    p1, p2 = np.deg2rad(lat1), np.deg2rad(lat2)
    dl = np.deg2rad(lon2 - lon1)
    h = np.sin((p2 - p1) / 2) ** 2 + np.cos(p1) * np.cos(p2) * np.sin(dl / 2) ** 2
    return 2 * R * np.arcsin(np.sqrt(np.clip(h, 0, 1)))


def main_cfg2(a):
    """3D: 10M particles on 3600 x 1800 x 50, 11 daily snapshots built in HBM (or, with
    --host-stream 1, held in host memory and pushed over PCIe) and streamed through a
    three-slot ring (two resident, one being converted), the paper's
    execute-one-day-then-advancetime loop (Sect. 3.1, Sect. 3.4)."""
    import torch
    from paper_1707_05163_amd import FieldSet, ParticleSet
    from synthetic import configs as SC

    torch.cuda.set_device(0)
    n = a.particles if a.particles is not None else 10_000_000
    w = SC.cfg2_global_3d(n_particles=n)
    days = min(a.days if a.days is not None else 10, w.fields.nt - 1)
    host = bool(a.host_stream)
    print(f"[bench] workload {w.name}: {w.n} particles x {days * 144} steps, "
          f"{w.fields.nt} snapshots, building fields in {'host memory' if host else 'HBM'}",
          file=sys.stderr, flush=True)
    cache = {}
    snaps = [SC.cfg2_snapshot_torch(w, s, "cuda", cache) for s in range(w.fields.nt)]
    del cache
    if host:  # the same values, held in (pageable) host memory
        snaps = [tuple(x.cpu().numpy() for x in sn) for sn in snaps]
        torch.cuda.empty_cache()
    lon0 = torch.from_numpy(w.lon0).cuda()
    lat0 = torch.from_numpy(w.lat0).cuda()
    dep0 = torch.from_numpy(w.depth0).cuda()
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    stride = a.error_stride if a.error_stride > 0 else 0
    total = 0.0
    psteps = 0
    kms = 0.0
    launches = 0
    last = None
    for it in range(a.warmup + a.steps):
        fs = FieldSet(w.grid.lon, w.grid.lat, w.grid.depth, "spherical", a.dtype, 3, 0.0)
        ps = ParticleSet(fs, lon0, lat0, dep0, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # the snapshots are complete before the timed region, so their pushes need no
        # ordering after the compute stream (stream 0): the upload and conversion of day
        # d + 2 run on the field set's side stream while day d is advected, into the
        # ring slot day d no longer reads; the execute of day d + 1 waits for them
        fs.push_snapshot(w.fields.times[0], *snaps[0], stream=0)
        fs.push_snapshot(w.fields.times[1], *snaps[1], stream=0)
        for d in range(days):
            ps.execute(86400.0, w.dt, 86400.0, output_stride=stride, sort_every=a.sort_every,
                       profile=it >= a.warmup, stencil_cache=bool(a.stencil_cache),
                       stream=stream)
            if d + 2 < w.fields.nt:
                fs.push_snapshot(w.fields.times[d + 2], *snaps[d + 2], stream=0)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(f"[bench] step {it}: {el * 1e3:.1f} ms", file=sys.stderr, flush=True)
        if it >= a.warmup:
            total += el
            c, _ = ps.status()
            psteps += c["particle_steps"]
            ms, k = ps.timing()
            kms += ms
            launches += k
        if last is not None:
            last[0].close()
            last[1].close()
        last = (ps, fs)
    rate = psteps / total
    avg_launch_s = kms / 1e3 / launches
    spl = psteps / launches
    S = 144
    half = a.dtype != "f32"
    bytes_per_step = (96 if half else 192) + 56.0 / S
    default = (n == 10_000_000 and days == 10 and a.dtype == "f32" and not host
               and a.stencil_cache == 1 and a.sort_every == SORT_EVERY["cfg2"]
               and a.error_stride == 100)
    roof, alg = roofline(spl, avg_launch_s, bytes_per_step, FLOPS_3D_STEP,
                         measured_traffic("cfg2", default))
    out = {
        "metric": "RK4 particle-steps/s", "value": rate, "unit": "particle-steps/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": total / a.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if a.dtype == "f32" else "f64+" + a.dtype,
        "data": "synthetic",
        "config": {"workload": f"cfg2_3d_3600x1800x50_{w.n}_fp32_fields_fp64_positions"
                   if a.dtype == "f32" else f"cfg2_3d_3600x1800x50_{w.n}_{a.dtype}_fields",
                   "grid": "3600x1800x50", "snapshots": w.fields.nt, "ring_slots": 3,
                   "snapshot_source": "host (PCIe)" if host else "HBM",
                   "particles": w.n, "rk4_steps": days * 144, "dt_s": w.dt,
                   "field_dtype": a.dtype, "positions": "f64",
                   "stencil_cache": a.stencil_cache, "sort_every": a.sort_every,
                   "record_stride": stride},
        "roofline": roof, "alg_bytes": alg,
        "counters": measured_counters("cfg2", default, spl, avg_launch_s),
        "kernel": {"name": "k_advect3d" if a.stencil_cache else "k_advect", "launches": launches,
                   "avg_launch_ms": round(avg_launch_s * 1e3, 4),
                   "particle_steps_per_launch": spl,
                   "kernel_share_of_step": round(kms / 1e3 / total, 4),
                   "kernel_only_particle_steps_per_s": spl / avg_launch_s},
    }
    if stride and a.error_report:
        # error in km against the FP64 oracle on the unquantised float32 fields, at
        # every output time, on the recorded subset ids = 0 mod stride
        from oracle import oracle as O
        print("[bench] oracle on the error subset", file=sys.stderr, flush=True)
        recs = last[0].records()
        ids = np.arange(0, w.n, stride)
        shape = (days + 1,) + tuple(np.shape(snaps[0][0]))
        U, V, W = (np.empty(shape, np.float32) for _ in range(3))
        for q in range(days + 1):
            for arr, v in ((U, 0), (V, 1), (W, 2)):
                x = snaps[q][v]
                arr[q] = x if isinstance(x, np.ndarray) else x.cpu().numpy()
        ofs = O.OracleFieldSet(w.grid.lon, w.grid.lat, w.grid.depth, w.fields.times[: days + 1],
                               U, V, W, spherical=True)
        st = O.make_state(w.lon0[ids], w.lat0[ids], w.depth0[ids], pid=ids.astype(np.uint32))
        threads = O.max_threads()
        t = time.perf_counter()
        orecs = O.run(ofs, st, w.dt, days * 86400.0, 86400.0, nthreads=threads)
        ot = time.perf_counter() - t
        per_day = []
        for m, o in enumerate(orecs):
            both = (o["status"] == 0) & (recs["status"][m] == 0)
            km = great_circle_km(recs["lon"][m][both], recs["lat"][m][both], o["lon"][both],
                                 o["lat"][both])
            dz = np.abs(recs["depth"][m][both] - o["depth"][both])
            per_day.append({"day": m, "median": float(np.median(km)),
                            "p95": float(np.percentile(km, 95)), "max": float(km.max()),
                            "depth_max_m": float(dz.max()),
                            "status_mismatch": int((o["status"] != recs["status"][m]).sum())})
        fin = per_day[-1]
        out["error_km_vs_fp64_oracle"] = {
            "subset": f"ids = 0 mod {stride} ({ids.size})", "median": fin["median"],
            "p95": fin["p95"], "max": fin["max"], "depth_max_m": fin["depth_max_m"],
            "status_mismatch": fin["status_mismatch"], "per_output_time": per_day}
        if a.cpu_baseline:
            ids1 = ids[:: a.cpu_1thread_stride]
            ps1, el1, _ = time_oracle(ofs, w, ids1, days * 144, 1)
            out["cpu_baseline"] = dict(
                value=st.psteps / ot, unit="particle-steps/s", cores=threads, kind="oracle",
                sample=f"ids = 0 mod {stride} ({ids.size}) for {days * 144} steps: "
                       f"{st.psteps} particle-steps in {ot:.2f} s on {threads} threads; one "
                       f"thread: ids = 0 mod {stride * a.cpu_1thread_stride} ({ids1.size}), "
                       f"{ps1} particle-steps in {el1:.2f} s",
                value_1thread=ps1 / el1, cpu_model=cpu_model(), nproc=os.cpu_count())
    print(json.dumps(out), flush=True)


def main_foram(a):
    """The worked example's chain (sinking, age, temperature sample, RK4_3D) on the
    synthetic stand-in for the foraminifera footprint experiment: 0.1 degree
    regional grid, 54 levels, 3-day snapshots with temperature, particles released
    at 2,440 m off Cape Town and tracked backward for 42 days with daily records."""
    import torch
    from paper_1707_05163_amd import FieldSet, ParticleSet
    from synthetic import configs as SC

    torch.cuda.set_device(0)
    n = a.particles if a.particles is not None else 1_000_000
    w = SC.foram_footprint(n_particles=n)
    m = w.meta
    print(f"[bench] foram: {w.n} particles x {w.nsteps} steps backward, "
          f"{w.grid.nx}x{w.grid.ny}x{w.grid.nz}, {w.fields.nt} snapshots", file=sys.stderr,
          flush=True)
    fs = FieldSet.from_workload(w)
    stream = torch.cuda.current_stream()
    runtime = w.nsteps * abs(w.dt)
    psets = [ParticleSet(fs, w.lon0, w.lat0, w.depth0, t0=w.t0)
             for _ in range(a.warmup + a.steps)]
    torch.cuda.synchronize()

    def step(ps, profile):
        ps.execute(runtime, w.dt, DAY_S, output_stride=1, sink_speed=m["sink_speed"],
                   dwell_depth=m["dwell_depth"], maxage=m["maxage"], sample=True,
                   sort_every=a.sort_every, profile=profile, stream=stream)

    for i in range(a.warmup):
        step(psets[i], False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        step(psets[a.warmup + i], True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    psteps = kms = launches = 0
    for ps in psets[a.warmup:]:
        c, st = ps.status()
        psteps += c["particle_steps"]
        ms, k = ps.timing()
        kms += ms
        launches += k
    aged = int(((st & 8) != 0).sum())
    avg_launch_s = kms / 1e3 / launches
    spl = psteps / launches
    # per step: the 3D RK4 stencil (192 B) plus the tracer's trilinear stencil at two
    # snapshots (8 x 2 x 4 B) and the state (position, temp, age, status) per record
    bytes_per_step = 192 + 64 + 72.0 / (DAY_S / abs(w.dt))
    roof, alg = roofline(spl, avg_launch_s, bytes_per_step, FLOPS_3D_STEP + 40)
    out = {
        "metric": "RK4 particle-steps/s", "value": psteps / el, "unit": "particle-steps/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup, "ms_per_step": el / a.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "grid": f"{w.grid.nx}x{w.grid.ny}x{w.grid.nz}",
                   "snapshots": w.fields.nt, "particles": w.n, "days": 42, "dt_s": w.dt,
                   "kernels": "sink+age+sample+RK4_3D", "maxage_days": 30},
        "roofline": roof, "alg_bytes": alg,
        "kernel": {"name": "k_advect3d (stencil cache, with the worked-example kernels)",
                   "launches": launches, "avg_launch_ms": round(avg_launch_s * 1e3, 4),
                   "particle_steps_per_launch": spl,
                   "kernel_share_of_step": round(kms / 1e3 / el, 4)},
        "aged_at_end": aged,
    }
    print(json.dumps(out), flush=True)


def main_cfg3(a):
    """64 uneven 2D runs (grids 64^2..1024^2, 1k..2M particles) with the Brownian
    term, advanced together by the batched persistent launch; the launch shape
    comes from the autotuner.  Also times the runs one after the other."""
    import torch
    from paper_1707_05163_amd import ParticleSet, FieldSet, autotune_batch, execute_batch
    from synthetic import configs as SC

    torch.cuda.set_device(0)
    ws = SC.cfg3_ensemble()
    ntot = sum(w.n for w in ws)
    print(f"[bench] cfg3: {len(ws)} runs, {ntot} particles, grids "
          f"{min(w.grid.nx for w in ws)}..{max(w.grid.nx for w in ws)}", file=sys.stderr,
          flush=True)
    fss = [FieldSet.from_workload(w) for w in ws]
    dev0 = [(torch.from_numpy(w.lon0).cuda(), torch.from_numpy(w.lat0).cuda()) for w in ws]
    stream = torch.cuda.current_stream()
    runtime = ws[0].nsteps * ws[0].dt

    def fresh():
        ps = [ParticleSet(f, x, y, stream=stream) for f, (x, y) in zip(fss, dev0)]
        torch.cuda.synchronize()
        return ps

    opts = [ParticleSet.opts(Kh=w.Kh, run_id=w.run_id, profile=True) for w in ws]
    cache = os.environ.get("LP_AUTOTUNE_CACHE", "/tmp/lp_autotune.json")
    ps = fresh()
    t = time.perf_counter()
    best = autotune_batch(ps, ws[0].dt, 24, opts, cache)
    tune_s = time.perf_counter() - t
    for o in opts:
        o.stencil_cache, o.sort_every = best["stencil_cache"], best["sort_every"]
        o.sort_steps = best["sort_steps"]
        o.graph = a.graph
    total = 0.0
    psteps = 0
    kms = 0.0
    launches = 0
    for it in range(a.warmup + a.steps):
        ps = fresh()
        t0 = time.perf_counter()
        execute_batch(ps, runtime, ws[0].dt, 86400.0, opts, block=best["block"], stream=stream)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        print(f"[bench] step {it}: {el * 1e3:.1f} ms", file=sys.stderr, flush=True)
        if it >= a.warmup:
            total += el
            psteps += sum(p.status()[0]["particle_steps"] for p in ps)
            ms, k = ps[0].timing()
            kms += ms
            launches += k
    # one more batched run with the other launch mode (graphs or direct launches)
    for o in opts:
        o.graph = 0 if a.graph else 1
    ps = fresh()
    t0 = time.perf_counter()
    execute_batch(ps, runtime, ws[0].dt, 86400.0, opts, block=best["block"], stream=stream)
    torch.cuda.synchronize()
    other_mode_ms = (time.perf_counter() - t0) * 1e3
    # the same runs one after the other, each with its own launches
    ps = fresh()
    standalone = 0.0
    for p, w in zip(ps, ws):
        t0 = time.perf_counter()
        p.execute(runtime, w.dt, 86400.0, Kh=w.Kh, run_id=w.run_id, stream=stream)
        torch.cuda.synchronize()
        standalone += time.perf_counter() - t0
    rate = psteps / total
    avg_launch_s = kms / 1e3 / launches
    spl = psteps / launches
    roof, alg = roofline(spl, avg_launch_s, STENCIL_BYTES_2D_F32 + STATE_BYTES_2D / 288.0,
                         FLOPS_2D_STEP + FLOPS_BROWNIAN)
    out = {
        "metric": "RK4 particle-steps/s", "value": rate, "unit": "particle-steps/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": total / a.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": "cfg3_ensemble_64_runs", "runs": len(ws), "particles": ntot,
                   "rk4_steps": ws[0].nsteps, "dt_s": ws[0].dt, "Kh": ws[0].Kh,
                   "autotuned": best, "autotune_s": round(tune_s, 3)},
        "roofline": roof, "alg_bytes": alg,
        "kernel": {"name": "graph of one output segment (sorts, k_advect2d_batch, compactions, "
                           "records)" if a.graph else "k_advect2d_batch", "launches": launches,
                   "avg_launch_ms": round(avg_launch_s * 1e3, 4),
                   "particle_steps_per_launch": spl},
        "batched_makespan_ms": total / a.steps * 1e3,
        "graph": a.graph,
        ("batched_direct_launch_ms" if a.graph else "batched_graph_ms"): other_mode_ms,
        "standalone_sum_ms": standalone * 1e3,
    }
    print(json.dumps(out), flush=True)


def main_cfg4(a):
    """Learned flow map on the 10-day periodic 0.25 degree field: train on RK4
    segments, then advance 4M particles for 30 days with the network where it passes
    the residual check and RK4 elsewhere; compare with fine (300 s) and coarse
    (3600 s) RK4, and measure every final position against the FP64 oracle."""
    import torch
    from paper_1707_05163_amd import FieldSet, ParticleSet, Surrogate
    from synthetic import configs as SC
    from oracle import oracle as O

    torch.cuda.set_device(0)
    n = a.particles if a.particles is not None else 4_000_000
    w = SC.cfg4_surrogate_field(n_particles=n)
    fs = FieldSet.from_workload(w)
    lon0 = torch.from_numpy(w.lon0).cuda()
    lat0 = torch.from_numpy(w.lat0).cuda()
    stream = torch.cuda.current_stream()
    days = a.days if a.days is not None else 30
    runtime = days * 86400.0
    print(f"[bench] cfg4: training on {a.train_segments} segments, {a.train_iters} steps",
          file=sys.stderr, flush=True)
    model = Surrogate(seed=1)
    tr = model.train(fs, n_segments=a.train_segments, iterations=a.train_iters,
                     round_size=1_000_000, batch=4096, lr=1e-3, stream=stream)
    print(f"[bench] train: {tr}", file=sys.stderr, flush=True)

    def timed(fn):
        ps = ParticleSet(fs, lon0, lat0, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        extra = fn(ps)
        torch.cuda.synchronize()
        return ps, time.perf_counter() - t0, extra

    fine_ps, fine_s, _ = timed(lambda p: p.execute(runtime, w.dt, stream=stream))
    coarse_ps, coarse_s, _ = timed(lambda p: p.execute(runtime, 3600.0, stream=stream))
    thresholds = [float(x) for x in str(a.residual_m).split(",")]
    surr = []
    for thr in thresholds:
        ps_, s_, st_ = timed(lambda p: p.execute_surrogate(model, runtime, dt=w.dt,
                                                           residual_m=thr, stream=stream))
        surr.append((thr, ps_, s_, st_))
        print(f"[bench] residual {thr} m: {s_:.3f} s {st_}", file=sys.stderr, flush=True)
    print(f"[bench] fine {fine_s:.3f} s, coarse {coarse_s:.3f} s", file=sys.stderr, flush=True)
    # errors against the FP64 oracle on a subset
    ids = np.arange(0, n, a.cpu_sample_stride * 40)
    ofs = O.OracleFieldSet.from_workload(w)
    st = O.make_state(w.lon0[ids], w.lat0[ids], pid=ids.astype(np.uint32))
    t0 = time.perf_counter()
    assert O.advance(ofs, st, w.dt, int(round(runtime / w.dt)), nthreads=O.max_threads()) == 0
    ot = time.perf_counter() - t0
    errs = {}
    runs = [("fine_rk4", fine_ps), ("coarse_rk4", coarse_ps)]
    runs += [(f"surrogate_{thr:g}m", p) for thr, p, _, _ in surr]
    for name, ps in runs:
        g = ps.get()
        _, stt = ps.status()
        both = (stt[ids] == 0) & (st.status == 0)
        km = great_circle_km(g["lon"][ids][both], g["lat"][ids][both], st.x[both], st.y[both])
        errs[name] = {"median_km": float(np.median(km)), "p95_km": float(np.percentile(km, 95)),
                      "max_km": float(km.max()), "compared": int(both.sum()),
                      "status_mismatch": int((stt[ids] != st.status).sum())}
    steps = n * int(round(runtime / w.dt))
    out = {
        "metric": "surrogate speedup over plain FP32-field RK4 at equal particle count",
        "value": fine_s / surr[0][2], "unit": "x", "n_gpus": 1, "steps": 1, "warmup": 0,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "bf16-mfma+f64", "data": "synthetic",
        "config": {"workload": w.name, "particles": n, "days": days, "segment_steps": 24,
                   "dt_s": w.dt, "residual_m": thresholds},
        "times_s": dict({"fine_rk4": fine_s, "coarse_rk4": coarse_s},
                        **{f"surrogate_{thr:g}m": s_ for thr, _, s_, _ in surr}),
        "fine_rk4_particle_steps_per_s": steps / fine_s,
        "surrogate_stats": {f"{thr:g}m": st_ for thr, _, _, st_ in surr}, "training": tr,
        "error_vs_fp64_oracle": errs,
        "oracle_sample": f"every {a.cpu_sample_stride * 4}th particle ({ids.size}) for "
                         f"{int(round(runtime / w.dt))} steps in {ot:.1f} s",
    }
    print(json.dumps(out), flush=True)


def report_rkf45(a, w, el, psteps, retried, kms, launches, psets):
    """Bench line of the adaptive RKF45 run on the cfg1 workload: accepted steps per
    second, with the simulated particle-days per second beside it (the RK4 line's
    1M particles x 30 days of the same workload)."""
    avg_launch_s = kms / 1e3 / launches
    attempts = psteps + retried
    per_launch = attempts / launches
    bytes_per_attempt = STENCIL_BYTES_RKF45_2D_F32 + STATE_BYTES_RKF45_2D * w.n / per_launch
    roof, alg = roofline(per_launch, avg_launch_s, bytes_per_attempt, FLOPS_RKF45_ATTEMPT_2D)
    ex = np.concatenate([p.step_exponents() for p in psets])
    days = w.nsteps * w.dt / 86400.0
    out = {
        "metric": "RKF45 accepted particle-steps/s", "value": psteps / el,
        "unit": "particle-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": el / a.steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.name, "grid": f"{w.grid.nx}x{w.grid.ny}",
                   "snapshots": w.fields.nt, "particles": w.n, "days": days,
                   "base_dt_s": w.dt, "tol_m": a.rkf_tol, "exp_range": [a.rkf_min_exp,
                                                                          a.rkf_max_exp],
                   "stencil_cache": a.stencil_cache},
        "roofline": roof, "alg_bytes": alg,
        "kernel": {"name": "k_rkf45_2d" if a.stencil_cache else "k_rkf45",
                   "launches": launches, "avg_launch_ms": round(avg_launch_s * 1e3, 4),
                   "attempts_per_launch": per_launch,
                   "kernel_share_of_step": round(kms / 1e3 / el, 4)},
        "retried_fraction": retried / max(attempts, 1),
        "particle_days_per_s": w.n * days * a.steps / el,
        "final_step_exponents": {int(k): int(v) for k, v in
                                 zip(*np.unique(ex, return_counts=True))},
    }
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.stencil_cache is None:
        a.stencil_cache = 0 if a.kernel == "rkf45" else 1
    if a.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1",
                          "n_gpus": a.gpus}))
        sys.exit(2)
    if a.calibrate_copy > 0:
        import torch
        n = int(a.calibrate_copy * 1e9) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {n * 4} bytes", file=sys.stderr, flush=True)
        del src, dst
    if a.config == "cfg2":
        return main_cfg2(a)
    if a.config == "cfg3":
        return main_cfg3(a)
    if a.config == "cfg4":
        return main_cfg4(a)
    if a.config == "foram":
        return main_foram(a)
    import torch
    from paper_1707_05163_amd import FieldSet, ParticleSet
    from synthetic import configs as SC

    torch.cuda.set_device(0)
    days = a.days if a.days is not None else 30
    n = a.particles if a.particles is not None else 1_000_000
    nsteps = days * 288
    w = SC.cfg1_global_eddies(n_particles=n, nsteps=nsteps)
    print(f"[bench] workload {w.name}: {w.n} particles x {w.nsteps} steps, "
          f"{w.fields.nt} snapshots {w.grid.nx}x{w.grid.ny}", file=sys.stderr, flush=True)
    fs = FieldSet.from_workload(w, dtype=a.dtype)
    lon0 = torch.from_numpy(w.lon0).cuda()
    lat0 = torch.from_numpy(w.lat0).cuda()
    stream = torch.cuda.current_stream()
    psets = [ParticleSet(fs, lon0, lat0, stream=stream) for _ in range(a.warmup + a.steps)]
    torch.cuda.synchronize()
    runtime = w.nsteps * w.dt

    def step(ps, profile):
        ps.execute(runtime, w.dt, w.outputdt, output_stride=a.output_stride,
                   sort_every=a.sort_every, profile=profile,
                   stencil_cache=bool(a.stencil_cache), kernel=a.kernel, tol=a.rkf_tol,
                   min_exp=a.rkf_min_exp, max_exp=a.rkf_max_exp, Kh=a.kh, stream=stream)

    for i in range(a.warmup):
        step(psets[i], False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(a.steps):
        step(psets[a.warmup + i], True)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0

    psteps = 0
    retried = 0
    kms = 0.0
    launches = 0
    for ps in psets[a.warmup:]:
        c, _ = ps.status()
        psteps += c["particle_steps"]
        retried += c["rejected_steps"]
        ms, k = ps.timing()
        kms += ms
        launches += k
    rate = psteps / el
    if a.kernel == "rkf45":
        return report_rkf45(a, w, el, psteps, retried, kms, launches, psets[a.warmup:])
    avg_launch_s = kms / 1e3 / launches
    steps_per_launch = psteps / launches
    S = w.outputdt / w.dt
    bytes_per_step = STENCIL_BYTES_2D_F32 * (0.5 if a.dtype != "f32" else 1.0) + STATE_BYTES_2D / S
    default = (n == 1_000_000 and days == 30 and a.dtype == "f32"
               and a.stencil_cache == 1 and a.sort_every == SORT_EVERY["cfg1"]
               and a.output_stride == 1 and a.kh == 0.0)
    roof, alg = roofline(steps_per_launch, avg_launch_s, bytes_per_step, FLOPS_2D_STEP,
                         measured_traffic("cfg1", default))
    out = {
        "metric": "RK4 particle-steps/s",
        "value": rate,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": el / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if a.dtype == "f32" else "f64+" + a.dtype,
        "data": "synthetic",
        "config": {"workload": w.name, "grid": f"{w.grid.nx}x{w.grid.ny}", "snapshots": w.fields.nt,
                   "particles": w.n, "rk4_steps": w.nsteps, "dt_s": w.dt,
                   "field_dtype": a.dtype, "output_stride": a.output_stride,
                   "sort_every": a.sort_every, "Kh": a.kh},
        "roofline": roof,
        "alg_bytes": alg,
        "counters": measured_counters("cfg1", default, steps_per_launch, avg_launch_s),
        "kernel": {"name": "k_advect2d" if a.stencil_cache else "k_advect", "launches": launches,
                   "avg_launch_ms": round(avg_launch_s * 1e3, 4),
                   "particle_steps_per_launch": steps_per_launch,
                   "kernel_share_of_step": round(kms / 1e3 / el, 4)},
    }
    if a.cpu_baseline:
        print("[bench] timing the FP64 oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_sample_stride, a.cpu_1thread_stride)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
