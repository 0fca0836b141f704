"""Benchmark: full time steps of the geodesic-interaction hot path on one GPU.

Default line (the largest single-GPU workload): the Gaussian-bump height
field on [0,10]^2 (316 x 316 cells split on diagonals, 199,712 faces, open
boundary), N = 20,000 particles (face-uniform, barycentric-uniform, seed 3),
harmonic repulsion k = 1, sigma = cutoff = 3 mean edge lengths, Brownian
dynamics kT = 0.1, friction 1, dt = 0.005. A step is one pass of the whole
hot path: Euclidean prefilter, window propagation + target query (geodesic
pairs), force sum, integrator, walk.

Prints ONE JSON line. ``value`` = geodesic neighbour pairs per second over the
timed FP64 steps (inputs resident in device memory); ``particle_steps_per_s``
is the second number of the metric; ``fp32`` is the FP32-mixed leg of the
same workload. ``c3`` holds the batched 16-surface workload (batched
FP32-mixed against single-surface FP64, the throughput target) and ``c5``
the all-pairs Coulomb FIRE iteration on 81,920 faces in both precisions,
each with its own roofline. ``roofline`` is for the dominant kernel (window
propagation), ``update_roofline`` for the force + integrator + walk kernel,
and ``cpu_baseline`` times the CPU oracle on a bounded sample of the same
workload on the host's cores and on one thread.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "geodesic pairs/sec + particle-steps/sec, FP32-mixed vs FP64 on one MI355X at 1e-5 rel err"
FP64_VECTOR_PEAK_TFLOPS = 78.6
FP32_VECTOR_PEAK_TFLOPS = 157.3
HBM_PEAK_GBPS = 8000.0
# algorithmic HBM bytes of one particle's time step in the update kernel
# (force sum, integrator, walk): its row (count 4 B, then per pair distance
# 8 B and tangent 24 B), its state read and written (face 4 B + barycentrics
# 24 B, twice), its velocity read and written (2 x 24 B), and the vertex
# positions and normal (96 B) of every face the walk visits (the start face
# and one per edge crossing)
UPDATE_BYTES_PARTICLE = 4 + 56 + 48 + 96
UPDATE_BYTES_PAIR = 32
UPDATE_BYTES_CROSSING = 96
# algorithmic floating-point work of one window propagation step (C's
# intercept, two child intervals with their frame changes and lower bounds,
# the bend-vertex test); divisions and square roots count as one
FLOPS_PER_WINDOW = 90.0


WORKLOAD_TEXT = {
    "c2": "bumpy sphere (icosphere L5, r=1+0.1 sin4t cos3p), 20480 faces, N=1000, harmonic sigma=cutoff=0.15, "
          "overdamped dt=0.01",
    "c4": "Gaussian-bump height field 10x10, 199712 faces, open boundary, N=20000, harmonic sigma=cutoff=3 mean "
          "edges, Brownian kT=0.1 friction=1 dt=0.005",
}

PMC_NAME = {"c2": "bumpy_sphere_n1000", "c4": "height_field_n20000"}


def pmc_file(workload, precision):
    tag = "fp64" if precision == "fp64" else "fp32mixed"
    return os.path.join(ROOT, "profiles", f"k_geodesic_{PMC_NAME.get(workload, workload)}_{tag}_pmc.json")


def code_hash(texts):
    """sha256 of source code with comments and whitespace removed, so that
    only a change of the code itself counts as a new kernel."""
    import hashlib
    import re
    h = hashlib.sha256()
    for t in texts:
        t = re.sub(r"/\*.*?\*/", " ", t, flags=re.S)
        t = re.sub(r"//[^\n]*", " ", t)
        h.update(" ".join(t.split()).encode())
    return h.hexdigest()


def measured_counters(workload, precision):
    """The committed counter record of k_geodesic on this workload and
    precision (HBM traffic per launch, LDS bandwidth, occupancy), or None
    when there is none or the kernel code differs from the one the counters
    saw."""
    try:
        rec = json.load(open(pmc_file(workload, precision)))
        src = [open(os.path.join(ROOT, f)).read() for f in rec["sources_hashed"]]
    except (OSError, KeyError, ValueError):
        return None
    if code_hash(src) != rec.get("kernel_code_sha256"):
        return None
    return rec


def host_cpu():
    """Cores this process may use and the CPU model (lscpu, else /proc/cpuinfo)."""
    import subprocess
    try:
        nproc = len(os.sched_getaffinity(0))
    except AttributeError:
        nproc = os.cpu_count() or 1
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout
        for ln in out.splitlines():
            if ln.strip().lower().startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except (OSError, subprocess.SubprocessError):
        pass
    if model is None:
        try:
            for ln in open("/proc/cpuinfo"):
                if ln.lower().startswith("model name"):
                    model = ln.split(":", 1)[1].strip()
                    break
        except OSError:
            pass
    return nproc, model


def cpu_baseline(w, budget_s=10.0, max_steps=500, single_sources=64):
    """The FP64 oracle on the host: full steps (pairs, forces, integrator,
    walk) of the same workload for about budget_s seconds on every core the
    process may use, then the pairs of single_sources sources spread over the
    particle range on one thread (the paper's own regime: one core)."""
    import oracle
    nproc, model = host_cpu()
    threads = int(os.environ.get("OMP_NUM_THREADS", nproc))
    om = oracle.OracleMesh(w.mesh.V, w.mesh.T)
    f, b = w.face.copy(), w.bary.copy()
    pairs = 0
    t0 = time.perf_counter()
    steps = 0
    while steps < max_steps and time.perf_counter() - t0 < budget_s:
        f, b, info = oracle.step(om, f, b, w.potential, w.integrator, steps, nthreads=threads)
        pairs += len(info["pairs"].dist)
        steps += 1
    dt = time.perf_counter() - t0
    n = len(w.face)
    # the geodesic stage alone (the GPU's pairs/s counts the whole step; the
    # oracle's force sum and integrators are plain Python loops)
    t2 = time.perf_counter()
    o2 = oracle.geodesic_pairs(om, w.face, w.bary, w.potential["cutoff"], nthreads=threads)
    dt2 = time.perf_counter() - t2
    src = np.unique(np.linspace(0, n - 1, single_sources).round().astype(np.int32))
    reps, p1 = 0, 0
    t1 = time.perf_counter()
    while reps == 0 or time.perf_counter() - t1 < 1.0:
        p1 += len(oracle.geodesic_pairs(om, w.face, w.bary, w.potential["cutoff"], sources=src, nthreads=1).dist)
        reps += 1
    dt1 = time.perf_counter() - t1
    return {"value": pairs / dt, "unit": "pairs/s", "cores": threads, "kind": "oracle",
            "sample": f"first {steps} full FP64 oracle steps (pairs+forces+walk) of the same workload, "
                      f"{dt:.1f} s wall, OpenMP over sources on {threads} threads",
            "particle_steps_per_s": steps * n / dt, "nproc": nproc, "cpu_model": model,
            "pairs_only": {"value": len(o2.dist) / dt2, "unit": "pairs/s", "cores": threads,
                           "sample": f"the geodesic pairs of all {n} sources once, {dt2:.2f} s"},
            "single_thread": {"value": p1 / dt1, "unit": "pairs/s", "cores": 1, "sources_per_s": reps * len(src) / dt1,
                              "sample": f"geodesic pairs of {len(src)} sources spread over the {n} particles, "
                                        f"one thread, {reps} repetitions in {dt1:.2f} s"}}


def _gsim_args(gsim, w):
    p, wi = w.potential, w.integrator
    pot = gsim.potential(p["kind"], p["k"], p["sigma"], p["cutoff"])
    if wi["kind"] == "brownian":
        ig = gsim.integrator("brownian", wi["dt"], 1.0, wi["kT"], wi["friction"], wi["seed"])
    elif wi["kind"] == "overdamped":
        ig = gsim.integrator("overdamped", wi["dt"], wi["mobility"])
    else:
        ig = gsim.integrator(wi["kind"], wi["dt"])
    return pot, ig


def bench_c3(args, gsim, W):
    """16 surfaces (icospheres L3-L6, 12 tori) stepped as one batch (one
    persistent geodesic launch per step, steps replayed from a HIP graph,
    autotuned launch shape) against the plain path: each surface stepped on
    its own, eagerly, in FP64."""
    ws = W.workload("c3")
    steps = args.steps

    def load(ctx):
        mids = []
        for w in ws:
            mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
            ctx.particles_set(mid, w.face, w.bary)
            mids.append(mid)
        return mids

    pots, igs = zip(*[_gsim_args(gsim, w) for w in ws])

    def batched(prec, tune):
        ctx = gsim.Context(0, prec)
        mids = load(ctx)
        pick = ctx.autotune(mids, pots, igs, reps=3) if tune else None
        ctx.step_batched(mids, pots, igs, max(args.warmup, 2))  # also captures the graph of `warmup` steps
        ctx.tune(graph_steps=steps)
        ctx.step_batched(mids, pots, igs, steps)  # capture of the timed graph
        for m, w in zip(mids, ws):
            ctx.particles_set(m, w.face, w.bary)
        ctx.synchronize()
        c0 = ctx.counters()["cum_pairs"]
        t0 = time.perf_counter()
        ctx.step_batched(mids, pots, igs, steps)
        ctx.synchronize()
        dt = time.perf_counter() - t0
        pairs = ctx.counters()["cum_pairs"] - c0
        # instrumented pass (stage events, no graph) for the kernel times
        for m, w in zip(mids, ws):
            ctx.particles_set(m, w.face, w.bary)
        ctx.timing(True)
        ctx.step_batched(mids, pots, igs, min(steps, 10))
        ctx.synchronize()
        stages = {k: v for k in ("prefilter", "geodesic", "update", "commit") for v, n in [ctx.timing_get(k)] if n}
        cnt = ctx.counters()
        ctx.timing(False)
        ctx.close()
        return dict(pairs_per_s=pairs / dt, ms_per_step=1e3 * dt / steps, pairs_per_step=pairs / steps,
                    stage_ms=stages, windows_per_step=cnt["cum_windows"] / max(cnt["cum_passes"], 1), tuned=pick)

    def single(prec):
        ctx = gsim.Context(0, prec)
        ctx.tune(graph_steps=0)
        mids = load(ctx)
        for m, p, g in zip(mids, pots, igs):
            ctx.step(m, p, g, max(args.warmup, 1))
        for m, w in zip(mids, ws):
            ctx.particles_set(m, w.face, w.bary)
        ctx.synchronize()
        c0 = ctx.counters()["cum_pairs"]
        t0 = time.perf_counter()
        for m, p, g in zip(mids, pots, igs):
            ctx.step(m, p, g, steps)
        ctx.synchronize()
        dt = time.perf_counter() - t0
        pairs = ctx.counters()["cum_pairs"] - c0
        ctx.close()
        return dict(pairs_per_s=pairs / dt, ms_per_step=1e3 * dt / steps, pairs_per_step=pairs / steps)

    b32 = batched("fp32", True)
    b64 = batched("fp64", True)
    s64 = single("fp64")
    s32 = single("fp32")
    n = sum(len(w.face) for w in ws)
    geo_ms = b32["stage_ms"]["geodesic"]
    achieved = FLOPS_PER_WINDOW * b32["windows_per_step"] / (geo_ms * 1e-3) / 1e12 if geo_ms > 0 else 0.0
    return {
        "metric": METRIC, "value": b32["pairs_per_s"], "unit": "pairs/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": b32["ms_per_step"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic",
        "config": {"workload": "16 surfaces batched: icospheres L3-L6 and 12 tori R=1 r=0.3 (1938-81920 faces), "
                               "N per surface at packing 0.3 in [200,4000] (15033 total), harmonic sigma=cutoff=2 "
                               "mean edges, overdamped dt=0.01 sigma^2; steps replayed from a HIP graph",
                   "n_particles": n, "surfaces": len(ws)},
        "particle_steps_per_s": n * steps / (b32["ms_per_step"] * 1e-3 * steps),
        "batched_fp32": b32, "batched_fp64": b64, "single_surface_fp64": s64, "single_surface_fp32": s32,
        "batched_fp32_over_single_fp64": b32["pairs_per_s"] / s64["pairs_per_s"],
        "roofline": {"bound": "alu", "achieved": achieved, "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP32_VECTOR_PEAK_TFLOPS, "traffic": None, "kernel": "k_geodesic",
                     "per_unit": f"{FLOPS_PER_WINDOW:.0f} flop/window",
                     "units_per_launch": b32["windows_per_step"], "avg_launch_ms": geo_ms},
    }


def bench_torus_nve(args, gsim, W):
    """Cost per velocity-Verlet (NVE) step against N on the aspect-3 benchmark
    torus (4648 faces) for interaction ranges sigma = 1, 1/2, 1/4 and 1/8, the
    setting of the paper's Fig. 3 scaling study (sigma = 1 its main curve);
    steps replayed from HIP graphs, as many as about half a second takes
    (at least 2, at most --steps). The exponent is the least-squares slope of
    log(ms/step) against log N."""
    out = {}
    for sig in (1.0, 0.5, 0.25, 0.125):
        rows = []
        for n in (512, 1024, 2048, 4096, 8192, 16384, 32768):
            w = W.workload(f"torus_nve_{n}_{sig}")
            pot, ig = _gsim_args(gsim, w)
            for prec in ("fp64", "fp32"):
                ctx = gsim.Context(0, prec)
                mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
                ctx.particles_set(mid, w.face, w.bary)
                t0 = time.perf_counter()
                ctx.step(mid, pot, ig, 1)
                ctx.synchronize()
                t1 = time.perf_counter() - t0
                k = max(2, min(args.steps, int(0.5 / max(t1, 1e-5))))
                ctx.tune(graph_steps=k)
                ctx.step(mid, pot, ig, k)  # warm-up, captures the graph
                ctx.synchronize()
                c0 = ctx.counters()["cum_pairs"]
                t0 = time.perf_counter()
                ctx.step(mid, pot, ig, k)
                ctx.synchronize()
                dt = time.perf_counter() - t0
                pairs = ctx.counters()["cum_pairs"] - c0
                ctx.close()
                rows.append({"n": n, "precision": prec, "steps": k, "ms_per_step": 1e3 * dt / k,
                             "pairs_per_step": pairs / k, "pairs_per_s": pairs / dt})
                print(f"[torus_nve] sigma={sig} n={n} {prec}: {1e3 * dt / k:.3f} ms/step ({k} steps)",
                      file=sys.stderr, flush=True)
        fits = {}
        for prec in ("fp64", "fp32"):
            xs = np.log([r["n"] for r in rows if r["precision"] == prec])
            ys = np.log([r["ms_per_step"] for r in rows if r["precision"] == prec])
            fits[prec] = float(np.polyfit(xs, ys, 1)[0])
            big = [r for r in rows if r["precision"] == prec and r["n"] >= 4096]
            fits[prec + "_n_ge_4096"] = float(np.polyfit(np.log([r["n"] for r in big]),
                                                         np.log([r["ms_per_step"] for r in big]), 1)[0])
        out[f"sigma_{sig}"] = {"runs": rows, "exponent": fits}
    return {"workload": "velocity Verlet NVE on the aspect-3 benchmark torus (R=3, r=1, 4648 faces), harmonic "
                        "repulsion of range sigma, dt=0.005, from rest, N = 512 .. 32768", "data": "synthetic",
            "results": out}


def bench_vsweep(args, gsim, W):
    """Cost per velocity-Verlet (NVE) step of N = 100 particles against the
    number of mesh vertices V at fixed span, interaction range span / 10
    (the paper's Sec. 4 mesh-size study): a sphere and tori of aspect ratio 3
    and 20. "submesh": windows pruned at the range (the cutoff kernel, or the
    whole-mesh kernel with the cutoff where a source's patch exceeds the
    cutoff kernel's limits); "full": every source's windows cover the whole
    mesh (no cutoff; the potential still vanishes beyond the range). FP64,
    steps replayed from HIP graphs. The exponent is the least-squares slope of
    log(ms/step) against log V; the full-mesh runs stop at a surface's first
    level whose step takes longer than a few seconds."""
    import math
    out = {}
    for surf, spec in W.VSWEEP.items():
        rows = []
        full_open = True
        for lv in spec["levels"]:
            w = W.workload(f"vsweep_{surf}_{lv}")
            nv = int(len(w.mesh.V))
            for mode in ("submesh", "full"):
                if mode == "full" and not full_open:
                    continue
                cut = w.potential["cutoff"] if mode == "submesh" else math.inf
                pot = gsim.potential("harmonic", 1.0, w.potential["sigma"], cut)
                ig = gsim.integrator("verlet", w.integrator["dt"])
                kernel = "cutoff" if mode == "submesh" else "whole_mesh"
                for attempt in (0, 1):
                    ctx = gsim.Context(0, "fp64")
                    if attempt:
                        ctx.tune(whole_mesh=1)
                        kernel = "whole_mesh"
                    mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
                    ctx.particles_set(mid, w.face, w.bary)
                    try:
                        t0 = time.perf_counter()
                        ctx.step(mid, pot, ig, 1)
                        ctx.synchronize()
                        t1 = time.perf_counter() - t0
                        break
                    except gsim.GsimError as e:
                        ctx.close()
                        if e.status != gsim.E_LIMIT or attempt:
                            raise
                k = max(2, min(10, int(2.0 / max(t1, 1e-4))))
                ctx.tune(graph_steps=k)
                ctx.step(mid, pot, ig, k)  # captures the graph
                ctx.synchronize()
                c0 = ctx.counters()
                t0 = time.perf_counter()
                ctx.step(mid, pot, ig, k)
                ctx.synchronize()
                dt = time.perf_counter() - t0
                c1 = ctx.counters()
                ctx.close()
                ms = 1e3 * dt / k
                rows.append({"level": lv, "V": nv, "faces": int(w.mesh.nf), "mode": mode, "kernel": kernel,
                             "ms_per_step": ms, "steps": k,
                             "pairs_per_step": (c1["cum_pairs"] - c0["cum_pairs"]) / k,
                             "windows_per_step": (c1["cum_windows"] - c0["cum_windows"]) / k})
                print(f"[vsweep] {surf} V={nv} {mode} ({kernel}): {ms:.3f} ms/step", file=sys.stderr, flush=True)
                if mode == "full" and ms > 1500.0:
                    full_open = False
        fits = {}
        for mode in ("submesh", "full"):
            pts = [(r["V"], r["ms_per_step"]) for r in rows if r["mode"] == mode]
            if len(pts) >= 3:
                fits[mode] = float(np.polyfit(np.log([p[0] for p in pts]), np.log([p[1] for p in pts]), 1)[0])
        out[surf] = {"span": spec["span"], "range": spec["span"] / 10.0, "runs": rows, "exponent": fits}
    return {"workload": "fixed-N mesh-size sweep: N=100, velocity Verlet NVE, harmonic range span/10, sphere and "
                        "tori of aspect 3 and 20 refined at fixed span", "data": "synthetic", "precision": "fp64",
            "results": out}


def bench_c5(args, gsim, W, with_cpu=True):
    """All-pairs Coulomb with FIRE on the icosphere L6 (81,920 faces, N = 2000):
    every iteration propagates every source over the whole mesh (3,998,000
    pairs). Two timed iterations per precision after one warm-up. With
    --c5-fire K, each precision then runs K FIRE iterations from the same
    start and the end energies are compared, and at the FP64 run's end state
    the FP32-mixed energy and forces are compared with the FP64 ones (the
    same state in both). The CPU oracle is timed on a sample of sources."""
    import math
    w = W.workload("c5a")
    wi = w.integrator
    pot = gsim.potential("coulomb", 1.0, 1.0, math.inf)
    ig = gsim.integrator("fire", wi["dt"], max_disp=wi["max_disp"])
    n = len(w.face)
    out = {}
    ends = {}
    for prec in ("fp64", "fp32"):
        ctx = gsim.Context(0, prec)
        mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
        ctx.particles_set(mid, w.face, w.bary)
        ctx.step(mid, pot, ig, 1)
        ctx.synchronize()
        ctx.timing(True)
        t0 = time.perf_counter()
        ctx.step(mid, pot, ig, 2)
        ctx.synchronize()
        dt = time.perf_counter() - t0
        c = ctx.counters()
        geo = ctx.timing_get("geodesic")[0]
        ctx.timing(False)
        wpi = c["cum_windows"] / 2
        pk = FP64_VECTOR_PEAK_TFLOPS if prec == "fp64" else FP32_VECTOR_PEAK_TFLOPS
        ach = FLOPS_PER_WINDOW * wpi / (geo * 1e-3) / 1e12 if geo > 0 else 0.0
        rec = measured_counters("c5a", prec)
        out[prec] = {"pairs_per_s": 2 * n * (n - 1) / dt, "s_per_iteration": dt / 2, "geodesic_ms": geo,
                     "windows_per_iteration": wpi, "windows_per_s": c["cum_windows"] / dt,
                     "roofline": {"bound": "alu", "achieved": ach, "peak": pk, "unit": "TFLOP/s", "frac": ach / pk,
                                  "traffic": rec["traffic_bytes_per_launch"] if rec else None,
                                  "kernel": "k_geodesic_all", "per_unit": f"{FLOPS_PER_WINDOW:.0f} flop/window",
                                  "units_per_launch": wpi, "avg_launch_ms": geo}}
        print(f"[c5] {prec}: {dt / 2:.3f} s per iteration", file=sys.stderr, flush=True)
        if args.c5_fire:
            ctx.particles_set(mid, w.face, w.bary)
            ctx.tune(graph_steps=0)
            done = 0
            t0 = time.perf_counter()
            while done < args.c5_fire:
                k = min(10, args.c5_fire - done)
                ctx.step(mid, pot, ig, k)
                ctx.synchronize()
                done += k
                print(f"[c5] {prec}: {done} FIRE iterations, {time.perf_counter() - t0:.0f} s", file=sys.stderr,
                      flush=True)
            _, E = ctx.compute_forces(mid, pot)
            f, b, _, _ = ctx.particles_get(mid)
            ends[prec] = (E, f, b)
            out[prec]["fire"] = {"iterations": args.c5_fire, "end_energy": E, "s": time.perf_counter() - t0}
        ctx.close()
    line = {"workload": "C5: icosphere L6 (81920 faces), N=2000, Coulomb all pairs, FIRE", "data": "synthetic",
            "pairs_per_iteration": n * (n - 1), "results": out,
            "fp32_over_fp64": out["fp32"]["pairs_per_s"] / out["fp64"]["pairs_per_s"]}
    if ends:
        E64, f64, b64 = ends["fp64"]
        E32 = ends["fp32"][0]
        # the same state (the FP64 run's end) in both precisions
        same = {}
        scale = None
        for prec in ("fp64", "fp32"):
            ctx = gsim.Context(0, prec)
            mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
            ctx.particles_set(mid, f64, b64)
            same[prec] = ctx.compute_forces(mid, pot)
            if prec == "fp64":
                # the force error's scale (the error metric of the tests): for
                # U = k/d, sum_j |U'| + d |U''| = sum_j 3k / d^2
                g = ctx.geodesic_pairs(mid, math.inf)
                rows = np.repeat(np.arange(n), np.diff(g["off"]))
                scale = np.bincount(rows, weights=3.0 * w.potential["k"] / g["dist"] ** 2, minlength=n)
            ctx.close()
        F64, e64 = same["fp64"]
        F32, e32 = same["fp32"]
        fn = np.linalg.norm(F64, axis=1)
        dF = np.linalg.norm(F32 - F64, axis=1)
        line["fire_end"] = {"iterations": args.c5_fire, "energy_fp64_run": E64, "energy_fp32_run": E32,
                            "energy_rel_diff_of_runs": abs(E32 - E64) / abs(E64),
                            "same_state_energy_rel_err": abs(e32 - e64) / abs(e64),
                            "same_state_force_err_max": float(np.max(dF / scale)),
                            "same_state_force_err_note": "|F32 - F64| over sum_j (|U'| + d |U''|) per particle",
                            "net_force_over_scale_median": float(np.median(fn / scale)),
                            "same_state_force_rel_err_median": float(np.median(dF / np.maximum(fn, 1e-300)))}
    if with_cpu and not args.no_cpu_baseline:
        import oracle
        om = oracle.OracleMesh(w.mesh.V, w.mesh.T)
        nproc, model = host_cpu()
        threads = int(os.environ.get("OMP_NUM_THREADS", nproc))
        src = (np.arange(threads, dtype=np.int32) * (n // threads)).astype(np.int32)  # one source per thread
        t0 = time.perf_counter()
        oracle.geodesic_pairs(om, w.face, w.bary, math.inf, sources=src)
        t = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": len(src) * (n - 1) / t, "unit": "pairs/s", "cores": threads,
                                "kind": "oracle", "nproc": nproc, "cpu_model": model,
                                "sample": f"rows of {len(src)} sources over the whole mesh, {t:.1f} s"}
    return line


def bench_quench(args, gsim, W):
    """The crystallization study of Sec. 5 as a batched workload: 64
    independent gradient-descent quenches of N = 500 particles on the
    aspect-3 torus (each its own surface of one batch, stepped by one launch
    per stage and replayed from HIP graphs), against the same quenches one
    surface at a time; then the in-surface Voronoi neighbours of every
    relaxed state give the 5- and 7-fold defects, the net defect charge
    sum(6 - z) (zero on a torus) and its split between the inner (negative
    Gaussian curvature) and outer halves of the torus."""
    M = 64
    ws = [W.workload(f"quench_{k}") for k in range(M)]
    w0 = ws[0]
    p, wi = w0.potential, w0.integrator
    pot = gsim.potential("harmonic", p["k"], p["sigma"], p["cutoff"])
    ig = gsim.integrator("overdamped", wi["dt"], wi["mobility"])
    steps = w0.steps
    ctx = gsim.Context(0, "fp64")
    mids = []
    for w in ws:
        mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
        ctx.particles_set(mid, w.face, w.bary)
        mids.append(mid)
    ctx.step_batched(mids, [pot] * M, [ig] * M, 2)  # warm-up, graph capture
    for mid, w in zip(mids, ws):
        ctx.particles_set(mid, w.face, w.bary)
    ctx.synchronize()
    t0 = time.perf_counter()
    ctx.step_batched(mids, [pot] * M, [ig] * M, steps)
    ctx.synchronize()
    t_batch = time.perf_counter() - t0
    print(f"[quench] {M} tori x {steps} steps batched: {t_batch:.3f} s", file=sys.stderr, flush=True)
    # one surface at a time (4 of them, scaled)
    t_single = 0.0
    for k in range(4):
        c1 = gsim.Context(0, "fp64")
        m1 = c1.mesh_upload(ws[k].mesh.V, ws[k].mesh.T)
        c1.particles_set(m1, ws[k].face, ws[k].bary)
        c1.step(m1, pot, ig, 2)
        c1.particles_set(m1, ws[k].face, ws[k].bary)
        c1.synchronize()
        t0 = time.perf_counter()
        c1.step(m1, pot, ig, steps)
        c1.synchronize()
        t_single += time.perf_counter() - t0
        c1.close()
    t_single *= M / 4
    # defects of the relaxed states
    R = 3.0
    t0 = time.perf_counter()
    n5 = n7 = 0
    q_in = q_out = 0.0
    n_in = n_out = 0
    net = []
    for mid in mids:
        off, nbr = ctx.voronoi_neighbours(mid)
        z = np.diff(off)
        _, _, _, xyz = ctx.particles_get(mid)
        rho = np.hypot(xyz[:, 0], xyz[:, 1])
        q = 6 - z
        n5 += int((z == 5).sum())
        n7 += int((z == 7).sum())
        net.append(int(q.sum()))
        q_in += float(q[rho < R].sum())
        q_out += float(q[rho >= R].sum())
        n_in += int((rho < R).sum())
        n_out += int((rho >= R).sum())
    t_vor = time.perf_counter() - t0
    ctx.close()
    n = 500
    return {"workload": "64 gradient-descent quenches of N=500 on the aspect-3 torus (R=3, r=1, 4648 faces), harmonic "
                        "repulsion of range 1.2 lattice spacings, 400 steps each; in-surface Voronoi defects",
            "data": "synthetic", "precision": "fp64",
            "batched": {"quenches_per_s": M / t_batch, "particle_steps_per_s": M * n * steps / t_batch,
                        "ms_per_step": 1e3 * t_batch / steps},
            "one_surface_at_a_time": {"quenches_per_s": M / t_single, "particle_steps_per_s": M * n * steps / t_single},
            "batched_speedup": t_single / t_batch,
            "voronoi_ms_per_surface": 1e3 * t_vor / M,
            "defects": {"five_fold_per_quench": n5 / M, "seven_fold_per_quench": n7 / M,
                        "net_charge_per_quench": sorted(set(net)),
                        "mean_charge_inner_half": q_in / max(n_in, 1), "mean_charge_outer_half": q_out / max(n_out, 1)}}


def bench_single(args, gsim, W, name):
    """Timed eager steps of one workload (c2 or c4) in the headline
    precision, the other precision beside it, the stage times, the rooflines
    of the geodesic and update kernels, and the CPU oracle baseline."""
    w = W.workload(name)
    pot, ig = _gsim_args(gsim, w)

    def run(precision):
        # timed region: eager steps with HIP events around the geodesic stage
        # only (on the library's stream; every event record costs the stream
        # a few microseconds, so the other stages are timed in a separate
        # short run afterwards)
        ctx = gsim.Context(0, precision)
        mid = ctx.mesh_upload(w.mesh.V, w.mesh.T)
        ctx.particles_set(mid, w.face, w.bary)
        for _ in range(args.warmup):
            ctx.step(mid, pot, ig, 1)
        ctx.synchronize()
        ctx.tune(time_geodesic_only=1)
        ctx.timing(True)
        ctx.synchronize()
        t0 = time.perf_counter()
        ctx.step(mid, pot, ig, args.steps)
        ctx.synchronize()
        dt = time.perf_counter() - t0
        cnt = ctx.counters()
        geo = ctx.timing_get("geodesic")[0]
        ctx.timing(False)
        ctx.tune(time_geodesic_only=0)
        ctx.timing(True)
        k = min(args.steps, 20)
        ctx.step(mid, pot, ig, k)
        ctx.synchronize()
        stages = {st: v for st in ("prefilter", "geodesic", "update", "commit") for v, nl in [ctx.timing_get(st)] if nl}
        cst = ctx.counters()
        ctx.timing(False)
        ctx.close()
        return dt, cnt, geo, stages, dict(steps=k, pairs=cst["cum_pairs"], crossings=cst["crossings"])

    def update_roofline(stages, stage_cnt):
        """HBM roofline of the update kernel (a4-a6) from its stage time and
        the algorithmic bytes of the particles' steps (pairs and crossings
        per step averaged over the stage run)."""
        ms = stages.get("update")
        if not ms:
            return None
        k = stage_cnt["steps"]
        pairs = stage_cnt["pairs"] / k
        cross = stage_cnt["crossings"] / k
        nbytes = n * UPDATE_BYTES_PARTICLE + pairs * UPDATE_BYTES_PAIR + cross * UPDATE_BYTES_CROSSING
        gbps = nbytes / (ms * 1e-3) / 1e9
        return {"bound": "hbm", "achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS,
                "traffic": None, "kernel": "k_update_batch",
                "per_unit": f"{UPDATE_BYTES_PARTICLE} B/particle + {UPDATE_BYTES_PAIR} B/pair + "
                            f"{UPDATE_BYTES_CROSSING} B/edge crossing",
                "units_per_launch": {"particles": n, "pairs": pairs, "crossings": cross},
                "bytes_per_launch": nbytes, "avg_launch_ms": ms}

    n = len(w.face)
    dt, cnt, geo_ms, stages, scnt = run(args.precision)
    pairs = cnt["cum_pairs"]
    win_per_launch = cnt["cum_windows"] / max(cnt["cum_passes"], 1)
    achieved = FLOPS_PER_WINDOW * win_per_launch / (geo_ms * 1e-3) / 1e12 if geo_ms > 0 else 0.0
    peak = FP64_VECTOR_PEAK_TFLOPS if args.precision == "fp64" else FP32_VECTOR_PEAK_TFLOPS
    rec = measured_counters(name, args.precision)
    line = {
        "metric": METRIC,
        "value": pairs / dt,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD_TEXT[name],
                   "n_particles": n, "faces": w.mesh.nf, "cutoff": w.potential["cutoff"],
                   "precision": args.precision},
        "particle_steps_per_s": n * args.steps / dt,
        "pairs_per_step": pairs / args.steps,
        "stage_ms": stages,
        "stage_ms_note": "all stages timed in a separate run of up to 20 steps after the timed region; with the "
                         "update fused into the geodesic launch there is no update stage, and the commit runs once "
                         "per call",
        "windows_per_step": win_per_launch,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
                     "frac": achieved / peak,
                     "traffic": rec["traffic_bytes_per_launch"] if rec else None,
                     "kernel": "k_geodesic", "per_unit": f"{FLOPS_PER_WINDOW:.0f} flop/window",
                     "units_per_launch": win_per_launch, "avg_launch_ms": geo_ms},
        "update_roofline": update_roofline(stages, scnt),
    }
    if rec:
        line["roofline"]["counters"] = {k: rec[k] for k in ("lds", "occupancy", "hbm_gbps", "valu_busy",
                                                             "source") if k in rec}
    if not args.no_compare:
        other = "fp64" if args.precision == "fp32" else "fp32"
        dt2, cnt2, geo2, st2, scnt2 = run(other)
        w2 = cnt2["cum_windows"] / max(cnt2["cum_passes"], 1)
        pk2 = FP64_VECTOR_PEAK_TFLOPS if other == "fp64" else FP32_VECTOR_PEAK_TFLOPS
        a2 = FLOPS_PER_WINDOW * w2 / (geo2 * 1e-3) / 1e12 if geo2 > 0 else 0.0
        rec2 = measured_counters(name, other)
        line[other] = {"pairs_per_s": cnt2["cum_pairs"] / dt2, "particle_steps_per_s": n * args.steps / dt2,
                       "ms_per_step": 1e3 * dt2 / args.steps, "stage_ms": st2, "windows_per_step": w2,
                       "roofline": {"bound": "alu", "achieved": a2, "peak": pk2, "unit": "TFLOP/s", "frac": a2 / pk2,
                                    "traffic": rec2["traffic_bytes_per_launch"] if rec2 else None,
                                    "kernel": "k_geodesic", "avg_launch_ms": geo2, "units_per_launch": w2},
                       "update_roofline": update_roofline(st2, scnt2)}
        line[f"{other}_over_{args.precision}"] = (cnt2["cum_pairs"] / dt2) / (pairs / dt)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(w)
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"],
                    help="precision of the headline line (the other one is timed beside it unless --no-compare)")
    ap.add_argument("--workload", default="c4", choices=["c2", "c3", "c4", "c5", "torus_nve", "vsweep", "quench"],
                    help="c4: open height field N=20000, Brownian (the default line, with the c3 and c5 legs); "
                         "c2: bumpy sphere N=1000; c3: 16 surfaces batched; "
                         "torus_nve: NVE cost vs N on the benchmark torus; "
                         "vsweep: NVE cost vs mesh size at N=100, full mesh and submeshed; "
                         "quench: 64 batched torus quenches with Voronoi defect statistics; "
                         "c5: all-pairs Coulomb FIRE on the L6 sphere")
    ap.add_argument("--no-compare", action="store_true", help="skip the other precision's leg")
    ap.add_argument("--no-legs", action="store_true", help="default line only: skip the c3 and c5 legs")
    ap.add_argument("--c5-fire", type=int, default=0, metavar="K",
                    help="c5: also run K FIRE iterations per precision and compare the end energies")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MB",
                    help="only run a plain device-to-device copy of this many MiB (hardware-counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        import torch
        nbytes = args.copy_calibration << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": nbytes}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "sources would shard across GPUs with one all-gather of particle state per step, not built here.",
              file=sys.stderr)
        sys.exit(2)

    from paper_2404_19751_amd import gsim, workloads as W

    if args.workload == "c3":
        print(json.dumps(bench_c3(args, gsim, W)), flush=True)
        return
    if args.workload == "torus_nve":
        print(json.dumps(bench_torus_nve(args, gsim, W)), flush=True)
        return
    if args.workload == "vsweep":
        print(json.dumps(bench_vsweep(args, gsim, W)), flush=True)
        return
    if args.workload == "quench":
        print(json.dumps(bench_quench(args, gsim, W)), flush=True)
        return
    if args.workload == "c5":
        print(json.dumps(bench_c5(args, gsim, W)), flush=True)
        return
    line = bench_single(args, gsim, W, args.workload)
    if args.workload == "c4" and not args.no_legs:
        line["c3"] = bench_c3(args, gsim, W)
        line["c5"] = bench_c5(args, gsim, W, with_cpu=False)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
