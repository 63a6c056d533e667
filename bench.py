#!/usr/bin/env python3
"""Benchmark of the connectivity-aware multilevel FEM hot path on one MI355X.

One step = the whole path on one synthetic input, inputs resident in HBM:
hierarchy (grid placement, triangle/cell pairs, octree, supports, split,
prolongation), assembly of M and L at every depth, the load vector, and the
solve of (M + t L) x = b to a relative residual of 1e-8 with the learned
smoother in mixed precision (FP32 V-cycle under FP64 conjugate gradients).
The learned smoother is trained before timing on small meshes of other
shapes.

Workload (default): the held-out (3,5) torus-knot tube, 65536 x 64 quads
(8,388,608 triangles, jitter seed 5901), octree depth 11, degree 1, split,
t = 1e-4, RHS f = z + 0.1 x^2.

Prints one JSON line.  `value` is the solve time to 1e-8 of the learned
mixed-precision solve (iterations only, solver set-up reported apart), mean
over the timed steps; the plain FP64 and plain mixed Gauss-Seidel solves of
the same system, DoF x cycles per second, the per-phase times, the roofline
of the dominant kernel and of the whole V-cycle, the other configurations
and the oracle's CPU baseline are reported beside it.
"""
from __future__ import annotations

import argparse
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # the held-out meshes of the learned smoother (never trained on)
    "knot_8m_depth11": dict(mesh="knot_8m", depth=11, t=1e-4, degree=1,
                            desc="held-out (3,5) torus-knot tube, tube radius 0.05, 65536 x 64 quads "
                                 "(8,388,608 tris, jitter seed 5901), octree depth 11, degree 1, split, "
                                 "t=1e-4, RHS f = z + 0.1 x^2"),
    "sphere_8m_depth11": dict(mesh="sphere_8m", depth=11, t=1e-3, degree=1,
                              desc="held-out noisy sphere: octahedron subdivided 10x (8,388,608 tris), "
                                   "16 Gaussian bumps of amplitude 0.05 (seed 5902), octree depth 11, degree 1, "
                                   "split, t=1e-3, RHS f = z + 0.1 x^2"),
    "two_sheets_256_depth8": dict(mesh="two_sheets_256", depth=8, t=1e-3, degree=1,
                                  desc="two parallel unit squares 1/256 apart, 2 x 256 x 256 split quads "
                                       "(262,144 tris), rotated to general position, octree depth 8, degree 1, "
                                       "split, t=1e-3, RHS +-sin(40 pi x)"),
    "knot_2m_depth10": dict(mesh="knot_2m", depth=10, t=1e-4, degree=1,
                            desc="(3,5) torus-knot tube, 16384 x 64 quads (2,097,152 tris, jitter seed 3), "
                                 "octree depth 10, degree 1, split, t=1e-4, RHS f = x (first coordinate)"),
}


def workload_input(meshgen, name):
    """(V, F, f) of a workload; f is nv x 1."""
    if name == "knot_8m":
        V, F = meshgen.torus_knot(nu=65536, nv=64, seed=5901)
    elif name == "sphere_8m":
        V, F = meshgen.noisy_sphere(10, seed=5902, base="octa")
    else:
        V, F, f = meshgen.config_mesh(name)
        return V, F, np.asfortranarray(f[:, :1])
    return V, F, np.asfortranarray(V[:, 2:3] + 0.1 * V[:, 0:1] ** 2)
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


CPU_SAMPLE = dict(nu=2048, nv=16, seed=5901, depth=8, t=1e-4)


def host_cpu():
    """Host processor model (lscpu) and the thread counts the oracle can use."""
    model = None
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True, timeout=20).stdout
        for line in out.splitlines():
            if line.startswith("Model name:"):
                model = line.split(":", 1)[1].strip()
    except (OSError, subprocess.SubprocessError):
        pass
    omp = os.environ.get("OMP_NUM_THREADS")
    return {"model": model, "os_cpu_count": os.cpu_count(),
            "omp_threads": int(omp) if omp and omp.isdigit() else os.cpu_count()}


def cpu_baseline(cf, ctx, meshgen, full, sample=CPU_SAMPLE):
    """The oracle (plain FP64 C++, V(2,2)-preconditioned CG, the GPU's plain
    method) on a bounded sample of the headline workload's family: the (3,5)
    knot tube at 2048 x 16 quads (65,536 triangles) and depth 8.  Each phase
    is timed by the oracle itself (steady_clock): hierarchy build, assembly,
    solver setup, solve to 1e-8.  The solve runs single-threaded and with
    OpenMP on all threads the host gives this process (same bits).  The
    sample's solve time is scaled to the headline workload by finest DoF x
    cycles (the oracle's cost per DoF-cycle times the full problem's DoF and
    the GPU's plain FP64 cycle count there).  The same sample is solved on
    the GPU with each of the headline's three solvers, and each solution is
    compared with the oracle's: relative M-norm of the difference, and the
    largest difference of the values at the mesh vertices over the largest
    value."""
    from oracle import Oracle
    import torch
    V, F = meshgen.torus_knot(nu=sample["nu"], nv=sample["nv"], seed=sample["seed"])
    f = np.asfortranarray(V[:, 2:3] + 0.1 * V[:, 0:1] ** 2)
    depth, t = sample["depth"], sample["t"]
    cpu = host_cpu()
    legs = {}
    for omp in (False, True):
        t0 = time.perf_counter()
        o = Oracle(V, F, depth, max_coarse=4096, openmp=omp).check().assemble()
        b = o.load_vector(f)
        x, info = o.solve(t, b, rtol=1e-8, max_iter=3000)
        wall = time.perf_counter() - t0
        ph = o.timing()
        legs["omp" if omp else "single"] = {"threads": cpu["omp_threads"] if omp else 1, "cycles": info["cycles"],
                                            "converged": bool(info["converged"]), "wall_s": wall,
                                            "phases_s": ph, "x": x, "o": o, "b": b}
        log(f"[bench] oracle ({'all threads' if omp else '1 thread'}): {info['cycles']} cycles, phases {ph}")
    n = legs["single"]["o"].count(depth, "functions")
    o, xo, b = legs["single"]["o"], legs["single"]["x"], legs["single"]["b"]
    Mo, Lo = o.matrices(depth)
    # the GPU's three solvers on the same sample, against the oracle's solution
    dev = torch.device("cuda:0")
    h = cf.camfe_hierarchy_build(ctx, torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev), depth=depth,
                                 max_coarse=4096)
    s = cf.camfe_assemble(h)
    errs = {}
    uo = o.eval_vertices(xo)
    mn = float(np.sqrt(xo[:, 0] @ (Mo @ xo[:, 0])))
    for tag, kw in (("plain_gs_fp64", dict(precision=0, smoother=0)),
                    ("plain_gs_mixed", dict(precision=1, smoother=0)),
                    ("learned_mixed", dict(precision=1, smoother=2)),
                    ("block_fp64", dict(precision=0, smoother=3))):
        cf.camfe_smoother_attach(s, full.get("model") if tag == "learned_mixed" else None)
        x, st = cf.camfe_solve(s, b, t=t, rtol=1e-8, max_iter=3000, **kw)
        d = x[:, 0] - xo[:, 0]
        r = np.linalg.norm(b[:, 0] - (Mo + t * Lo) @ x[:, 0]) / np.linalg.norm(b)
        errs[tag] = {"fell_back": int(st["fell_back"]), "rel_M_norm_error": float(np.sqrt(d @ (Mo @ d)) / mn),
                     "rel_vertex_error": float(np.abs(cf.camfe_eval_vertices(s, len(V), x) - uo).max() /
                                               np.abs(uo).max()),
                     "rel_residual_in_oracle_matrices": float(r), "cycles": st["cycles"]}
    cf.camfe_smoother_attach(s, None)
    cf.camfe_system_destroy(s)
    cf.camfe_hierarchy_destroy(h)
    scale = full["dof"] * full["cycles_fp64"] / (n * legs["single"]["cycles"])
    out = {}
    for k, leg in legs.items():
        sol = leg["phases_s"]["solve"]
        out[k] = {"threads": leg["threads"], "cycles": leg["cycles"], "converged": leg["converged"],
                  "phases_s": {kk: round(v, 4) for kk, v in leg["phases_s"].items()},
                  "solve_s_sample": sol, "dof_cycles_per_s": n * leg["cycles"] / sol,
                  "solve_s_scaled_to_workload": sol * scale}
    top = out["omp"]
    return {"value": top["solve_s_scaled_to_workload"], "unit": "s", "cores": top["threads"], "kind": "oracle",
            "sample": f"(3,5) knot tube {sample['nu']}x{sample['nv']} quads ({len(F)} tris, jitter seed "
                      f"{sample['seed']}), depth {depth}, n={n}, t={t}, FP64 V(2,2)-preconditioned CG to 1e-8 "
                      f"({top['cycles']} cycles, {top['solve_s_sample']:.2f} s on {top['threads']} threads); "
                      f"scaled by DoF x cycles to the workload ({full['dof']} DoF, {full['cycles_fp64']} cycles)",
            "host": cpu, "single_thread": out["single"], "all_threads": out["omp"],
            "gpu_error_vs_oracle_on_sample": errs}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gs_colour_two_sheets_d8_traffic.md")
TRAFFIC_FILE_D10 = os.path.join(ROOT, "profiles", "gs_colour_knot_d10_traffic.md")
# counter summaries of the finest-depth colour sweeps, per workload
TRAFFIC_FILES = {"two_sheets_256_depth8": TRAFFIC_FILE, "knot_2m_depth10": TRAFFIC_FILE_D10,
                 "knot_8m_depth11": os.path.join(ROOT, "profiles", "gs_colour_knot_8m_d11_traffic.md")}
KERNEL_SOURCE = os.path.join(ROOT, "paper_1505_03615_amd", "csrc", "sell_kernels.hpp")


def measured_traffic(path=TRAFFIC_FILE, key="traffic_bytes_per_launch"):
    """HBM bytes per launch of the finest-depth FP64 colour sweep from a
    committed counter summary, or None when the sweep kernels' source has
    changed since the counters were taken (the summary records the source's SHA-256)."""
    import hashlib
    try:
        text = open(path).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    sha = hashlib.sha256(open(KERNEL_SOURCE, "rb").read()).hexdigest()
    if vals.get("kernel_source_sha256") != sha:
        return None
    try:
        return float(vals[key])
    except (KeyError, ValueError):
        return None


def roofline(cf, s, meas, reps=50, with_traffic=True, main_precision=1, traffic_file=TRAFFIC_FILE, depth=None):
    """Algorithmic bytes of one launch of the finest-depth kernel over its
    average duration (HIP events around a captured graph of back-to-back
    launches on the library's stream), against the HBM peak, in both
    precisions.  The top level describes main_precision (1: the FP32 sweep,
    which takes the larger share of the bench step: the mixed and the
    learned solves run it), the other precision sits beside it.
    with_traffic: attach the committed counter figures (taken on the
    two-sheet depth-8 workload only).  depth (optional): the finest depth,
    whose packed-matrix figures (slices, slices with 16-bit columns,
    entries) are attached."""
    res = {}
    precs = (0, 1) if meas in ("gs_colour", "residual") else (0,)
    if main_precision not in precs:
        main_precision = 0
    for p in precs:
        avg, by = cf.camfe_measure_kernel(s, meas, p, reps)
        achieved = by / (avg / 1000.0) / 1e9
        key = "traffic_bytes_per_launch" + ("_fp32" if p == 1 else "")
        res[p] = {"kernel": meas + " (finest depth, " + ("FP32" if p else "FP64") + ")", "achieved": achieved,
                  "frac": achieved / PEAK_HBM_GBS,
                  "traffic": measured_traffic(traffic_file, key) if (meas == "gs_colour" and with_traffic) else None,
                  "avg_launch_us": 1000.0 * avg, "bytes_per_launch": by}
        if meas == "gs_colour":
            # what any launch of this size costs on the same graph: an empty
            # kernel on the sweep's grid, and a plain copy of the same bytes
            e_ms, _ = cf.camfe_measure_kernel(s, "empty", p, reps)
            c_ms, c_by = cf.camfe_measure_kernel(s, "copy", p, reps)
            c_gbs = c_by / (c_ms / 1000.0) / 1e9
            res[p]["launch_floor"] = {"empty_us": 1000.0 * e_ms, "copy_us": 1000.0 * c_ms, "copy_bytes": c_by,
                                      "copy_GBs": c_gbs, "copy_frac": c_gbs / PEAK_HBM_GBS}
    out = {"bound": "hbm", "peak": PEAK_HBM_GBS, "unit": "GB/s", **res[main_precision]}
    if len(precs) == 2:
        out["fp64" if main_precision == 1 else "fp32"] = res[1 - main_precision]
    if depth is not None:
        sl, c16, ent = cf.camfe_system_sell_stats(s, depth)
        out["sell_finest"] = {"slices": sl, "slices_16bit_columns": c16, "entries": ent}
    return out


def calibrate_copy(torch, dev):
    """A plain device copy of 2^27 doubles (1 GiB read, 1 GiB written), three
    times: the reference for scaling the memory counters."""
    a = torch.empty(1 << 27, dtype=torch.float64, device=dev)
    bb = torch.empty_like(a)
    for _ in range(3):
        bb.copy_(a)
    torch.cuda.synchronize()


def train_smoother(cf, ctx, meshgen, steps=150, sweep=1):
    """Learned smoother trained (untimed) on small members of the three training
    families: an icosphere, two close parallel sheets and a knot tube.
    sweep 1: multicolour SOR with learned per-row weights; 0: damped Jacobi."""
    fams = [(meshgen.icosphere(4)[:2], 6, 1e-3),
            (meshgen.two_sheets(64, 1.0 / 64)[:2], 6, 1e-3),
            (meshgen.torus_knot(nu=2048, nv=16, seed=5), 7, 1e-4)]
    hs, ss = [], []
    for (V, F), depth, t in fams:
        h = cf.camfe_hierarchy_build(ctx, V, F, depth=depth, degree=1, max_coarse=4096)
        hs.append(h)
        ss.append(cf.camfe_assemble(h))
    t0 = time.perf_counter()
    m, hist = cf.camfe_smoother_train(ctx, ss, t=1e-3, levels=3, steps=steps, nu=2, bf16=True, lr=3e-3, seed=1,
                                      sweep=sweep, cycle=0)
    secs = time.perf_counter() - t0
    for s, h in zip(ss, hs):
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)
    return m, {"sweep": "multicolour SOR" if sweep == 1 else "damped Jacobi", "loss": "smoothing (2 sweeps)",
               "steps": steps, "seconds": secs,
               "loss_first": float(hist[0]), "loss_last": float(hist[-1]),
               "families": "icosphere L4 depth 6; two sheets 64x64 depth 6; (3,5) knot 2048x16 depth 7"}


def vcycle_bytes(cf, s, h, k, sv, sx, nu=4, gamma=1, direct=True, nu_below=None):
    """Algorithmic bytes of one V-cycle (gamma 1) or W-cycle (gamma 2): per
    depth d above the coarsest, (nu + 1) passes over the matrix values and
    three vector accesses per row (nu sweeps and the residual), the parent
    map read twice (restriction and prolongation, 4 B per entry) and the
    transfer vectors; at the coarsest depth the dense inverse (8 n0^2) and its
    vectors, or nu sweeps when it is only relaxed.  A W-cycle visits depth d
    gamma^(D - d) times; nu_below (default nu) is the sweep count below the
    finest depth.  Counts come from the library's two-call exports with zero
    capacity."""
    import ctypes
    lib = cf.load()
    fin, d0 = cf.camfe_hierarchy_levels(h)
    nz = ctypes.c_int64()
    total = 0.0
    for d in range(d0, fin + 1):
        visits = float(gamma) ** (fin - d)
        nud = nu if (d == fin or nu_below is None) else nu_below
        n = cf.camfe_hierarchy_info(h, d)[2]
        cf._check(lib.camfe_export_matrix(s, d, 0, None, None, None, 0, ctypes.byref(nz)))
        z = nz.value
        if d == d0:
            total += visits * ((8.0 * n * n + 2.0 * n * k * sx) if direct else nud * (z * sv + 3.0 * n * k * sx))
            continue
        cf._check(lib.camfe_export_prolongation(h, d, None, None, None, 0, ctypes.byref(nz)))
        pn = nz.value
        nc = cf.camfe_hierarchy_info(h, d - 1)[2]
        total += visits * ((nud + 1) * (z * sv + 3.0 * n * k * sx) + 2.0 * 4.0 * pn + (3.0 * n + 2.0 * nc) * k * sx)
    return total


def cycle_roofline(bytes_per_cycle, ms, cycles):
    t = ms / 1000.0 / max(cycles, 1)
    gbs = bytes_per_cycle / t / 1e9
    return {"bytes_per_cycle": bytes_per_cycle, "ms_per_cycle": 1000.0 * t, "GBs": gbs, "frac": gbs / PEAK_HBM_GBS}


SOLVERS = (("plain_gs_fp64", dict(precision=0, smoother=0)),
           ("plain_gs_mixed", dict(precision=1, smoother=0)),
           ("learned_mixed", dict(precision=1, smoother=2)),
           # cell-block Schwarz (smoother 3, FP64 cycles, damping chosen per depth): CG capped at 500
           # iterations, then Gauss-Seidel redoes the solve
           ("block_fp64", dict(precision=0, smoother=3, max_iter=500)))


# sweep schedules tried per solver: (sweeps before and after at the finest
# depth, sweeps before and after at every coarser depth); 0 = the same
SCHEDULES = ((2, 0), (2, 1), (3, 1), (1, 0))


def schedule_kw(sched):
    nu, nc = sched
    return dict(nu_pre=nu, nu_post=nu, nu_coarse=nc)


def tune_schedules(cf, s, b, t, model, which, max_iter=4000):
    """Every solver of `which` to 1e-8 once warm with each of SCHEDULES on one
    system; the fastest schedule per solver (iteration time, set-up excluded).
    The same rule for every solver, so their comparison stays even."""
    out = {}
    for tag, kw in SOLVERS:
        if tag not in which:
            continue
        cf.camfe_smoother_attach(s, model if tag == "learned_mixed" else None)
        kw = dict(kw)
        mi = kw.pop("max_iter", max_iter)
        times, cycles = {}, {}
        for sc in SCHEDULES:
            cf.camfe_solve(s, b, t=t, rtol=1e-8, max_iter=4, **kw, **schedule_kw(sc))
            _, st = cf.camfe_solve(s, b, t=t, rtol=1e-8, max_iter=mi, **kw, **schedule_kw(sc))
            times[sc] = st["seconds"] if st["converged"] else float("inf")
            cycles[sc] = st["cycles"]
        best = min(times, key=times.get)
        out[tag] = {"chosen": list(best),
                    "seconds": {f"{a},{c}": (round(v, 4) if v != float("inf") else None) for (a, c), v in times.items()},
                    "cycles": {f"{a},{c}": v for (a, c), v in cycles.items()}}
        log(f"[bench] schedule {tag}: {best} from " + json.dumps(out[tag]["seconds"]) + " (null: not converged)")
    cf.camfe_smoother_attach(s, None)
    return out


def solve_comparison(cf, s, h, b, t, model, which=("plain_gs_fp64", "plain_gs_mixed", "learned_mixed", "block_fp64"),
                     max_iter=4000, schedules=None):
    """Each solver to 1e-8 on one assembled system, warm: a 4-iteration solve
    first builds the solver state and captures the graphs, then the full
    solve runs once.  Iteration time (set-up excluded), cycles, DoF x cycles
    per second, and the whole V-cycle's algorithmic bytes over its measured
    time (a captured plain V(2,2)-cycle, FP64 and FP32).  schedules: solver ->
    (nu, nu below), else V(2,2) everywhere."""
    fin = cf.camfe_hierarchy_levels(h)[0]
    n = cf.camfe_hierarchy_info(h, fin)[2]
    res = {"dof": int(n)}
    for tag, kw in SOLVERS:
        if tag not in which:
            continue
        cf.camfe_smoother_attach(s, model if tag == "learned_mixed" else None)
        kw = dict(kw)
        mi = kw.pop("max_iter", max_iter)
        kw.update(schedule_kw(tuple(schedules[tag]) if schedules and tag in schedules else (2, 0)))
        cf.camfe_solve(s, b, t=t, rtol=1e-8, max_iter=4, **kw)
        x, st = cf.camfe_solve(s, b, t=t, rtol=1e-8, max_iter=mi, **kw)
        res[tag] = {"s": st["seconds"], "cycles": st["cycles"], "rel_residual": st["rel_residual"],
                    "converged": bool(st["converged"]), "fell_back": int(st["fell_back"]),
                    "setup_s": st["setup_seconds"], "dof_cycles_per_s": n * st["cycles"] / st["seconds"]}
        if kw.get("smoother") == 3:
            om, lam = cf.camfe_block_damping(s, t)
            res[tag]["damping_per_depth"] = [round(float(v), 4) for v in om]
            res[tag]["lambda_max_estimate_per_depth"] = [round(float(v), 4) for v in lam]
        log(f"[bench] {tag}: {st['cycles']} cycles, {1000 * st['seconds']:.0f} ms")
    cf.camfe_smoother_attach(s, None)
    if "plain_gs_fp64" in res and "learned_mixed" in res:
        res["speedup_learned_mixed_vs_plain_fp64"] = res["plain_gs_fp64"]["s"] / res["learned_mixed"]["s"]
    if "plain_gs_mixed" in res and "learned_mixed" in res:
        res["speedup_learned_mixed_vs_plain_mixed"] = res["plain_gs_mixed"]["s"] / res["learned_mixed"]["s"]
    res["vcycle_roofline"] = whole_cycle(cf, s, h)
    if schedules and "plain_gs_mixed" in schedules and tuple(schedules["plain_gs_mixed"]) != (2, 0):
        sc = tuple(schedules["plain_gs_mixed"])
        res["vcycle_roofline_chosen_schedule"] = {"schedule": list(sc), **whole_cycle(cf, s, h, schedule=sc)}
    return res


def whole_cycle(cf, s, h, reps=10, schedule=(2, 0)):
    """One plain Gauss-Seidel V-cycle (captured, back to back) against the
    HBM peak: algorithmic bytes of the cycle (vcycle_bytes) over its measured
    time.  schedule = (sweeps each way at the finest depth, below; 0 = same)."""
    a, c = schedule
    name = "vcycle" if (a, c) == (2, 0) else f"vcycle:{a},{c}"
    out = {}
    for p, (sv, sx) in ((0, (8, 8)), (1, (4, 4))):
        ms, _ = cf.camfe_measure_kernel(s, name, p, reps)
        by = vcycle_bytes(cf, s, h, 1, sv, sx, nu=2 * a, nu_below=2 * (c if c > 0 else a))
        gbs = by / (ms / 1000.0) / 1e9
        out["fp64" if p == 0 else "fp32"] = {"bytes_per_cycle": by, "ms_per_cycle": ms, "GBs": gbs,
                                            "frac": gbs / PEAK_HBM_GBS}
    return out


def assembly_eval(cf, ctx, meshgen, reps=2):
    """Assembly of M and L at every depth (the FP64 matrix-core kernel) on the
    bench workload, the config-3 knot (degree 1) and two degree-2 cases: event
    time of the assembly launches, the useful flops of their dense
    contractions (2 NB^2 per quadrature point for M and for each of the three
    gradient products), and that rate against the FP64 matrix peak.  Best of
    `reps` assemblies of one hierarchy."""
    import torch
    dev = torch.device("cuda:0")
    cases = [("two sheets 2 x 256 x 256 quads, depth 8, degree 1", meshgen.config_mesh("two_sheets_256")[:2], 8, 1),
             ("(3,5) knot tube 2,097,152 tris, depth 10, degree 1", meshgen.torus_knot(nu=16384, nv=64, seed=3), 10, 1),
             ("icosphere level 3 (1280 tris), depth 5, degree 2", meshgen.icosphere(3), 5, 2),
             ("noisy sphere 327,680 tris, depth 8, degree 2", meshgen.noisy_sphere(7, seed=5), 8, 2)]
    out = []
    for name, (V, F), depth, degree in cases:
        h = cf.camfe_hierarchy_build(ctx, torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev), depth=depth,
                                     degree=degree, max_coarse=4096)
        best = None
        for _ in range(reps):
            cf.camfe_ctx_kernel_timing(ctx, True)
            s = cf.camfe_assemble(h)
            cf.camfe_ctx_kernel_timing(ctx, False)
            ms, launches, flops = cf.camfe_ctx_kernel_time(ctx, "assemble")
            cf.camfe_system_destroy(s)
            if best is None or ms < best[0]:
                best = (ms, launches, flops)
        cf.camfe_hierarchy_destroy(h)
        ms, launches, flops = best
        tf = flops / (ms / 1000.0) / 1e12
        out.append({"case": name, "tris": int(len(F)), "assemble_kernel_ms": ms, "launches": int(launches),
                    "useful_mfma_flops": flops, "achieved_tflops": tf, "peak_tflops": PEAK_FP64_TFLOPS,
                    "frac": tf / PEAK_FP64_TFLOPS})
        log("[bench] assembly: " + json.dumps(out[-1]))
    return out


def flow_eval(cf, ctx, meshgen, steps=10, max_coarse=4096):
    """Config 3: tracked cMCF steps (M_t + delta/2 L_0) X' = M_t X on the (3,5)
    knot tube (2,097,152 triangles, depth 10), delta/2 = 1e-4, the three
    coordinate columns, mixed precision, 1e-8 per step.  A step re-weights and
    re-assembles M_t at every depth, refreshes the solver and solves.  Two
    steps from the initial surface with each sweep setting (finest, below) =
    (2, 2), (2, 1), (3, 1) choose the fastest; the timed steps then start
    again from the initial surface (the mass-block cache is already built)."""
    import torch
    V, F = meshgen.torus_knot(nu=16384, nv=64, seed=3)
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    h = cf.camfe_hierarchy_build(ctx, torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev), depth=10, degree=1,
                                 max_coarse=max_coarse)
    s = cf.camfe_assemble(h)
    X = cf.camfe_linear_coeffs(s, h)
    torch.cuda.synchronize()
    setup = time.perf_counter() - t0
    tune = {}
    for nu, nc in ((2, 0), (2, 1), (3, 1)):
        Xt = torch.from_numpy(np.asfortranarray(X)).to(dev)
        for k in range(2):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            Xt, st = cf.camfe_flow_step(s, Xt, 2e-4, rtol=1e-8, max_iter=1000, precision=1, nu_pre=nu, nu_post=nu,
                                        nu_coarse=nc)
            torch.cuda.synchronize()
        tune[nu, nc] = 1000.0 * (time.perf_counter() - t1) if st["converged"] else float("inf")
    nu, nc = min(tune, key=tune.get)
    Xd = torch.from_numpy(np.asfortranarray(X)).to(dev)
    per, cyc, solve_s = [], [], []
    for k in range(steps):
        t1 = time.perf_counter()
        Xd, st = cf.camfe_flow_step(s, Xd, 2e-4, rtol=1e-8, max_iter=1000, precision=1, nu_pre=nu, nu_post=nu,
                                    nu_coarse=nc)
        torch.cuda.synchronize()
        per.append(time.perf_counter() - t1)
        cyc.append(st["cycles"])
        solve_s.append(st["seconds"])
        if not st["converged"]:
            break
    n = cf.camfe_hierarchy_info(h, 10)[2]
    # FP32 cycles, three columns, the chosen sweeps
    vb = vcycle_bytes(cf, s, h, 3, 4, 4, nu=2 * nu, nu_below=2 * (nc if nc > 0 else nu))
    # the same colour-sweep measurement as the bench's roofline, on this
    # 2.2M-function finest depth (launches about twelve times larger)
    big = roofline(cf, s, "gs_colour", reps=10, with_traffic=False, depth=10)
    # counters taken on this same workload
    big["traffic"] = measured_traffic(TRAFFIC_FILE_D10, "traffic_bytes_per_launch_fp32")
    big["fp64"]["traffic"] = measured_traffic(TRAFFIC_FILE_D10)
    cf.camfe_system_destroy(s)
    cf.camfe_hierarchy_destroy(h)
    return {"mesh": "(3,5) knot tube, 2,097,152 tris, depth 10", "dof": int(n), "steps": len(per),
            "gs_colour_roofline_depth10": big,
            # solve iterations of steps 2.. (the first also builds the mass-block cache)
            "vcycle_roofline": cycle_roofline(vb, 1000.0 * float(np.sum(solve_s[1:])), int(np.sum(cyc[1:]))),
            "hierarchy_and_assembly_ms": 1000.0 * setup, "ms_per_step": 1000.0 * float(np.mean(per)),
            "first_step_ms": 1000.0 * per[0], "cycles_per_step": [int(c) for c in cyc],
            "sweeps_finest_below": [nu, nc],
            "sweep_autotune_second_step_ms": {f"{a},{c}": v for (a, c), v in tune.items()},
            "context": "the paper's Table 1: 1.52 s per step for its 1.27M-DoF system (CPU, its own solver)"}


def flow_study_eval(cf, ctx, meshgen, T=0.01, steps=(4, 8, 16), ref_steps=64, depth=8):
    """The cMCF study (Section 5.3) on a genus-0 two-lobe surface: a U-shaped
    capsule (tube radius 0.2, arms 1.0 long and 0.004 apart, 128 vertices
    per ring), depth 8 (finest cells about 0.007 wide, wider than the gap).
    Flow time T is reached in n tracked steps of T/n, split and unsplit,
    mixed precision, 1e-10 per step.  Every surface is compared with the
    split FP64 flow in ref_steps steps: RMS and largest vertex distance over
    all vertices and over the facing walls (vertices of the arms within 0.05
    of the plane between them, where the unsplit functions straddle the
    gap), and the wall time of the n steps."""
    import torch
    V, F = meshgen.u_tube(nv=128, ncap=16)
    dev = torch.device("cuda:0")
    Vd, Fd = torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev)
    wall_mask = torch.from_numpy((np.abs(V[:, 0]) < 0.05) & (V[:, 1] > 0.0)).to(dev)
    systems = {}
    for split in (1, 0):
        h = cf.camfe_hierarchy_build(ctx, Vd, Fd, depth=depth, split=split, max_coarse=4096)
        systems[split] = (h, cf.camfe_assemble(h))

    def run(split, n, precision):
        h, s = systems[split]
        X = cf.camfe_linear_coeffs(s, h)
        Xd = torch.from_numpy(np.asfortranarray(X)).to(dev)
        cycles = 0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(n):
            Xd, st = cf.camfe_flow_step(s, Xd, T / n, rtol=1e-10, max_iter=2000, precision=precision)
            cycles += st["cycles"]
            if not st["converged"]:
                raise RuntimeError("flow step did not converge")
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        return cf.camfe_eval_vertices(s, len(V), Xd), wall, cycles

    ref, ref_wall, _ = run(1, ref_steps, 0)
    rows = []
    for split in (1, 0):
        for n in steps:
            P, wall, cyc = run(split, n, 1)
            d = torch.linalg.norm(P - ref, dim=1)
            dw = d[wall_mask]
            rows.append({"split": split, "steps": n, "delta": T / n, "wall_ms": 1000.0 * wall,
                         "ms_per_step": 1000.0 * wall / n, "cycles": int(cyc),
                         "rms_vertex_error": float(torch.sqrt((d * d).mean()).item()),
                         "max_vertex_error": float(d.max().item()),
                         "rms_facing_wall_error": float(torch.sqrt((dw * dw).mean()).item()),
                         "max_facing_wall_error": float(dw.max().item())})
            log("[bench] flow study: " + json.dumps(rows[-1]))
    out = {"mesh": f"U-shaped capsule, {len(F)} tris, arms 0.004 apart, depth {depth}", "flow_time": T,
           "facing_wall_vertices": int(wall_mask.sum().item()), "vertices": int(len(V)),
           "functions": {"split": int(cf.camfe_hierarchy_info(systems[1][0], depth)[2]),
                         "unsplit": int(cf.camfe_hierarchy_info(systems[0][0], depth)[2])},
           "reference": f"split, FP64, {ref_steps} steps, {1000.0 * ref_wall:.0f} ms", "rows": rows}
    for split in (1, 0):
        h, s = systems[split]
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)
    return out


SPEC_GAP = 0.02


def spectrum_eval(cf, ctx, meshgen, depths=(4, 5, 6, 7), rot_depth=5, rotations=6, nev=16):
    """The spectral study (Section 5.1) on two concentric icospheres (level 6,
    2 x 81,920 triangles) 0.02 apart, closer than a cell at every depth used:
    the nev smallest eigenvalues of L x = lambda M x by camfe_eigs (block
    nev + 8, sigma 1, 1e-9), split and unsplit, against the exact spectrum
    l(l+1) and l(l+1)/1.02^2 (multiplicity 2l + 1 each).  Resolution sweep
    over depths; rotation sweep at one depth (rotations about seeded random
    axes): the spread of each eigenvalue over the rotations."""
    import torch
    dev = torch.device("cuda:0")
    exact = []
    for l in range(8):
        exact += [l * (l + 1.0)] * (2 * l + 1) + [l * (l + 1.0) / (1 + SPEC_GAP) ** 2] * (2 * l + 1)
    exact = np.sort(exact)[:nev]
    nz = exact > 0

    def spectrum(V, F, depth, split):
        h = cf.camfe_hierarchy_build(ctx, torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev), depth=depth,
                                     split=split, max_coarse=4096)
        s = cf.camfe_assemble(h)
        n = cf.camfe_hierarchy_info(h, depth)[2]
        ev, _, st = cf.camfe_eigs(s, h, nev, sigma=1.0, max_iter=400, tol=1e-9, solve_rtol=1e-10, precision=1,
                                  vectors=False)
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)
        return np.asarray(ev), int(n), st

    V, F = meshgen.nested_spheres(6, SPEC_GAP)
    res = []
    for depth in depths:
        for split in (1, 0):
            ev, n, st = spectrum(V, F, depth, split)
            err = np.abs(ev[nz] - exact[nz]) / exact[nz]
            res.append({"depth": depth, "split": split, "functions": n, "zero_eigenvalues": int((np.abs(ev) < 1e-6).sum()),
                        "max_rel_error": float(err.max()), "mean_rel_error": float(err.mean()),
                        "eigs_ms": 1000.0 * st["seconds"], "iterations": st["iterations"],
                        "solve_cycles": st["solve_cycles"], "converged": st["converged"],
                        "eigenvalues": [round(float(x), 5) for x in ev]})
            log("[bench] spectrum: " + json.dumps({k: v for k, v in res[-1].items() if k != "eigenvalues"}))
    rng = np.random.default_rng(5100)
    rot = {1: [], 0: []}
    for r in range(rotations):
        axis = rng.normal(size=3)
        R = meshgen.rodrigues(axis, rng.uniform(0.1, 3.0))
        Vr, Fr = meshgen.nested_spheres(6, SPEC_GAP, rotation=R)
        for split in (1, 0):
            ev, _, _ = spectrum(Vr, Fr, rot_depth, split)
            rot[split].append(ev)
    spread = {}
    for split in (1, 0):
        E = np.array(rot[split])[:, nz]
        spread["split" if split else "unsplit"] = {
            "max_rel_spread": float(((E.max(0) - E.min(0)) / E.mean(0)).max()),
            "mean_rel_spread": float(((E.max(0) - E.min(0)) / E.mean(0)).mean()),
            "max_rel_error": float((np.abs(E - exact[nz]) / exact[nz]).max())}
        log("[bench] spectrum rotations: " + json.dumps(spread))
    return {"mesh": "two concentric icospheres, level 6, radii 1 and 1.02 (163,840 tris)", "nev": nev,
            "exact": [round(float(x), 5) for x in exact], "resolution": res,
            "rotations": {"depth": rot_depth, "count": rotations, **spread}}


CUBES_ALPHA = 0.01


def cubes_eval(cf, ctx, meshgen, depth=5):
    """Figure cubes (Section 5.2): the 6x6x6 unit cubes (each face 4 x 4 split
    quads, 41,472 triangles) with a solid 3D checker as the colour f, the
    screened Poisson fit (L + alpha M) u = g + alpha s with alpha = 0.01 and
    g the gradient constraint, depth 5, one W-cycle with ten Gauss-Seidel
    sweeps before and after each coarse correction, from a seeded guess
    uniform in [0, 1], for every minimum depth, split and unsplit.  The
    coarsest depth is relaxed (ten sweeps each way).  Residual after the
    cycle over the norm of the guess, column by column (max over the three
    colour columns),
    the warm W-cycle time (a second identical solve replays the captured
    graph) and the gradient-load time."""
    import torch
    V, F, col = meshgen.cubes_checker()
    dev = torch.device("cuda:0")
    Vd, Fd = torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev)
    cold = torch.from_numpy(np.asfortranarray(col)).to(dev)
    rows = []
    for split in (1, 0):
        for m in range(depth + 1):
            h = cf.camfe_hierarchy_build(ctx, Vd, Fd, depth=depth, split=split, min_depth=m, max_coarse=0)
            s = cf.camfe_assemble(h)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            g = cf.camfe_gradient_load(s, h, cold)
            torch.cuda.synchronize()
            grad_ms = 1000.0 * (time.perf_counter() - t0)
            b = (g + CUBES_ALPHA * cf.camfe_load_vector(s, h, cold)) / CUBES_ALPHA
            n = b.shape[0]
            x0 = torch.from_numpy(np.asfortranarray(np.random.default_rng(6200).uniform(0.0, 1.0, size=(n, 3))))
            x0 = x0.to(dev)
            secs = []
            for _ in range(2):
                x, st = cf.camfe_solve(s, b, t=1.0 / CUBES_ALPHA, rtol=0.0, max_iter=1, nu_pre=10, nu_post=10,
                                       method=1, x0=x0, cycle=2)
                secs.append(st["seconds"])
            r = CUBES_ALPHA * (b - cf.camfe_apply(s, 2, 1.0 / CUBES_ALPHA, x))
            res = float((torch.linalg.norm(r, dim=0) / torch.linalg.norm(x0, dim=0)).max().item())
            wb = vcycle_bytes(cf, s, h, 3, 8, 8, nu=20, gamma=2, direct=False)
            rows.append({"split": split, "min_depth": m, "finest_functions": int(n),
                         "coarsest_functions": int(cf.camfe_hierarchy_info(h, m)[2]),
                         "residual_over_guess": res, "w_cycle_ms": 1000.0 * secs[1],
                         "w_cycle_bytes": wb, "w_cycle_GBs": wb / secs[1] / 1e9, "gradient_load_ms": grad_ms})
            log("[bench] cubes: " + json.dumps(rows[-1]))
            cf.camfe_system_destroy(s)
            cf.camfe_hierarchy_destroy(h)
    rs = {r["min_depth"]: r["residual_over_guess"] for r in rows if r["split"] == 1}
    rp = {r["min_depth"]: r["residual_over_guess"] for r in rows if r["split"] == 0}
    return {"mesh": "6x6x6 unit cubes, pitch 2, 41,472 tris, 3D checker colour", "depth": depth,
            "alpha": CUBES_ALPHA, "cycle": "W(10,10), relaxed coarsest", "rows": rows,
            "split_gain_full_vs_finest_only": rs[depth] / rs[0],
            "unsplit_gain_full_vs_finest_only": rp[depth] / rp[0]}


def stripe_knot_eval(cf, ctx, meshgen, nu=8192, nv=64, depth=9, alpha=0.01):
    """Colour fitting (Section 5.2) on a self-intersecting (3,5) knot tube
    (radius 0.35, 8192 x 64 quads = 1,048,576 tris, the teaser's setting):
    stripe texture f = cos(40 s) along the knot, gradient constraint g and
    value load s, (L + alpha M) u = g + alpha s solved to 1e-8 (FP64 CG),
    split against unsplit.  Errors |u - f| at the vertices, RMS and largest,
    near the crossings (vertices within 0.05 of another strand) and
    elsewhere."""
    import torch
    dev = torch.device("cuda:0")
    V, F, f, spar = meshgen.stripe_knot(nu=nu, nv=nv)
    near = torch.from_numpy(meshgen.near_other_strand(V, spar, 0.05)).to(dev)
    Vd, Fd, fd = torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev), torch.from_numpy(f).to(dev)
    rows = []
    for split in (1, 0):
        h = cf.camfe_hierarchy_build(ctx, Vd, Fd, depth=depth, split=split, max_coarse=4096)
        s = cf.camfe_assemble(h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b = (cf.camfe_gradient_load(s, h, fd) + alpha * cf.camfe_load_vector(s, h, fd)) / alpha
        torch.cuda.synchronize()
        load_ms = 1000 * (time.perf_counter() - t0)
        cf.camfe_solve(s, b, t=1.0 / alpha, rtol=1e-8, max_iter=4)
        x, st = cf.camfe_solve(s, b, t=1.0 / alpha, rtol=1e-8, max_iter=4000)
        e = (cf.camfe_eval_vertices(s, len(V), x)[:, 0] - fd[:, 0]).abs()
        rows.append({"split": split, "functions": int(cf.camfe_hierarchy_info(h, depth)[2]),
                     "cycles": st["cycles"], "solve_ms": 1000 * st["seconds"], "load_ms": load_ms,
                     "rms_error_near_crossings": float(torch.sqrt((e[near] ** 2).mean()).item()),
                     "max_error_near_crossings": float(e[near].max().item()),
                     "rms_error_elsewhere": float(torch.sqrt((e[~near] ** 2).mean()).item())})
        log("[bench] stripe knot: " + json.dumps(rows[-1]))
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)
    return {"mesh": f"self-intersecting (3,5) knot tube, radius 0.35, {nu}x{nv} quads ({len(F)} tris)",
            "depth": depth, "alpha": alpha, "texture": "cos(40 s) along the knot",
            "near_crossings_vertices": int(near.sum().item()), "vertices": int(len(V)), "rows": rows}


def batch_eval(cf, ctx, meshgen, count=64, seed=4000, t=1e-3, schedule=(2, 0)):
    """Config 4: `count` uneven meshes from meshgen.config4_batch (icospheres
    L3-7, tori with R/r in [2, 6] and 1k-1.3M triangles, noisy icospheres
    L3-8; depth clamp(round(log2(side / mean edge)), 6, 10); 1-16 N(0, 1)
    right-hand sides each), solved to 1e-8 in FP64: one system at a time
    (every system warm, iterations summed), then as one batch with a member
    per (mesh, chunk of <= 4 columns) so that one pass covers every column,
    with the default colour-sweep tile and with the autotuner's tile per
    level.  schedule = (sweeps each way at the finest depth, below; 0 = the
    same), for both the single systems and the batch."""
    skw = schedule_kw(schedule)
    import torch
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    members = meshgen.config4_batch(count, seed)
    gen_s = time.perf_counter() - t0
    systems = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for m in members:
        h = cf.camfe_hierarchy_build(ctx, torch.from_numpy(m["V"]).to(dev), torch.from_numpy(m["F"]).to(dev),
                                     depth=m["depth"], degree=1, max_coarse=4096)
        s = cf.camfe_assemble(h)
        b = cf.camfe_load_vector(s, h, torch.from_numpy(m["fv"]).to(dev))
        systems.append((h, s, b))
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t0
    dof = [int(cf.camfe_hierarchy_info(h, m["depth"])[2]) for (h, _, _), m in zip(systems, members)]
    log(f"[bench] batch: {len(members)} meshes, {sum(len(m['F']) for m in members)} tris, {sum(dof)} DoF, "
        f"generated in {gen_s:.1f} s, built and assembled in {setup_s:.1f} s")
    single = 0.0
    single_cycles = []
    for h, s, b in systems:
        cf.camfe_solve(s, b, t=t, rtol=1e-8, max_iter=4, **skw)
        x, st = cf.camfe_solve(s, b, t=t, rtol=1e-8, max_iter=2000, **skw)
        single += st["seconds"]
        single_cycles.append(st["cycles"])
    mem, chunks = [], []
    for h, s, b in systems:
        for c0 in range(0, b.shape[1], 4):
            mem.append(s)
            chunks.append(b[:, c0:c0 + 4])
    t0 = time.perf_counter()
    bt = cf.camfe_batch_create(ctx, mem, t)
    create_s = time.perf_counter() - t0
    levels, rows = cf.camfe_batch_info(bt)
    runs = {}
    for tag in ("default_tiles", "autotuned_tiles"):
        if tag == "autotuned_tiles":
            t0 = time.perf_counter()
            tiles, tms = cf.camfe_batch_autotune(bt, precision=0, reps=10)
            tune_s = time.perf_counter() - t0
        cf.camfe_batch_solve(bt, chunks, t, rtol=1e-8, max_iter=4, **skw)      # capture
        xs, sts = cf.camfe_batch_solve(bt, chunks, t, rtol=1e-8, max_iter=2000, **skw)
        its = sorted(x["iterations"] for x in sts)
        runs[tag] = {"solve_s": sts[0]["seconds"], "iterations": its[-1],
                     "member_iterations_median": its[len(its) // 2], "member_iterations_sum": int(sum(its)),
                     "all_converged": bool(all(x["converged"] for x in sts)),
                     "max_rel_residual": float(max(x["rel_residual"] for x in sts))}
        log(f"[bench] batch {tag}: " + json.dumps(runs[tag]))
    cf.camfe_batch_destroy(bt)
    for h, s, b in systems:
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)
    return {"meshes": len(members), "sweeps_finest_below": list(schedule),
            "tris_total": int(sum(len(m["F"]) for m in members)),
            "tris_min_max": [int(min(len(m["F"]) for m in members)), int(max(len(m["F"]) for m in members))],
            "dof_total": int(sum(dof)), "depths": [m["depth"] for m in members],
            "rhs": [int(m["fv"].shape[1]) for m in members], "kinds": [m["kind"] for m in members],
            "generate_s": gen_s, "build_assemble_load_s": setup_s,
            "one_at_a_time": {"solve_s": single, "cycles_max": int(max(single_cycles)),
                              "cycles_sum": int(sum(single_cycles))},
            "batch": {"members": len(mem), "levels": int(levels), "rows": int(rows), "create_s": create_s, **runs},
            "autotuner": {"tiles_per_level_coarsest_first": [list(cf.TILES[int(v)]) for v in tiles],
                          "tile_is": "(wavefronts per 64-row slice, entries per lane issued together)",
                          "ms_per_sweep": [float(v) for v in tms], "tune_s": tune_s},
            "speedup_batch_vs_one_at_a_time": single / runs["autotuned_tiles"]["solve_s"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="knot_8m_depth11", choices=list(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--max-coarse", type=int, default=4096,
                    help="coarsest depth = finest with at most this many functions (solved directly)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--no-sphere", action="store_true", help="skip the held-out noisy sphere (8.4M tris, depth 11)")
    ap.add_argument("--fixed-schedule", action="store_true",
                    help="V(2,2) for every solver instead of choosing each one's sweep schedule first")
    ap.add_argument("--no-sheets", action="store_true", help="skip the two-sheet coupling test (depth 8)")
    ap.add_argument("--no-flow", action="store_true", help="skip the config-3 flow steps")
    ap.add_argument("--batch-meshes", type=int, default=64, help="meshes of the config-4 batch (0: skip)")
    ap.add_argument("--batch-only", action="store_true", help="only the config-4 batch")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the roofline measurement: hierarchy, assembly, solver setup (no cycles), then the "
                         "measured kernel; for profiler runs whose only Gauss-Seidel launches are the measured ones")
    ap.add_argument("--flow-only", action="store_true", help="only the config-3 flow steps (for profiler runs)")
    ap.add_argument("--cubes-only", action="store_true",
                    help="only the minimum-depth experiment of Figure cubes (W-cycles, gradient constraint)")
    ap.add_argument("--no-cubes", action="store_true", help="skip the Figure cubes experiment")
    ap.add_argument("--no-stripe-knot", action="store_true",
                    help="skip the stripe-texture colour fit on the self-intersecting knot")
    ap.add_argument("--spectrum-only", action="store_true",
                    help="only the spectral study (nested spheres, resolution and rotation sweeps)")
    ap.add_argument("--no-spectrum", action="store_true", help="skip the spectral study")
    ap.add_argument("--flow-study-only", action="store_true",
                    help="only the cMCF study on the two-lobe surface (split against unsplit)")
    ap.add_argument("--no-flow-study", action="store_true", help="skip the cMCF study")
    ap.add_argument("--assembly-only", action="store_true",
                    help="only the assembly measurement (four meshes, both degrees); for matrix-core counter runs")
    ap.add_argument("--no-assembly", action="store_true", help="skip the assembly measurement")
    ap.add_argument("--build-only", action="store_true",
                    help="only the hierarchy build of the workload, four times (the last three timed); for "
                         "kernel-trace runs of the set-up path")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}))
        sys.exit(2)

    import torch
    from paper_1505_03615_amd import camfe as cf, meshgen
    assert torch.cuda.is_available(), "bench needs a GPU"
    cf.load()
    wl = WORKLOADS[args.workload]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    ctx = cf.camfe_ctx_create(0, stream)

    only = {"flow_config3": (args.flow_only, lambda: flow_eval(cf, ctx, meshgen)),
            "spectrum": (args.spectrum_only, lambda: spectrum_eval(cf, ctx, meshgen)),
            "flow_study": (args.flow_study_only, lambda: flow_study_eval(cf, ctx, meshgen)),
            "colour_fit_cubes": (args.cubes_only, lambda: cubes_eval(cf, ctx, meshgen)),
            "assembly": (args.assembly_only, lambda: assembly_eval(cf, ctx, meshgen)),
            "batch_config4": (args.batch_only, lambda: batch_eval(cf, ctx, meshgen, max(args.batch_meshes, 1)))}
    for key, (flag, fn) in only.items():
        if flag:
            out = {key: fn()}
            cf.camfe_ctx_destroy(ctx)
            print(json.dumps(out), flush=True)
            return

    log(f"[bench] workload {args.workload}: generating the mesh")
    V, F, f = workload_input(meshgen, wl["mesh"])
    Vd = torch.from_numpy(V).to(dev)
    Fd = torch.from_numpy(F).to(dev)
    fd = torch.from_numpy(np.asfortranarray(f)).to(dev)
    traffic_file = TRAFFIC_FILES.get(args.workload)

    if args.build_only:
        times = []
        for i in range(4):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            h = cf.camfe_hierarchy_build(ctx, Vd, Fd, depth=wl["depth"], degree=wl["degree"],
                                         max_coarse=args.max_coarse)
            torch.cuda.synchronize()
            times.append(1000.0 * (time.perf_counter() - t0))
            log(f"[bench] hierarchy build {i}: {times[-1]:.1f} ms")
            cf.camfe_hierarchy_destroy(h)
        cf.camfe_ctx_destroy(ctx)
        print(json.dumps({"hierarchy_build": {"workload": wl["desc"], "ms": times, "best_of_last_3_ms": min(times[1:])}}),
              flush=True)
        return

    if args.roofline_only:
        h = cf.camfe_hierarchy_build(ctx, Vd, Fd, depth=wl["depth"], degree=wl["degree"], max_coarse=args.max_coarse)
        s = cf.camfe_assemble(h)
        b = cf.camfe_load_vector(s, h, fd)
        cf.camfe_solve(s, b, t=wl["t"], rtol=1e-8, max_iter=0)     # solver setup only
        out = {"roofline": roofline(cf, s, "gs_colour", with_traffic=traffic_file is not None,
                                    traffic_file=traffic_file, depth=wl["depth"])}
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)
        if args.calibrate_copy:
            calibrate_copy(torch, dev)
        cf.camfe_ctx_destroy(ctx)
        print(json.dumps(out), flush=True)
        return

    log("[bench] training the learned smoother")
    model, train_info = train_smoother(cf, ctx, meshgen, sweep=1)
    keep = {}
    sched = {}
    if not args.fixed_schedule:
        log("[bench] sweep schedule per solver, chosen on the workload before the warm-up")
        h = cf.camfe_hierarchy_build(ctx, Vd, Fd, depth=wl["depth"], degree=wl["degree"], max_coarse=args.max_coarse)
        s = cf.camfe_assemble(h)
        b = cf.camfe_load_vector(s, h, fd)
        sched = tune_schedules(cf, s, b, wl["t"], model, [tag for tag, _ in SOLVERS])
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)
    learned_kw = schedule_kw(tuple(sched["learned_mixed"]["chosen"]) if sched else (2, 0))

    def step(record, keep_last=False):
        """The whole path once: build, assemble, load, learned mixed solve."""
        t0 = time.perf_counter()
        h = cf.camfe_hierarchy_build(ctx, Vd, Fd, depth=wl["depth"], degree=wl["degree"],
                                     max_coarse=args.max_coarse)
        t1 = time.perf_counter()
        s = cf.camfe_assemble(h)
        t2 = time.perf_counter()
        b = cf.camfe_load_vector(s, h, fd)
        t3 = time.perf_counter()
        cf.camfe_smoother_attach(s, model)
        x, st = cf.camfe_solve(s, b, t=wl["t"], rtol=1e-8, max_iter=4000, precision=1, smoother=2, **learned_kw)
        t4 = time.perf_counter()
        if record is not None:
            record.append(dict(build=t1 - t0, assemble=t2 - t1, load=t3 - t2, solve_call=t4 - t3, st=st))
        if keep_last:
            keep.update(h=h, s=s, b=b, x=x)
        else:
            cf.camfe_system_destroy(s)
            cf.camfe_hierarchy_destroy(h)

    log(f"[bench] warmup {args.warmup}")
    # the first warm-up step runs with per-launch event timing (every launch
    # bracketed, so host gaps inflate small kernels) to rank the kernels
    ranking = {}
    for i in range(args.warmup):
        if i == 0:
            cf.camfe_ctx_kernel_timing(ctx, True)
        step(None)
        if i == 0:
            ranking = {k: cf.camfe_ctx_kernel_time(ctx, k) for k in cf.KERNELS}
            cf.camfe_ctx_kernel_timing(ctx, False)
            log("[bench] kernel event times (ms): " +
                ", ".join(f"{k}={v[0]:.2f}/{v[1]}" for k, v in sorted(ranking.items(), key=lambda kv: -kv[1][0])))
    rec = []
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(rec, keep_last=(i == args.steps - 1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / args.steps
    h, s, b = keep["h"], keep["s"], keep["b"]
    fin, d0 = cf.camfe_hierarchy_levels(h)
    n = cf.camfe_hierarchy_info(h, fin)[2]
    sts = [r["st"] for r in rec]
    solve_s = float(np.mean([x["seconds"] for x in sts]))
    cycles = float(np.mean([x["cycles"] for x in sts]))
    log("[bench] plain Gauss-Seidel solves of the same system")
    comp = solve_comparison(cf, s, h, b, wl["t"], model, which=("plain_gs_fp64", "plain_gs_mixed", "block_fp64"),
                            schedules={k: v["chosen"] for k, v in sched.items()})
    comp["learned_mixed"] = {"s": solve_s, "cycles": cycles, "rel_residual": float(max(x["rel_residual"] for x in sts)),
                             "converged": bool(all(x["converged"] for x in sts)),
                             "fell_back": int(max(x["fell_back"] for x in sts)),
                             "setup_s": float(np.mean([x["setup_seconds"] for x in sts])),
                             "dof_cycles_per_s": n * cycles / solve_s, "timed_steps": len(sts)}
    for k, v in sched.items():
        comp[k]["schedule"] = v
    if not sched:
        comp["schedule"] = "V(2,2) for every solver"
    comp["speedup_learned_mixed_vs_plain_fp64"] = comp["plain_gs_fp64"]["s"] / solve_s
    comp["speedup_learned_mixed_vs_plain_mixed"] = comp["plain_gs_mixed"]["s"] / solve_s
    phases = {k: 1000.0 * float(np.mean([r[k] for r in rec])) for k in ("build", "assemble", "load", "solve_call")}
    out = {
        "metric": "solve time to 1e-8 rel. residual, DoF*cycles/s; learned vs plain smoother",
        "value": solve_s,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 V-cycle (learned SOR smoother, BF16 MLP weights) under f64 CG; f64 assembly",
        "data": "synthetic",
        "config": {"workload": wl["desc"], "dof_finest": int(n), "levels": [fin, d0], "max_coarse": args.max_coarse},
        "value_is": "learned-smoother mixed-precision solve to 1e-8, iterations only (solver set-up in "
                    "solvers.learned_mixed.setup_s), mean over the timed steps; every solver runs the sweep "
                    "schedule that was fastest for it among (sweeps at the finest depth, sweeps below) = "
                    "(2,2), (2,1), (3,1), (1,1) in untimed solves of the same system before the warm-up "
                    "(solvers.<name>.schedule); the held-out sphere and the sheets use V(2,2)",
        "phases_ms": phases,
        "solvers": comp,
        "learned_training": train_info,
    }
    if ranking:
        out["kernel_event_ms_warmup"] = {k: v[0] for k, v in ranking.items() if v[1]}
        a_ms, a_n, a_flops = ranking["assemble"]
        if a_ms > 0:
            tf = a_flops / (a_ms / 1000.0) / 1e12
            out["assembly_mfma"] = {"kernel": "assemble (all depths, FP64 matrix cores)", "ms": a_ms,
                                    "useful_flops": a_flops, "achieved_tflops": tf, "peak_tflops": PEAK_FP64_TFLOPS,
                                    "frac": tf / PEAK_FP64_TFLOPS}
        dom = max(ranking, key=lambda k: ranking[k][0])
        if dom == "assemble":
            tot_ms, launches, work = ranking[dom]
            achieved = work / (tot_ms / 1000.0) / 1e12
            out["roofline"] = {"bound": "mfma", "kernel": dom, "achieved": achieved, "peak": PEAK_FP64_TFLOPS,
                               "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_TFLOPS, "traffic": None}
        else:
            meas = dom if dom in ("gs_colour", "residual", "spmv_dot") else "gs_colour"
            out["roofline"] = roofline(cf, s, meas, with_traffic=traffic_file is not None, traffic_file=traffic_file,
                                       depth=wl["depth"])
        out["roofline"]["whole_vcycle"] = comp["vcycle_roofline"]
        if "vcycle_roofline_chosen_schedule" in comp:
            out["roofline"]["whole_vcycle_chosen_schedule"] = comp["vcycle_roofline_chosen_schedule"]
    cf.camfe_smoother_attach(s, None)
    cf.camfe_system_destroy(s)
    cf.camfe_hierarchy_destroy(h)
    if args.workload == "knot_8m_depth11" and not args.no_sphere:
        out["held_out_sphere"] = system_eval(cf, ctx, meshgen, "sphere_8m_depth11", model, args.max_coarse)
    if not args.no_sheets:
        out["two_sheets_config2"] = system_eval(cf, ctx, meshgen, "two_sheets_256_depth8", model, args.max_coarse)
    if not args.no_flow:
        log("[bench] flow steps (config 3)")
        out["flow_config3"] = flow_eval(cf, ctx, meshgen)
        log("[bench] flow: " + json.dumps(out["flow_config3"]))
    if args.batch_meshes > 0:
        log(f"[bench] batch of {args.batch_meshes} meshes (config 4)")
        out["batch_config4"] = batch_eval(cf, ctx, meshgen, args.batch_meshes)
        log("[bench] batch: " + json.dumps(out["batch_config4"]))
    if not args.no_cubes:
        log("[bench] Figure cubes: one W-cycle per minimum depth, split and unsplit")
        out["colour_fit_cubes"] = cubes_eval(cf, ctx, meshgen)
    if not args.no_stripe_knot:
        log("[bench] stripe texture on a self-intersecting knot, split and unsplit")
        out["colour_fit_stripe_knot"] = stripe_knot_eval(cf, ctx, meshgen)
    if not args.no_flow_study:
        log("[bench] cMCF study: two-lobe surface, split against unsplit")
        out["flow_study"] = flow_study_eval(cf, ctx, meshgen)
    if not args.no_spectrum:
        log("[bench] spectral study: nested spheres, split against unsplit")
        out["spectrum"] = spectrum_eval(cf, ctx, meshgen)
    if not args.no_assembly:
        out["assembly"] = assembly_eval(cf, ctx, meshgen, reps=1)
    if args.calibrate_copy:
        calibrate_copy(torch, dev)
    if not args.no_cpu_baseline and args.workload == "knot_8m_depth11":
        log("[bench] cpu baseline (oracle)")
        # the oracle runs V(2,2)-cycles: scale by the GPU's FP64 V(2,2) cycle count
        c22 = sched["plain_gs_fp64"]["cycles"]["2,0"] if sched else comp["plain_gs_fp64"]["cycles"]
        out["cpu_baseline"] = cpu_baseline(cf, ctx, meshgen, {"dof": int(n), "cycles_fp64": c22, "model": model})
        # every solver's result against the oracle's FP64 solution, on the oracle-sized sample
        out["error_vs_oracle"] = {"sample": out["cpu_baseline"]["sample"].split(";")[0],
                                  **out["cpu_baseline"]["gpu_error_vs_oracle_on_sample"]}
    cf.camfe_model_destroy(model)
    cf.camfe_ctx_destroy(ctx)
    print(json.dumps(out), flush=True)


def system_eval(cf, ctx, meshgen, name, model, max_coarse):
    """Another workload solved once warm with each solver (no timed steps):
    build, assembly and load times, then solve_comparison."""
    import torch
    wl = WORKLOADS[name]
    dev = torch.device("cuda:0")
    log(f"[bench] {name}: generating the mesh")
    V, F, f = workload_input(meshgen, wl["mesh"])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    h = cf.camfe_hierarchy_build(ctx, torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev), depth=wl["depth"],
                                 degree=wl["degree"], max_coarse=max_coarse)
    t1 = time.perf_counter()
    s = cf.camfe_assemble(h)
    t2 = time.perf_counter()
    b = cf.camfe_load_vector(s, h, torch.from_numpy(np.asfortranarray(f)).to(dev))
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    res = {"workload": wl["desc"], "tris": int(len(F)),
           "phases_ms": {"build": 1000 * (t1 - t0), "assemble": 1000 * (t2 - t1), "load": 1000 * (t3 - t2)}}
    res.update(solve_comparison(cf, s, h, b, wl["t"], model))
    cf.camfe_system_destroy(s)
    cf.camfe_hierarchy_destroy(h)
    log(f"[bench] {name}: " + json.dumps(res))
    return res


if __name__ == "__main__":
    main()
