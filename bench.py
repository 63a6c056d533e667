#!/usr/bin/env python3
"""Benchmark of the connectivity-aware multilevel FEM hot path on one MI355X.

One step = the whole path on one synthetic input, inputs resident in HBM:
hierarchy (grid placement, triangle/cell pairs, octree, supports, split,
prolongation), assembly of M and L at every depth, the load vector, and the
solve of (M + t L) x = b to a relative residual of 1e-8 three times: with the
FP64 Gauss-Seidel V-cycle, with the FP32 Gauss-Seidel V-cycle under FP64
refinement, and with the FP32 V-cycle whose smoother is the learned multicolour SOR
(conjugate gradients preconditioned by one V-cycle in all three).  The
learned smoother is trained before timing on small meshes of other shapes.

Workload: two parallel unit squares 1/256 apart, each a 256 x 256 grid of
split quads (262,144 triangles), turned to general position, octree depth 8,
t = 1e-3, RHS +-sin(40 pi x) on the two sheets.

Prints one JSON line.  `value` is finest-depth DoF x V-cycles of the three
solves per second of the whole step; the per-phase times and the solve-only figures
are reported beside it.
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
    "two_sheets_256_depth8": dict(mesh="two_sheets_256", depth=8, t=1e-3, degree=1),
    # for --roofline-only: the colour sweep at the knot's 2.2M-function depth 10
    "knot_2m_depth10": dict(mesh="knot_2m", depth=10, t=1e-4, degree=1),
}
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(sample_n=128, sample_depth=7):
    """The oracle (single-threaded FP64 C++) on a bounded sample of the same
    workload: the two-sheet coupling test at 128 x 128 quads per sheet and
    depth 7 (a quarter of the triangles, same voxel-to-triangle ratio)."""
    from oracle import Oracle
    from paper_1505_03615_amd import meshgen
    V, F, f = meshgen.config_mesh("two_sheets", n=sample_n, gap=1.0 / sample_n)
    t0 = time.perf_counter()
    o = Oracle(V, F, sample_depth, max_coarse=2048).check().assemble()
    b = o.load_vector(f)
    x, info = o.solve(1e-3, b, rtol=1e-8, max_iter=2000)
    secs = time.perf_counter() - t0
    n = o.count(sample_depth, "functions")
    return {"value": n * info["cycles"] / secs, "unit": "DoF*cycles/s", "cores": 1, "kind": "oracle",
            "sample": f"two sheets {sample_n}x{sample_n} quads each ({len(F)} tris), depth {sample_depth}, "
                      f"n={n}, FP64 V-cycle-preconditioned CG to 1e-8: {info['cycles']} cycles in {secs:.2f} s "
                      f"(build+assemble+load+solve)",
            "seconds": secs, "converged": bool(info["converged"])}


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "gs_colour_two_sheets_d8_traffic.md")
TRAFFIC_FILE_D10 = os.path.join(ROOT, "profiles", "gs_colour_knot_d10_traffic.md")
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


def roofline(cf, s, meas, reps=50, with_traffic=True, main_precision=1):
    """Algorithmic bytes of one launch of the finest-depth kernel over its
    average duration (HIP events around a captured graph of back-to-back
    launches on the library's stream), against the HBM peak, in both
    precisions.  The top level describes main_precision (1: the FP32 sweep,
    which takes the larger share of the bench step: the mixed and the
    learned solves run it), the other precision sits beside it.
    with_traffic: attach the committed counter figures (taken on the
    two-sheet depth-8 workload only)."""
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
                  "traffic": measured_traffic(TRAFFIC_FILE, key) if (meas == "gs_colour" and with_traffic) else None,
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


def held_out_eval(cf, ctx, meshgen, model, size, model_jacobi=None):
    """Held-out meshes (never trained on): the (3,5) knot tube and a noisy
    sphere, each about 8.4M triangles at depth 11 (size 'full'), or 2.1M at
    depth 10 ('small').  Solve (M + t L) x = b to 1e-8 with the plain FP64
    Gauss-Seidel V-cycle and with the learned smoother in mixed precision;
    each solve is run twice and the second (warm) run is reported."""
    import torch
    full = size == "full"
    meshes = {
        "knot": (meshgen.torus_knot(nu=65536 if full else 16384, nv=64, seed=3), 11 if full else 10, 1e-4),
        "noisy_sphere": (meshgen.noisy_sphere(10 if full else 9, seed=7, base="octa"), 11 if full else 10, 1e-3),
    }
    out = {}
    dev = torch.device("cuda:0")
    for name, ((V, F), depth, t) in meshes.items():
        log(f"[bench] held-out {name}: {len(F)} tris, depth {depth}")
        h = cf.camfe_hierarchy_build(ctx, torch.from_numpy(V).to(dev), torch.from_numpy(F).to(dev), depth=depth,
                                     degree=1, max_coarse=4096)
        s = cf.camfe_assemble(h)
        fv = torch.from_numpy(np.asfortranarray(V[:, 2:3] + 0.1 * V[:, 0:1] ** 2)).to(dev)
        b = cf.camfe_load_vector(s, h, fv)
        n = cf.camfe_hierarchy_info(h, depth)[2]
        res = {"tris": int(len(F)), "depth": depth, "t": t, "dof": int(n)}
        runs = [("plain_gs_fp64", dict(precision=0, smoother=0), None),
                ("plain_gs_mixed", dict(precision=1, smoother=0), None),
                ("learned_mixed", dict(precision=1, smoother=2), model)]
        if model_jacobi is not None:
            runs.append(("learned_jacobi_mixed", dict(precision=1, smoother=2), model_jacobi))
        for tag, kw, mdl in runs:
            cf.camfe_smoother_attach(s, mdl)
            for _ in range(2):
                x, st = cf.camfe_solve(s, b, t=t, rtol=1e-8, max_iter=3000, **kw)
            res[tag] = {"ms": 1000.0 * st["seconds"], "cycles": st["cycles"], "rel_residual": st["rel_residual"],
                        "converged": bool(st["converged"]), "fell_back": int(st["fell_back"])}
            log(f"[bench] held-out {name} {tag}: {res[tag]['cycles']} cycles, {res[tag]['ms']:.0f} ms")
        res["speedup_learned_vs_plain"] = res["plain_gs_fp64"]["ms"] / res["learned_mixed"]["ms"]
        # whole V-cycle (inside CG, whose vector work is not counted) against the HBM peak
        b64 = vcycle_bytes(cf, s, h, 1, 8, 8)
        b32 = vcycle_bytes(cf, s, h, 1, 4, 4)
        res["vcycle_roofline"] = {
            "plain_gs_fp64": cycle_roofline(b64, res["plain_gs_fp64"]["ms"], res["plain_gs_fp64"]["cycles"]),
            "plain_gs_mixed": cycle_roofline(b32, res["plain_gs_mixed"]["ms"], res["plain_gs_mixed"]["cycles"])}
        cf.camfe_smoother_attach(s, None)
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)
        out[name] = res
        log(f"[bench] held-out {name}: " + json.dumps(res))
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
    big = roofline(cf, s, "gs_colour", reps=10, with_traffic=False)
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


def batch_eval(cf, ctx, meshgen, count=16, seed=4000):
    """Config 4 (scaled): `count` meshes of uneven size (icospheres, tori,
    noise-displaced spheres), depth clamp(round(log2(side / mean edge)), 6, 10),
    1-16 random right-hand sides each; one batched solve against the same
    systems solved one at a time (FP64, 1e-8)."""
    import torch
    rng = np.random.default_rng(seed)
    systems, rhs = [], []
    dev = torch.device("cuda:0")
    for i in range(count):
        kind = i % 3
        if kind == 0:
            V, F = meshgen.icosphere(int(rng.integers(3, 7)))
        elif kind == 1:
            R = float(rng.uniform(2.0, 6.0))
            nu = int(rng.integers(24, 400))
            V, F = meshgen.torus(R, 1.0, nu, max(8, int(nu / R)))
        else:
            V, F = meshgen.noisy_sphere(int(rng.integers(3, 7)), seed=seed + i)
        e = np.linalg.norm(V[F[:, 1]] - V[F[:, 0]], axis=1).mean()
        side = 1.125 * (V.max(0) - V.min(0)).max()
        depth = int(np.clip(round(np.log2(side / e)), 6, 10))
        h = cf.camfe_hierarchy_build(ctx, V, F, depth=depth, degree=1, max_coarse=4096)
        sy = cf.camfe_assemble(h)
        k = int(rng.integers(1, 17))
        b = cf.camfe_load_vector(sy, h, rng.normal(size=(len(V), k)))
        systems.append((h, sy, len(F), depth, k))
        rhs.append(b)
    t_single = 0.0
    for (h, sy, nt, depth, k), b in zip(systems, rhs):
        cf.camfe_solve(sy, b, t=1e-3, rtol=1e-8, max_iter=600)      # setup and capture
        x, st = cf.camfe_solve(sy, b, t=1e-3, rtol=1e-8, max_iter=600)
        t_single += st["seconds"]
    t0 = time.perf_counter()
    bt = cf.camfe_batch_create(ctx, [x[1] for x in systems], 1e-3)
    create = time.perf_counter() - t0
    xs, sts = cf.camfe_batch_solve(bt, rhs, 1e-3, rtol=1e-8, max_iter=600)    # capture
    xs, sts = cf.camfe_batch_solve(bt, rhs, 1e-3, rtol=1e-8, max_iter=600)
    levels, rows = cf.camfe_batch_info(bt)
    cf.camfe_batch_destroy(bt)
    # the same work as one member per (mesh, chunk of <= 4 columns): a single
    # pass of the batch then covers every column, where the per-mesh layout
    # takes one pass per column chunk over all meshes
    members, chunks = [], []
    for (h, sy, nt, depth, k), b in zip(systems, rhs):
        for c0 in range(0, k, 4):
            members.append(sy)
            chunks.append(np.asfortranarray(b[:, c0:c0 + 4]))
    t0 = time.perf_counter()
    bt = cf.camfe_batch_create(ctx, members, 1e-3)
    create_c = time.perf_counter() - t0
    xc, stc = cf.camfe_batch_solve(bt, chunks, 1e-3, rtol=1e-8, max_iter=600)    # capture
    xc, stc = cf.camfe_batch_solve(bt, chunks, 1e-3, rtol=1e-8, max_iter=600)
    levels_c, rows_c = cf.camfe_batch_info(bt)
    cf.camfe_batch_destroy(bt)
    out = {"meshes": count, "tris": [int(x[2]) for x in systems], "depths": [int(x[3]) for x in systems],
           "rhs": [int(x[4]) for x in systems], "batch_rows": int(rows), "batch_levels": int(levels),
           "batch_create_ms": 1000.0 * create, "batch_solve_ms": 1000.0 * sts[0]["seconds"],
           "one_at_a_time_solve_ms": 1000.0 * t_single,
           "all_converged": bool(all(x["converged"] for x in sts)),
           "max_rel_residual": float(max(x["rel_residual"] for x in sts)),
           "per_chunk_members": len(members), "per_chunk_rows": int(rows_c),
           "per_chunk_create_ms": 1000.0 * create_c, "per_chunk_solve_ms": 1000.0 * stc[0]["seconds"],
           "per_chunk_all_converged": bool(all(x["converged"] for x in stc)),
           "per_chunk_max_rel_residual": float(max(x["rel_residual"] for x in stc))}
    for h, sy, _, _, _ in systems:
        cf.camfe_system_destroy(sy)
        cf.camfe_hierarchy_destroy(h)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="two_sheets_256_depth8", choices=list(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--max-coarse", type=int, default=4096,
                    help="coarsest depth = finest with at most this many functions (solved directly)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--held-out", default="small", choices=["full", "small", "none"],
                    help="learned-smoother evaluation on held-out meshes (8.4M or 2.1M tris)")
    ap.add_argument("--no-flow", action="store_true", help="skip the config-3 flow steps")
    ap.add_argument("--batch-meshes", type=int, default=16, help="meshes of the config-4 batch (0: skip)")
    ap.add_argument("--roofline-only", action="store_true",
                    help="only the roofline measurement: hierarchy, assembly, solver setup (no cycles), then the "
                         "measured kernel; for profiler runs whose only Gauss-Seidel launches are the measured ones")
    ap.add_argument("--flow-only", action="store_true", help="only the config-3 flow steps (for profiler runs)")
    ap.add_argument("--cubes-only", action="store_true",
                    help="only the minimum-depth experiment of Figure cubes (W-cycles, gradient constraint)")
    ap.add_argument("--no-cubes", action="store_true", help="skip the Figure cubes experiment")
    ap.add_argument("--nu-coarse", default="auto",
                    help="sweeps each way below the finest depth in the step's solves: 'auto' (the warm-up times "
                         "(finest, below) = (2, 2), (2, 1) and (3, 1) per solve and keeps the fastest) or an "
                         "integer (with two sweeps each way at the finest depth; 0: as at the finest)")
    ap.add_argument("--spectrum-only", action="store_true",
                    help="only the spectral study (nested spheres, resolution and rotation sweeps)")
    ap.add_argument("--no-spectrum", action="store_true", help="skip the spectral study")
    ap.add_argument("--flow-study-only", action="store_true",
                    help="only the cMCF study on the two-lobe surface (split against unsplit)")
    ap.add_argument("--no-flow-study", action="store_true", help="skip the cMCF study")
    ap.add_argument("--assembly-only", action="store_true",
                    help="only the assembly measurement (four meshes, both degrees); for matrix-core counter runs")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build measures one GPU only; run with --gpus 1"}))
        sys.exit(2)

    import torch
    from paper_1505_03615_amd import camfe as cf, meshgen
    assert torch.cuda.is_available(), "bench needs a GPU"
    cf.load()
    wl = WORKLOADS[args.workload]
    V, F, f = meshgen.config_mesh(wl["mesh"])
    dev = torch.device("cuda:0")
    Vd = torch.from_numpy(V).to(dev)
    Fd = torch.from_numpy(F).to(dev)
    fd = torch.from_numpy(np.asfortranarray(f)).to(dev)
    stream = torch.cuda.current_stream()
    ctx = cf.camfe_ctx_create(0, stream)

    if args.flow_only:
        out = {"flow_config3": flow_eval(cf, ctx, meshgen)}
        cf.camfe_ctx_destroy(ctx)
        print(json.dumps(out), flush=True)
        return

    if args.spectrum_only:
        out = {"spectrum": spectrum_eval(cf, ctx, meshgen)}
        cf.camfe_ctx_destroy(ctx)
        print(json.dumps(out), flush=True)
        return

    if args.flow_study_only:
        out = {"flow_study": flow_study_eval(cf, ctx, meshgen)}
        cf.camfe_ctx_destroy(ctx)
        print(json.dumps(out), flush=True)
        return

    if args.cubes_only:
        out = {"colour_fit_cubes": cubes_eval(cf, ctx, meshgen)}
        cf.camfe_ctx_destroy(ctx)
        print(json.dumps(out), flush=True)
        return

    if args.assembly_only:
        out = {"assembly": assembly_eval(cf, ctx, meshgen)}
        cf.camfe_ctx_destroy(ctx)
        print(json.dumps(out), flush=True)
        return

    if args.roofline_only:
        h = cf.camfe_hierarchy_build(ctx, Vd, Fd, depth=wl["depth"], degree=wl["degree"], max_coarse=args.max_coarse)
        s = cf.camfe_assemble(h)
        b = cf.camfe_load_vector(s, h, fd)
        cf.camfe_solve(s, b, t=wl["t"], rtol=1e-8, max_iter=0)     # solver setup only
        out = {"roofline": roofline(cf, s, "gs_colour", with_traffic=args.workload == "two_sheets_256_depth8")}
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)
        if args.calibrate_copy:
            calibrate_copy(torch, dev)
        cf.camfe_ctx_destroy(ctx)
        print(json.dumps(out), flush=True)
        return

    keep = {}
    log("[bench] training the learned smoothers")
    model, train_info = train_smoother(cf, ctx, meshgen, sweep=1)
    model_jac, train_info_jac = train_smoother(cf, ctx, meshgen, sweep=0)

    SOLVES = (("plain_fp64", dict(precision=0, max_iter=2000)), ("mixed_fp32_fp64", dict(precision=1, max_iter=2000)),
              ("learned_mixed", dict(precision=1, smoother=2, max_iter=4000)))
    # (sweeps each way at the finest depth, below it; 0: as at the finest)
    nuc = {k: (2, 0 if args.nu_coarse == "auto" else int(args.nu_coarse)) for k, _ in SOLVES}
    tune = {}

    def autotune():
        """Time each solve to 1e-8 with (finest, below) sweeps (2, 2), (2, 1)
        and (3, 1) (best of two, warm) and keep the fastest: the paper fixes
        no sweep count."""
        h = cf.camfe_hierarchy_build(ctx, Vd, Fd, depth=wl["depth"], degree=wl["degree"], max_coarse=args.max_coarse)
        s = cf.camfe_assemble(h)
        b = cf.camfe_load_vector(s, h, fd)
        cf.camfe_smoother_attach(s, model)
        for key, kw in SOLVES:
            tune[key] = {}
            for nu, nc in ((2, 0), (2, 1), (3, 1)):
                best = float("inf")
                for _ in range(2):
                    _, st = cf.camfe_solve(s, b, t=wl["t"], rtol=1e-8, nu_pre=nu, nu_post=nu, nu_coarse=nc, **kw)
                    if st["converged"] and not st["fell_back"]:
                        best = min(best, 1000.0 * st["seconds"])
                tune[key][nu, nc] = best
            nuc[key] = min(tune[key], key=tune[key].get)
        cf.camfe_system_destroy(s)
        cf.camfe_hierarchy_destroy(h)
        log("[bench] sweep autotune (iteration ms): " +
            json.dumps({k: {f"{a},{c}": v for (a, c), v in d.items()} for k, d in tune.items()}) +
            " -> " + json.dumps(nuc))

    def step(record, keep_last=False):
        t0 = time.perf_counter()
        h = cf.camfe_hierarchy_build(ctx, Vd, Fd, depth=wl["depth"], degree=wl["degree"],
                                     max_coarse=args.max_coarse)
        t1 = time.perf_counter()
        s = cf.camfe_assemble(h)
        t2 = time.perf_counter()
        b = cf.camfe_load_vector(s, h, fd)
        t3 = time.perf_counter()
        sw = {k: dict(nu_pre=v[0], nu_post=v[0], nu_coarse=v[1]) for k, v in nuc.items()}
        x64, st64 = cf.camfe_solve(s, b, t=wl["t"], rtol=1e-8, max_iter=2000, precision=0, **sw["plain_fp64"])
        t4 = time.perf_counter()
        x32, st32 = cf.camfe_solve(s, b, t=wl["t"], rtol=1e-8, max_iter=2000, precision=1, **sw["mixed_fp32_fp64"])
        t5 = time.perf_counter()
        cf.camfe_smoother_attach(s, model)
        xl, stl = cf.camfe_solve(s, b, t=wl["t"], rtol=1e-8, max_iter=4000, precision=1, smoother=2,
                                 **sw["learned_mixed"])
        t6 = time.perf_counter()
        fin, d0 = cf.camfe_hierarchy_levels(h)
        n = cf.camfe_hierarchy_info(h, fin)[2]
        if record is not None:
            record.append(dict(build=t1 - t0, assemble=t2 - t1, load=t3 - t2, solve64=t4 - t3, solve32=t5 - t4,
                               solvel=t6 - t5, st64=st64, st32=st32, stl=stl, n=n, levels=(fin, d0),
                               xs=(x64, x32, xl)))
        if keep_last:
            keep["h"], keep["s"] = h, s
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
    if args.nu_coarse == "auto":
        autotune()
    rec = []
    torch.cuda.synchronize()
    log(f"[bench] timing {args.steps} steps")
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(rec, keep_last=(i == args.steps - 1))
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1000.0 / args.steps
    n = rec[0]["n"]
    cyc64 = np.mean([r["st64"]["cycles"] for r in rec])
    cyc32 = np.mean([r["st32"]["cycles"] for r in rec])
    cycl = np.mean([r["stl"]["cycles"] for r in rec])
    solve64 = np.mean([r["solve64"] for r in rec])
    solve32 = np.mean([r["solve32"] for r in rec])
    solvel = np.mean([r["solvel"] for r in rec])
    phases = {k: 1000.0 * float(np.mean([r[k] for r in rec]))
              for k in ("build", "assemble", "load", "solve64", "solve32", "solvel")}
    out = {
        "metric": "solve time to 1e-8 rel. residual, DoF*cycles/s; learned vs plain smoother",
        "value": n * (cyc64 + cyc32 + cycl) / (ms / 1000.0),
        "unit": "DoF*cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 (mixed-precision solve: f32 V-cycle, f64 CG)",
        "data": "synthetic",
        "config": {"workload": "two parallel unit squares 1/256 apart, 2 x 256 x 256 split quads "
                               "(262,144 tris), rotated to general position, octree depth 8, degree 1, "
                               "split, t=1e-3, RHS +-sin(40 pi x)",
                   "dof_finest": int(n), "levels": list(rec[0]["levels"]), "max_coarse": args.max_coarse},
        "phases_ms": phases,
        # sweeps each way (at the finest depth, below it; 0: as at the finest), per solve
        "sweeps_finest_below": {k: list(v) for k, v in nuc.items()},
        "sweep_autotune_iteration_ms": {k: {f"{a},{c}": v for (a, c), v in d.items()} for k, d in tune.items()},
        "solve_to_1e-8_ms": {"plain_fp64": 1000.0 * solve64, "mixed_fp32_fp64": 1000.0 * solve32,
                             "learned_mixed": 1000.0 * solvel},
        "solve_cycles": {"plain_fp64": float(cyc64), "mixed_fp32_fp64": float(cyc32), "learned_mixed": float(cycl)},
        # the iterations alone (solver setup excluded), and the setup the first solve of a system pays
        "solve_iterations_ms": {k: 1000.0 * float(np.mean([r[st]["seconds"] for r in rec]))
                                for k, st in (("plain_fp64", "st64"), ("mixed_fp32_fp64", "st32"),
                                              ("learned_mixed", "stl"))},
        "solver_setup_ms": 1000.0 * float(np.mean([r["st64"]["setup_seconds"] for r in rec])),
        "solve_dof_cycles_per_s": {"plain_fp64": n * cyc64 / solve64, "mixed_fp32_fp64": n * cyc32 / solve32,
                                   "learned_mixed": n * cycl / solvel},
        "rel_residual": {"plain_fp64": float(max(r["st64"]["rel_residual"] for r in rec)),
                         "mixed_fp32_fp64": float(max(r["st32"]["rel_residual"] for r in rec)),
                         "learned_mixed": float(max(r["stl"]["rel_residual"] for r in rec))},
        "learned_fell_back": int(max(r["stl"]["fell_back"] for r in rec)),
        # difference of each solution from the FP64 one (all three reach 1e-8 residuals)
        "rel_diff_from_fp64_solution": {
            "mixed_fp32_fp64": max(float(torch.linalg.norm(r["xs"][1] - r["xs"][0]) / torch.linalg.norm(r["xs"][0]))
                                   for r in rec),
            "learned_mixed": max(float(torch.linalg.norm(r["xs"][2] - r["xs"][0]) / torch.linalg.norm(r["xs"][0]))
                                 for r in rec)},
        "learned_training": train_info,
        "learned_jacobi_training": train_info_jac,
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
            out["roofline"] = roofline(cf, keep["s"], meas)
    cf.camfe_system_destroy(keep["s"])
    cf.camfe_hierarchy_destroy(keep["h"])
    if args.held_out != "none":
        out["learned_held_out"] = held_out_eval(cf, ctx, meshgen, model, args.held_out, model_jac)
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
    if not args.no_flow_study:
        log("[bench] cMCF study: two-lobe surface, split against unsplit")
        out["flow_study"] = flow_study_eval(cf, ctx, meshgen)
    if not args.no_spectrum:
        log("[bench] spectral study: nested spheres, split against unsplit")
        out["spectrum"] = spectrum_eval(cf, ctx, meshgen)
    cf.camfe_model_destroy(model)
    cf.camfe_model_destroy(model_jac)
    if args.calibrate_copy:
        calibrate_copy(torch, dev)
    if not args.no_cpu_baseline:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline()
    cf.camfe_ctx_destroy(ctx)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
