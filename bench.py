"""Benchmark: matrix-free operator throughput and time to solve on one MI355X.

Workload (N=1): the Poisson problem on [0,1]^3, 16^3 coarse cubes refined
four times towards the corner at the origin (cells with centre within 0.5),
one-irregular, Q4 elements with 5^3 Gauss points: 1,068,726 cells, about 68M
free DoFs.  A *step* is one application of the matrix-free operator of the
finest level to a vector (gather with hanging-node constraints, sum
factorisation, quadrature-point scaling, transposed steps, constrained
scatter-add) in FP64, the paper's vmult.  ``value`` = free DoFs x steps / time
of the timed region (inputs resident in HBM).  After the timed region the
script solves the same problem to a relative residual of 1e-10 with the FP64
V-cycle and with the FP32 V-cycle (FP64 CG), and reports both times; it also
times, on the 2808-cell Q2 mesh, the plain FP64 solve, the mixed-precision
variant (FP32 levels, bfloat16 on the two coarsest) and the learned coarse
correction (trained on the GPU on 20,000 coarse right-hand sides recorded from
the solver); and the batch of 8 right-hand sides solved in one call with
polynomial coarsening Q6 -> Q3 -> Q1 on the 306,536-cell sphere-shell mesh.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "vmult_q4_cube16_ball4_hbm_traffic.md")
# sources that determine the operator kernels, their metadata and their compilation
OPERATOR_SOURCES = [os.path.join("paper_2203_12292_amd", "csrc", f) for f in
                    ("kernels.hip", "kernels.hpp", "slots.hpp", "dofs.cpp", "dofs.hpp", "fe1d.hpp", "common.hpp")]
OPERATOR_SOURCES.append(os.path.join("paper_2203_12292_amd", "build.py"))


def operator_source_digest():
    h = hashlib.sha256()
    for f in OPERATOR_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic():
    """HBM bytes per operator application from the committed counter summary,
    or None when the operator's sources changed after the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as fh:
            text = fh.read()
    except OSError:
        return None
    m_sha = re.search(r"source_sha256:\s*([0-9a-f]{64})", text)
    m_val = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    if not (m_sha and m_val) or m_sha.group(1) != operator_source_digest():
        return None
    return float(m_val.group(1))


def _pmc_rows(folder, counter):
    """(dispatch id, kernel name, grid size, value) of every dispatch in a
    rocprofv3 --pmc csv output folder for one counter, in dispatch order."""
    out = []
    for path in glob.glob(os.path.join(folder, "**", "*counter_collection.csv"), recursive=True):
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                out.append((int(row["Dispatch_Id"]), _kname(row["Kernel_Name"]), int(row["Grid_Size"]),
                            float(row["Counter_Value"])))
    return sorted(out)


def _kname(name):
    """Kernel name without return type, namespace and argument list."""
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(")[0].replace("void ", "").replace("mfmg::", "").strip()


# the plain FP64 Q4 operator on one vector, axis-aligned cells, default mode
# (fused kind 4: no fused step, the shared DoFs' contributions added to the
# output atomically) and the clearing of the output's shared DoFs before it
_Q4_VMULT = re.compile(r"vmult_batch_kernel<4, double, double, 4(, 0)?(, false)?>$")
_Q4_CLEAR = "clear_shared_kernel<double>"


def _q4_pairs(rows):
    """Finest-level applications in a list of (t0, name, grid, value) rows:
    each batch-kernel dispatch with the shared-DoF clearing just before it;
    the finest level is the pair whose clearing has the largest grid (it is
    sized by the level's shared DoFs).  Returns [(clear row, batch row)]."""
    pairs = [(rows[q], rows[q + 1]) for q in range(len(rows) - 1)
             if rows[q][1] == _Q4_CLEAR and _Q4_VMULT.match(rows[q + 1][1])]
    g = max(a[2] for a, _ in pairs)
    return [(a, b) for a, b in pairs if a[2] == g]


def trace_summary(trace_csv, bench_json, commands):
    """Markdown summary of a rocprofv3 --kernel-trace run of this script: the
    finest-level operator dispatches (largest grid of each operator kernel)
    against the benchmark's own HIP-event average, and the top kernels."""
    import numpy as np
    rows = []
    with open(trace_csv, newline="") as fh:
        for r in csv.DictReader(fh):
            if r.get("Kind", "KERNEL_DISPATCH") != "KERNEL_DISPATCH":
                continue
            grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
            t0, t1 = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
            rows.append((t0, _kname(r["Kernel_Name"]), grid, (t1 - t0) * 1e-3))
    rows.sort()
    with open(bench_json) as fh:
        bench = json.loads(fh.read().strip().splitlines()[-1])
    sel = _q4_pairs(rows)
    vm_name = sel[0][1][1]
    clr = (sel[0][0][2], len(sel), float(np.mean([a[3] for a, _ in sel])))
    vm = (sel[0][1][2], len(sel), float(np.mean([b[3] for _, b in sel])))
    rows = [(name, g, us) for _, name, g, us in rows]
    ev = bench["roofline"]["avg_launch_ms"] * 1e3
    tot = {}
    for name, _, us in rows:
        t = tot.setdefault(name, [0.0, 0])
        t[0] += us
        t[1] += 1
    top = sorted(tot.items(), key=lambda kv: -kv[1][0])[:12]
    alg = bench["roofline"]["alg_bytes_per_launch"]
    cfg = bench["config"]
    lines = [
        "# Operator (vmult) on the 16^3 + 4 ball-step mesh, Q4, FP64 - kernel trace",
        "",
        f"Workload: {cfg['cells']} cells ({cfg['hanging_cells']} with hanging nodes), Q4,",
        f"{cfg['free_dofs']} free DoFs.  Command (repository root on the GPU machine), then this summary:",
        "",
    ] + [f"    {c}" for c in commands] + [
        "",
        "| finest-level kernel | grid (work items) | dispatches | average |",
        "|---|---:|---:|---:|",
        f"| {_Q4_CLEAR} | {clr[0]} | {clr[1]} | {clr[2]:.1f} us |",
        f"| {vm_name} | {vm[0]} | {vm[1]} | {vm[2]:.1f} us |",
        f"| sum = one operator application | | | {vm[2] + clr[2]:.1f} us |",
        "",
        f"The benchmark's HIP-event average over its {bench['steps']} timed steps in the same run: {ev:.1f} us",
        f"per application ({100.0 * abs(ev - vm[2] - clr[2]) / ev:.1f} % from the trace).",
        "",
        f"Algorithmic traffic 16 B/DoF = {alg / 1e9:.3f} GB per application -> "
        f"{alg / ((vm[2] + clr[2]) * 1e-6) / 1e9:.0f} GB/s from the trace,",
        f"{bench['roofline']['achieved']:.0f} GB/s from the events "
        f"({100.0 * bench['roofline']['frac']:.1f} % of 8 TB/s).",
        "",
        "Top kernels of the whole run (all levels, set-up and solves included):",
        "",
        "| total | calls | average | kernel |",
        "|---:|---:|---:|---|",
    ] + [f"| {t[0] / 1e3:.1f} ms | {t[1]} | {t[0] / t[1]:.1f} us | {k} |" for k, t in top]
    return "\n".join(lines)


def pmc_summary(fetch_dir, write_dir, n, commands):
    """Markdown summary of the two counter passes: HBM bytes of one finest-level
    operator application (shared-DoF clearing + batch kernel), calibrated by a
    plain elementwise kernel that reads and writes n doubles."""
    import numpy as np

    def pick(rows):
        """(mean value, dispatches, grid) of the finest-level shared-DoF
        clearing and batch kernel and of the calibration copy (elementwise
        kernel with the largest grid)."""
        sel = _q4_pairs(rows)
        cp = [r for r in rows if "elementwise_kernel" in r[1]]
        cp_g = max(r[2] for r in cp)
        cp = [r for r in cp if r[2] == cp_g]
        return {"clear": (float(np.mean([a[3] for a, _ in sel])), len(sel), sel[0][0][2]),
                "vmult": (float(np.mean([b[3] for _, b in sel])), len(sel), sel[0][1][2]),
                "copy": (float(np.mean([r[3] for r in cp])), len(cp), cp_g)}

    res = {}
    for label, folder, counter in (("fetch", fetch_dir, "FETCH_SIZE"), ("write", write_dir, "WRITE_SIZE")):
        res[label] = pick(_pmc_rows(folder, counter))
    f_fetch = 8.0 * n / (res["fetch"]["copy"][0] * 1024.0)
    f_write = 8.0 * n / (res["write"]["copy"][0] * 1024.0)
    kib = {lab: res[lab]["vmult"][0] + res[lab]["clear"][0] for lab in ("fetch", "write")}
    traffic = kib["fetch"] * 1024.0 * f_fetch + kib["write"] * 1024.0 * f_write
    alg = 16.0 * n
    lines = [
        "# HBM traffic of one operator application, 16^3 + 4 ball-step mesh, Q4, FP64",
        "",
        f"{n} free DoFs.  Two counter passes of the benchmark (the finest-level",
        "applications are the (shared-DoF clearing, batch kernel) dispatch",
        "pairs whose clearing has the largest grid), then this summary:",
        "",
    ] + [f"    {c}" for c in commands] + [
        "",
        "| kernel | grid | dispatches | FETCH_SIZE (KiB) | WRITE_SIZE (KiB) |",
        "|---|---:|---:|---:|---:|",
    ]
    for key, name in (("clear", _Q4_CLEAR), ("vmult", "vmult_batch_kernel<4, double, double, 4, ...> (plain FP64 operator)"),
                      ("copy", "elementwise kernel y = 1.0 * x (calibration, n doubles)")):
        fv, fd, fg = res["fetch"][key]
        wv, _, _ = res["write"][key]
        lines.append(f"| {name} | {fg} | {fd} | {fv:.0f} | {wv:.0f} |")
    lines += [
        "",
        f"Calibration: the copy moves 8n = {8 * n} bytes each way; counter scale",
        f"factors {f_fetch:.4f} (FETCH_SIZE) and {f_write:.4f} (WRITE_SIZE).",
        "",
        f"traffic_bytes_per_launch: {traffic:.0f}",
        f"algorithmic_bytes_per_launch: {alg:.0f}",
        f"traffic / algorithmic: {traffic / alg:.3f}",
        f"source_sha256: {operator_source_digest()}",
        "",
        "The benchmark reports this traffic only while the hash of the operator",
        "sources (kernels, metadata layout, build flags) still matches.",
    ]
    return "\n".join(lines)


class _Progress(dict):
    """Result dict that reports each finished stage on stderr."""

    def __setitem__(self, key, value):
        super().__setitem__(key, value)
        print(f"[bench] {key}: {json.dumps(value)[:200]}", file=sys.stderr, flush=True)


def _events_time(fn, k, stream):
    import torch
    starts = [torch.cuda.Event(enable_timing=True) for _ in range(k)]
    ends = [torch.cuda.Event(enable_timing=True) for _ in range(k)]
    for i in range(k):
        starts[i].record(stream)
        fn()
        ends[i].record(stream)
    torch.cuda.synchronize()
    return [s.elapsed_time(e) for s, e in zip(starts, ends)]


def _ebe_passes(local, x, seconds):
    """Passes of the oracle's element-by-element apply over `local` in `seconds`
    (one thread)."""
    from threadpoolctl import threadpool_limits
    with threadpool_limits(limits=1):
        t0 = time.time()
        passes = 0
        while True:
            for (C, Ae, _), xl in zip(local, x):
                _ = C.T @ (Ae @ (C @ xl))
            passes += 1
            if time.time() - t0 >= seconds:
                break
        return passes, time.time() - t0


_EBE = {}


def _ebe_worker(args):
    lo, hi, seconds = args
    local, x = _EBE["local"], _EBE["x"]
    passes, dt = _ebe_passes(local[lo:hi], x[lo:hi], seconds)
    return passes * (hi - lo), dt


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(desc, k, target_seconds=10.0, max_cells=4000):
    """The oracle's element-by-element operator (sum_e C_e^T A_e C_e x) timed
    on a bounded sample of the workload's cells (set-up of the constraint rows
    excluded, as the GPU set-up is): on one core, and on every core of the
    host (the sample split over one process per core, all timed at once).
    Returns cells/s for both, the core counts and the sample size."""
    import multiprocessing as mp

    import numpy as np

    from oracle import fe, octree
    from oracle.space import Space
    tree = octree.build_mesh(desc)
    S = Space(tree, k, build=False)
    n_cells_total = len(S.cells)
    rng = np.random.default_rng(0)
    sample = [S.cells[i] for i in sorted(rng.choice(n_cells_total, size=min(max_cells, n_cells_total),
                                                     replace=False))]
    Aref = fe.reference_stiffness(k)
    local = []
    t_setup = time.time()
    for cell in sample:
        rows = S.cell_rows(cell)
        keys = sorted({kk for row in rows for kk, _ in row})
        pos = {kk: q for q, kk in enumerate(keys)}
        C = np.zeros((len(rows), len(keys)))
        for r, row in enumerate(rows):
            for kk, v in row:
                C[r, pos[kk]] += v
        local.append((C, S.cell_h(cell) * Aref, len(keys)))
        if time.time() - t_setup > 60:
            break
    x = [np.random.default_rng(i).uniform(-1, 1, m) for i, (_, _, m) in enumerate(local)]
    passes, dt = _ebe_passes(local, x, target_seconds)
    one = passes * len(local) / dt
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    _EBE["local"], _EBE["x"] = local, x
    m = len(local)
    chunks = [(m * w // cores, m * (w + 1) // cores, target_seconds) for w in range(cores)]
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_ebe_worker, chunks)
    _EBE.clear()
    allc = sum(cells / dt for cells, dt in res)
    return {"cells_per_s_1core": one, "cells_per_s_all": allc, "cores": cores, "n_sample": m,
            "n_cells_total": n_cells_total, "seconds": target_seconds}


def oracle_solve_baseline(desc, k):
    """The oracle's own solver on a small workload: PCG (FP64) preconditioned
    by its V-cycle (Chebyshev degree 3, exact coarse solve), x0 = 0, relative
    residual 1e-10, f = 1; the hierarchy's assembly is excluded (as the GPU
    set-up is).  One thread."""
    from threadpoolctl import threadpool_limits

    from oracle import octree
    from oracle.hierarchy import Hierarchy
    from oracle.space import assemble_load, constant
    t0 = time.time()
    H = Hierarchy(octree.build_mesh(desc), k)
    b = assemble_load(H.spaces[-1], constant(1.0))
    setup = time.time() - t0
    with threadpool_limits(limits=1):
        t0 = time.time()
        x, its, hist = H.solve(b, rtol=1e-10)
        dt = time.time() - t0
    return {"seconds": dt, "iterations": its, "free_dofs": int(b.size), "setup_s": round(setup, 1), "cores": 1}


PROFILE_WORKLOADS = {
    # name: (mesh descriptor name in synth, degree, scheme, level dtype, vectors, what runs)
    "q4_f64_vmult": ("CFG2", 4, "h_then_p", "f64", 1, "vmult"),
    "q4_f32_vmult": ("CFG2", 4, "h_then_p", "f32", 1, "vmult"),
    "q6_f32x8_vmult": ("CFG4", 6, "p_then_h", "f32", 8, "vmult"),
    "q6_f32x1_vmult": ("CFG4", 6, "p_then_h", "f32", 1, "vmult"),
    "q6_f32x8_transfer": ("CFG4", 6, "p_then_h", "f32", 8, "transfer"),
    "q6_f32x8_smooth": ("CFG4", 6, "p_then_h", "f32", 8, "smooth"),
    "q4_f64_smooth": ("CFG2", 4, "h_then_p", "f64", 1, "smooth"),
    "q4_f64_vmult_uniform64": ("UNIFORM64", 4, "h", "f64", 1, "vmult"),
    "q4_f64_vmult_octant7": ("OCTANT7", 4, "h", "f64", 1, "vmult"),
    "q4_f64_vmult_shell8": ("SHELL8", 4, "h", "f64", 1, "vmult"),
}


def run_profile_workload(name, steps, warmup):
    """Set up one workload and run only its kernels `steps` times after
    `warmup` untimed runs: the finest-level operator (vmult), the transfer
    between the finest level and the next (prolongate_add + restrict_add), or
    one Chebyshev smoothing step of degree 3 on the finest level (smooth).
    Prints the mean HIP-event time per run (library stream)."""
    import numpy as np
    import torch

    import synth
    from paper_2203_12292_amd import mfmg
    mesh_name, k, scheme, dt, nv, what = PROFILE_WORKLOADS[name]
    schemes = {"h": mfmg.SCHEME_H, "h_then_p": mfmg.SCHEME_H_THEN_P, "p_then_h": mfmg.SCHEME_P_THEN_H}
    tdt = {"f64": torch.float64, "f32": torch.float32}[dt]
    code = {"f64": mfmg.F64, "f32": mfmg.F32}[dt]
    dev = torch.device("cuda:0")
    print(f"[profile] {name}: set-up", file=sys.stderr, flush=True)
    S = mfmg.Solver(mfmg.Mesh(getattr(synth, mesh_name)), k, schemes[scheme], level_dtypes=[code], max_rhs=nv)
    fine = S.n_levels - 1
    n = S.n_dofs(fine)
    nc = S.n_dofs(fine - 1)
    x = torch.from_numpy(synth.uniform_vector(n * nv, seed=12292)).to(dev).to(tdt)
    y = torch.zeros_like(x)
    xc = torch.from_numpy(synth.uniform_vector(nc * nv, seed=7)).to(dev).to(tdt)
    yc = torch.zeros_like(xc)
    if what == "vmult":
        def run():
            S.vmult(fine, y, x, n_vec=nv)
    elif what == "transfer":
        def run():
            S.prolongate_add(fine, y, xc, n_vec=nv)
            S.restrict_add(fine, yc, x, n_vec=nv)
    else:
        def run():
            S.smooth(fine, y, x, x_is_zero=False, n_vec=nv)
    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    ms = _events_time(run, steps, torch.cuda.current_stream())
    print(f"[profile] {name}: {n} DoFs x {nv} vectors, {float(np.mean(ms)):.4f} ms per run", file=sys.stderr,
          flush=True)


def hanging_node_overhead(k=4, reps=20):
    """The operator on the paper's two test meshes, whose leaves carry
    hanging-node constraints in very different shares (octant L = 7: 6 %,
    shell L = 8: 38 %; Section 4), against a uniform mesh of similar size
    without any: time per DoF and per application, FP64, and the extra time
    per DoF relative to the uniform mesh (the paper's bound for high degrees
    is 20 %, Section 3.2)."""
    import numpy as np
    import torch

    import synth
    from paper_2203_12292_amd import mfmg
    dev = torch.device("cuda:0")
    out = {}
    # the uniform mesh comes from one cell by six global steps, as the paper's
    # meshes do, so that its hierarchy has a small coarse grid
    for name, desc in (("uniform64", synth.UNIFORM64), ("octant7", synth.OCTANT7), ("shell8", synth.SHELL8)):
        print(f"[bench] hanging-node overhead: {name}", file=sys.stderr, flush=True)
        mesh = mfmg.Mesh(desc)
        cells, nh = mesh.info()
        S = mfmg.Solver(mesh, k, mfmg.SCHEME_H, max_rhs=1)
        fine = S.n_levels - 1
        n = S.n_dofs(fine)
        x = torch.from_numpy(synth.uniform_vector(n, seed=12292)).to(dev)
        y = torch.empty_like(x)
        for _ in range(3):
            S.vmult(fine, y, x)
        ms = float(np.mean(_events_time(lambda: S.vmult(fine, y, x), reps, torch.cuda.current_stream())))
        out[name] = {"cells": cells[-1], "hanging_cells": nh, "hanging_share": nh / cells[-1], "free_dofs": n,
                     "ms": ms, "ns_per_dof": ms * 1e6 / n, "dofs_per_s": n / (ms * 1e-3),
                     "hbm_frac": 16.0 * n / (ms * 1e-3) / (HBM_PEAK_GBS * 1e9)}
        del S, x, y
        torch.cuda.empty_cache()
    base = out["uniform64"]["ns_per_dof"]
    for name in ("octant7", "shell8"):
        out[name]["overhead_vs_uniform"] = out[name]["ns_per_dof"] / base - 1.0
    return out


def ls_sweep():
    """Iterations of global coarsening against local smoothing on the paper's
    octant and shell meshes (L = 6, Q4) and the config-1 mesh (Q2) under
    several Chebyshev settings (degree, smoothing range, Lanczos steps and
    safety factor of the eigenvalue estimate); one JSON line per solve."""
    import torch

    import synth
    from paper_2203_12292_amd import mfmg
    dev = torch.device("cuda:0")
    settings = ((3, 20.0, 15, 1.2), (3, 20.0, 60, 1.2), (3, 20.0, 15, 1.5), (3, 10.0, 15, 1.2),
                (3, 30.0, 15, 1.2), (5, 20.0, 15, 1.2), (6, 20.0, 15, 1.2))
    for mname, desc, k in (("octant6", synth.octant_mesh(6), 4), ("shell6", synth.shell_mesh(6), 4),
                           ("cube4_g1_ball2", synth.CFG1, 2)):
        mesh = mfmg.Mesh(desc)
        for sch_name, sch in (("gc", mfmg.SCHEME_H), ("ls", mfmg.SCHEME_LS)):
            for deg, rng, eit, saf in settings:
                S = mfmg.Solver(mesh, k, sch, cheb_degree=deg, smoothing_range=rng, eig_iterations=eit,
                                eig_safety=saf)
                b = torch.zeros(S.n_dofs(), dtype=torch.float64, device=dev)
                S.rhs(b)
                x = torch.zeros_like(b)
                st = S.solve(x, b, rtol=1e-10, max_it=100)
                print(json.dumps({"mesh": mname, "degree": k, "scheme": sch_name, "cheb_degree": deg,
                                  "smoothing_range": rng, "eig_iterations": eit, "eig_safety": saf,
                                  "iterations": st["iterations"],
                                  "lambda_max": [S.smoother_range(l)[1] for l in range(1, S.n_levels)]}),
                      flush=True)
                del S


def kernel_summary(trace_dir, pmc_dirs, title, commands, top=10, last=0):
    """Markdown summary of a rocprofv3 run of one --profile workload: the
    kernels by total time (dispatch count, median and mean duration) from
    the kernel trace, and the mean of each counter per kernel from the --pmc
    runs.  With last > 0 only the last `last` dispatches of each kernel name
    count (the timed loop of the workload, after its set-up); otherwise the
    largest grid of each name."""
    import numpy as np
    rows = []
    for path in glob.glob(os.path.join(trace_dir, "**", "*kernel_trace.csv"), recursive=True):
        with open(path, newline="") as fh:
            for r in csv.DictReader(fh):
                grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
                rows.append((int(r["Start_Timestamp"]), _kname(r["Kernel_Name"]), grid,
                             (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3))
    rows.sort()
    if last > 0:
        keep = {}
        for row in rows:
            keep.setdefault(row[1], []).append(row)
        rows = sorted(r for v in keep.values() for r in v[-last:])
    by = {}
    for _, name, grid, us in rows:
        by.setdefault((name, grid), []).append(us)
    lines = [f"# {title}", "", "Commands:", ""] + [f"    {c}" for c in commands] + [""]
    lines += ["| kernel | grid (threads) | dispatches | median us | mean us | total ms |", "|---|---|---|---|---|---|"]
    top_names = []
    for (name, grid), v in sorted(by.items(), key=lambda kv: -sum(kv[1]))[:top]:
        lines.append(f"| `{name}` | {grid} | {len(v)} | {np.median(v):.1f} | {np.mean(v):.1f} | {sum(v) / 1e3:.2f} |")
        top_names.append(name)
    for d in pmc_dirs:
        recs = []
        for path in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
            with open(path, newline="") as fh:
                for r in csv.DictReader(fh):
                    recs.append((int(r["Dispatch_Id"]), _kname(r["Kernel_Name"]), int(r["Grid_Size"]),
                                 r["Counter_Name"], float(r["Counter_Value"])))
        recs.sort()
        best = {}
        if last > 0:
            ids = {}
            for did, name, grid, _, _ in recs:
                lst = ids.setdefault(name, [])
                if not lst or lst[-1] != did:
                    lst.append(did)
            chosen = {name: set(v[-last:]) for name, v in ids.items()}
            for did, name, grid, cn, cv in recs:
                if did in chosen[name]:
                    best.setdefault(name, (grid, {}))[1].setdefault(cn, []).append(cv)
        else:
            vals = {}
            for _, name, grid, cn, cv in recs:
                vals.setdefault((name, grid), {}).setdefault(cn, []).append(cv)
            for (name, grid), cs in vals.items():
                if name not in best or grid > best[name][0]:
                    best[name] = (grid, cs)
        if not best:
            continue
        counters = sorted({c for _, cs in best.values() for c in cs})
        which = f"last {last} dispatches of each kernel" if last > 0 else "largest grid of each kernel"
        lines += ["", f"Counters ({os.path.basename(d.rstrip('/'))}; mean per dispatch, {which}):", ""]
        lines += ["| kernel | grid | " + " | ".join(counters) + " |", "|---|---|" + "---|" * len(counters)]
        order = [n for n in dict.fromkeys(top_names) if n in best] or sorted(best, key=lambda n: -best[n][0])[:top]
        for name in order:
            grid, cs = best[name]
            lines.append(f"| `{name}` | {grid} | " +
                         " | ".join(f"{np.mean(cs[c]):.4g}" if c in cs else "" for c in counters) + " |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--skip-cpu-baseline", action="store_true")
    ap.add_argument("--skip-solves", action="store_true")
    ap.add_argument("--pmc-summary", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="print the HBM traffic summary of two rocprofv3 --pmc runs and exit (no GPU)")
    ap.add_argument("--pmc-n", type=int, default=0, help="free DoFs of the profiled run (for --pmc-summary)")
    ap.add_argument("--pmc-command", action="append", default=[], help="command lines to quote in the summary")
    ap.add_argument("--trace-summary", nargs=2, metavar=("KERNEL_TRACE_CSV", "BENCH_JSON"),
                    help="print the kernel-trace summary of a profiled run and exit (no GPU)")
    ap.add_argument("--ls-sweep", action="store_true",
                    help="GC against LS iterations under several smoother settings (GPU), then exit")
    ap.add_argument("--kernel-summary", nargs="+", metavar="DIR",
                    help="print a markdown summary of a kernel-trace folder and --pmc folders and exit (no GPU)")
    ap.add_argument("--summary-title", default="rocprofv3 summary")
    ap.add_argument("--summary-last", type=int, default=0,
                    help="count only the last N dispatches of each kernel (the timed loop)")
    ap.add_argument("--profile", choices=sorted(PROFILE_WORKLOADS),
                    help="run only the kernels of one workload --steps times (for rocprofv3) and exit")
    args = ap.parse_args()
    if args.ls_sweep:
        ls_sweep()
        return
    if args.kernel_summary:
        print(kernel_summary(args.kernel_summary[0], args.kernel_summary[1:], args.summary_title, args.pmc_command,
                             last=args.summary_last))
        return
    if args.profile:
        run_profile_workload(args.profile, args.steps, args.warmup)
        return
    if args.trace_summary:
        print(trace_summary(args.trace_summary[0], args.trace_summary[1], args.pmc_command))
        return
    if args.pmc_summary:
        print(pmc_summary(args.pmc_summary[0], args.pmc_summary[1], args.pmc_n, args.pmc_command))
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU sharding of the "
              "operator is not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2203_12292_amd import mfmg

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    desc = synth.CFG2
    k = 4
    t0 = time.time()
    mesh = mfmg.Mesh(desc)
    cells, n_hang = mesh.info()
    solver = mfmg.Solver(mesh, k, mfmg.SCHEME_H_THEN_P)
    setup_s = time.time() - t0
    fine = solver.n_levels - 1
    info = solver.level_info(fine)
    n = info["n_dofs"]
    x = torch.from_numpy(synth.uniform_vector(n, seed=12292)).to(dev)
    y = torch.empty_like(x)

    def op():
        solver.vmult(fine, y, x)

    for _ in range(args.warmup):
        op()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    ms = _events_time(op, args.steps, stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    avg_ms = float(np.mean(ms))
    value = n * args.steps / wall
    alg_bytes = 16.0 * n  # read src + write dst, FP64 (metadata reported separately)
    achieved = alg_bytes / (avg_ms * 1e-3) / 1e9
    # a plain elementwise kernel over the same vector (calibration of the HBM byte counters)
    for _ in range(3):
        torch.mul(x, 1.0, out=y)
    torch.cuda.synchronize()

    out = {
        "metric": "matrix-free vmult DoFs/s & %HBM peak; time-to-solve 1e-10, plain FP64 vs mixed/learned",
        "value": value,
        "unit": "DoFs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "poisson_cube16_ball4_q4", "cells": cells[-1], "free_dofs": n, "degree": k,
                   "quadrature": "gauss 5^3", "hanging_cells": n_hang, "levels": solver.n_levels,
                   "setup_s": round(setup_s, 2)},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": recorded_traffic(),
                     "kernel": "clear_shared_kernel + vmult_batch_kernel (one operator application)",
                     "alg_bytes_per_launch": alg_bytes, "avg_launch_ms": avg_ms},
    }

    print(f"[bench] operator: {avg_ms:.3f} ms per application, {value:.3e} DoFs/s", file=sys.stderr, flush=True)
    if not args.skip_solves:
        solves = _Progress()
        b = torch.zeros(n, dtype=torch.float64, device=dev)
        solver.rhs(b)
        xs = torch.zeros_like(b)
        st = solver.solve(xs, b, rtol=1e-10, max_it=100)
        st = solver.solve(xs, b, rtol=1e-10, max_it=100)
        solves["cube16_q4_fp64"] = {"seconds": st["time_ms"] * 1e-3, "iterations": st["iterations"],
                                    "residual": st["final_residual"]}
        # PCG started from one full-multigrid pass
        sf = mfmg.Solver(mesh, k, mfmg.SCHEME_H_THEN_P, fmg_start=True)
        xf = torch.zeros_like(b)
        for _ in range(2):
            st = sf.solve(xf, b, rtol=1e-10, max_it=100)
        solves["cube16_q4_fp64_fmg_start"] = {"seconds": st["time_ms"] * 1e-3, "iterations": st["iterations"],
                                              "residual": st["final_residual"], "start_residual": st["history"][0]}
        del sf, xf
        # full multigrid: one pass, one or two V-cycles per level; its distance to
        # the converged PCG solution (1e-10) is the algebraic error it leaves
        r = torch.empty_like(b)
        x_ref = xs.clone()
        for cycles in (1, 2):
            for _ in range(2):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                solver.fmg(xs, b, cycles=cycles)
                e1.record()
                torch.cuda.synchronize()
            solver.vmult(fine, r, xs)
            res = float(torch.linalg.norm(b - r) / torch.linalg.norm(b))
            err = float(torch.linalg.norm(xs - x_ref) / torch.linalg.norm(x_ref))
            solves[f"cube16_q4_fmg_{cycles}_vcycles"] = {"seconds": e0.elapsed_time(e1) * 1e-3,
                                                       "relative_residual": res,
                                                       "relative_distance_to_solution": err}
        del solver
        torch.cuda.empty_cache()
        s32 = mfmg.Solver(mesh, k, mfmg.SCHEME_H_THEN_P, level_dtypes=[mfmg.F32])
        st = s32.solve(xs, b, rtol=1e-10, max_it=100, flexible=True)
        st = s32.solve(xs, b, rtol=1e-10, max_it=100, flexible=True)
        solves["cube16_q4_fp32_vcycle"] = {"seconds": st["time_ms"] * 1e-3, "iterations": st["iterations"],
                                           "residual": st["final_residual"]}
        del s32
        # geometric local smoothing (Section 2.1, the paper's comparison method) on
        # the same problem: refinement-level levels down to the 16^3 coarse grid,
        # then polynomial levels there as in the global-coarsening runs
        for name, dts in (("cube16_q4_ls_fp64", []), ("cube16_q4_ls_fp32_vcycle", [mfmg.F32])):
            torch.cuda.empty_cache()
            t0 = time.time()
            sls = mfmg.Solver(mesh, k, mfmg.SCHEME_LS_THEN_P, level_dtypes=dts)
            setup_ls = time.time() - t0
            for _ in range(2):
                st = sls.solve(xs, b, rtol=1e-10, max_it=100, flexible=bool(dts))
            solves[name] = {"seconds": st["time_ms"] * 1e-3, "iterations": st["iterations"],
                            "residual": st["final_residual"], "levels": sls.n_levels, "setup_s": round(setup_ls, 2)}
            del sls
        # geometric and polynomial coarsening in one step (Q4 -> Q2 -> Q1 with the mesh)
        torch.cuda.empty_cache()
        t0 = time.time()
        shp = mfmg.Solver(mesh, k, mfmg.SCHEME_HP)
        setup_hp = time.time() - t0
        for _ in range(2):
            st = shp.solve(xs, b, rtol=1e-10, max_it=100)
        solves["cube16_q4_hp_fp64"] = {"seconds": st["time_ms"] * 1e-3, "iterations": st["iterations"],
                                       "residual": st["final_residual"], "levels": shp.n_levels,
                                       "setup_s": round(setup_hp, 2)}
        del shp
        # -div(c grad u), c constant per cell (coarser levels average it over the
        # leaves): a 1:1000 checkerboard of 0.25-cubes (aligned with every
        # level's cells), and a c = 1000 ball inclusion of radius 0.3 about the
        # centre, whose boundary no level resolves exactly
        for name, co, cap in (("cube16_q4_checker1000_fp64", synth.COEF_CHECKER_1000, 200),
                              ("cube16_q4_inclusion1000_fp64", synth.COEF_INCLUSION, 200)):
            torch.cuda.empty_cache()
            t0 = time.time()
            sco = mfmg.Solver(mesh, k, mfmg.SCHEME_H_THEN_P, coef=co)
            setup_co = time.time() - t0
            st = sco.solve(xs, b, rtol=1e-10, max_it=cap, raise_on_fail=False)
            solves[name] = {"seconds": st["time_ms"] * 1e-3, "iterations": st["iterations"],
                            "converged": st["converged"], "residual": st["final_residual"],
                            "setup_s": round(setup_co, 2)}
            del sco
        m1 = mfmg.Mesh(synth.CFG1)
        for drop in (1, 2):  # early switch to the coarse solver, on a level with hanging nodes
            s1 = mfmg.Solver(m1, 2, mfmg.SCHEME_H, drop_coarse=drop)
            b1 = torch.zeros(s1.n_dofs(), dtype=torch.float64, device=dev)
            s1.rhs(b1)
            x1 = torch.zeros_like(b1)
            for _ in range(3):
                st = s1.solve(x1, b1, rtol=1e-10, max_it=100)
            solves[f"cube4_q2_fp64_coarse_switch_{drop}"] = {
                "seconds": st["time_ms"] * 1e-3, "iterations": st["iterations"], "residual": st["final_residual"],
                "levels": s1.n_levels, "coarse_dofs": s1.n_dofs(0)}
            del s1
        for name, dts, graph in (("cube4_q2_fp64", [], False),
                                 ("cube4_q2_mixed_bf16", [mfmg.BF16, mfmg.BF16, mfmg.F32], False),
                                 ("cube4_q2_fp64_graph", [], True),
                                 ("cube4_q2_mixed_bf16_graph", [mfmg.BF16, mfmg.BF16, mfmg.F32], True)):
            # (graph: the V-cycles of the solve replayed from a HIP graph)
            s1 = mfmg.Solver(m1, 2, mfmg.SCHEME_H, level_dtypes=dts, graph_vcycle=graph)
            b1 = torch.zeros(s1.n_dofs(), dtype=torch.float64, device=dev)
            s1.rhs(b1)
            x1 = torch.zeros_like(b1)
            for _ in range(3):
                st = s1.solve(x1, b1, rtol=1e-10, max_it=100, flexible=bool(dts))
            solves[name] = {"seconds": st["time_ms"] * 1e-3, "iterations": st["iterations"],
                            "residual": st["final_residual"]}
        # the paper's octant mesh shape (Section 4, L = 6: 34,903 cells, Q4):
        # global coarsening against local smoothing
        mo = mfmg.Mesh(synth.octant_mesh(6))
        for name, sch in (("octant6_q4_gc_fp64", mfmg.SCHEME_H), ("octant6_q4_ls_fp64", mfmg.SCHEME_LS)):
            so = mfmg.Solver(mo, 4, sch)
            bo = torch.zeros(so.n_dofs(), dtype=torch.float64, device=dev)
            so.rhs(bo)
            xo = torch.zeros_like(bo)
            for _ in range(2):
                st = so.solve(xo, bo, rtol=1e-10, max_it=100)
            solves[name] = {"seconds": st["time_ms"] * 1e-3, "iterations": st["iterations"],
                            "residual": st["final_residual"], "free_dofs": so.n_dofs(), "levels": so.n_levels}
            del so
        s1 = mfmg.Solver(m1, 2, mfmg.SCHEME_LS)
        b1 = torch.zeros(s1.n_dofs(), dtype=torch.float64, device=dev)
        s1.rhs(b1)
        x1 = torch.zeros_like(b1)
        for _ in range(3):
            st = s1.solve(x1, b1, rtol=1e-10, max_it=100)
        solves["cube4_q2_ls_fp64"] = {"seconds": st["time_ms"] * 1e-3, "iterations": st["iterations"],
                                      "residual": st["final_residual"]}
        del s1
        # learned coarse correction on a mesh whose coarse level matters:
        # 6^3 coarse cubes (Q2 coarse problem of 1,331 DoFs, the network's
        # size limit is 2,048), two uniform steps and one ball step
        m5 = mfmg.Mesh(synth.CFG5_GAIN)
        s1 = mfmg.Solver(m5, 2, mfmg.SCHEME_H)
        b1 = torch.zeros(s1.n_dofs(), dtype=torch.float64, device=dev)
        x1 = torch.zeros_like(b1)
        t0 = time.time()
        s1.net_record(20000)
        j = 0
        while s1.net_n_recorded() < 20000:
            g = synth.gaussian_rhs_training(j)
            s1.rhs(b1, mfmg.RHS_GAUSS, g, n_terms=g.shape[0])
            s1.solve(x1, b1, rtol=1e-10, max_it=60)
            j += 1
        t_rec = time.time() - t0
        t0 = time.time()
        hist = s1.net_train(epochs=30, batch_rows=8192, lr=2e-3, init_seed=7, shuffle_seed=11)
        t_train = time.time() - t0
        s1.net_record(0)
        g = synth.gaussian_rhs_training(100000)
        s1.rhs(b1, mfmg.RHS_GAUSS, g, n_terms=g.shape[0])
        learned = {"mesh": "cube6_g2_ball1", "free_dofs": s1.n_dofs(), "coarse_dofs": s1.n_dofs(0),
                   "pairs": 20000, "record_s": round(t_rec, 2), "train_s": round(t_train, 2),
                   "train_loss_first_last": [hist[0], hist[-1]], "tau": 0.9}
        # network_alone: every prediction accepted (no exact fallback)
        for name, mode, tau in (("exact", mfmg.COARSE_EXACT, 0.9), ("learned", mfmg.COARSE_LEARNED, 0.9),
                                ("none", mfmg.COARSE_ZERO, 0.9), ("network_alone", mfmg.COARSE_LEARNED, 1e300)):
            s1.net_mode(mode, tau)
            for _ in range(3):
                if mode != mfmg.COARSE_EXACT:
                    s1.net_counts()
                st = s1.solve(x1, b1, rtol=1e-10, max_it=200, flexible=True)
            rec = {"seconds": st["time_ms"] * 1e-3, "iterations": st["iterations"], "residual": st["final_residual"]}
            if mode == mfmg.COARSE_LEARNED:
                a, r, rel = s1.net_counts()
                rec.update({"accepted": a, "rejected": r, "mean_rel_coarse_residual": rel})
            learned[name] = rec
        solves["cube6_q2_learned_coarse"] = learned
        del s1
        # p-multigrid Q6 -> Q3 -> Q1 + global coarsening, 8 right-hand sides
        m4 = mfmg.Mesh(synth.CFG4)
        t0 = time.time()
        s4 = mfmg.Solver(m4, 6, mfmg.SCHEME_P_THEN_H, level_dtypes=[mfmg.F32], max_rhs=8)
        setup4 = time.time() - t0
        n4 = s4.n_dofs()
        params = np.stack(synth.gaussian_rhs_batch(8))
        b4 = torch.zeros(n4 * 8, dtype=torch.float64, device=dev)
        s4.rhs(b4, mfmg.RHS_GAUSS, params, n_terms=4, n_vec=8)
        x4 = torch.zeros_like(b4)
        st = s4.solve(x4, b4, rtol=1e-10, max_it=100, flexible=True, n_vec=8)
        # the FP32 operator of the finest Q6 level on all 8 vectors at once
        f4 = s4.n_levels - 1
        x32 = torch.from_numpy(synth.uniform_vector(n4 * 8, seed=12292)).to(dev).float()
        y32 = torch.empty_like(x32)
        for _ in range(3):
            s4.vmult(f4, y32, x32, n_vec=8)
        ms4 = float(np.mean(_events_time(lambda: s4.vmult(f4, y32, x32, n_vec=8), 10, stream)))
        alg4 = 8.0 * 8 * n4
        out["roofline_q6_fp32_8vec"] = {
            "bound": "hbm", "achieved": alg4 / (ms4 * 1e-3) / 1e9, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": alg4 / (ms4 * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
            "kernel": "vmult_batch_kernel<6, float> + reduce_shared_vec_kernel, 8 interleaved vectors",
            "alg_bytes_per_launch": alg4, "avg_launch_ms": ms4, "dofs_per_s": 8 * n4 / (ms4 * 1e-3)}
        del x32, y32
        solves["cube12_spheres_q6_pmg_8rhs_fp32_vcycle"] = {
            "seconds": st["time_ms"] * 1e-3, "iterations": st["iterations"], "residual": st["final_residual"],
            "free_dofs": n4, "n_rhs": 8, "levels": s4.n_levels, "setup_s": round(setup4, 2)}
        del s4
        torch.cuda.empty_cache()
        t0 = time.time()
        s4 = mfmg.Solver(m4, 6, mfmg.SCHEME_HP, level_dtypes=[mfmg.F32], max_rhs=8)
        setup4 = time.time() - t0
        x4.zero_()
        st = s4.solve(x4, b4, rtol=1e-10, max_it=100, flexible=True, n_vec=8)
        solves["cube12_spheres_q6_hp_8rhs_fp32_vcycle"] = {
            "seconds": st["time_ms"] * 1e-3, "iterations": st["iterations"], "residual": st["final_residual"],
            "free_dofs": n4, "n_rhs": 8, "levels": s4.n_levels, "setup_s": round(setup4, 2)}
        del s4
        out["time_to_solve"] = dict(solves)
        out["hanging_node_overhead_q4"] = hanging_node_overhead()

    if not args.skip_cpu_baseline:
        print("[bench] CPU baseline: the oracle on the host cores", file=sys.stderr, flush=True)
        cb = cpu_baseline(desc, k)
        dofs_per_cell = n / cells[-1]
        out["cpu_baseline"] = {
            "value": cb["cells_per_s_all"] * dofs_per_cell, "unit": "DoFs/s", "cores": cb["cores"],
            "kind": "oracle",
            "sample": f"element-by-element C_e^T A_e C_e apply (numpy FP64) over {cb['n_sample']} random cells of "
                      f"the {cb['n_cells_total']}-cell mesh, {cb['seconds']:.0f} s per run, one process per core; "
                      f"DoFs/s = cells/s x {dofs_per_cell:.1f} free DoFs per cell",
            "value_1core": cb["cells_per_s_1core"] * dofs_per_cell,
            "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "oracle_solve_cube4_q2": oracle_solve_baseline(synth.CFG1, 2)}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
