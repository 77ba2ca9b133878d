#!/usr/bin/env python3
"""Benchmark: batched phase-diagram scan of the 3x3 toric code in two fields
(complex64) against the plain per-point complex128 run, on one MI355X.

One benchmark step = one pass of the whole hot path over the batch: every
state of the 32 x 32 (hx, hz) grid is initialized (Eq. (ini1)), ramped from
the toric code through M = 1000 second-order Trotter steps (T = 20) and
observed (energy, Wilson and 't Hooft loops, fields, weight histogram), all
inside one HIP-graph launch.

Printed: one JSON line with amplitude-updates/s (sum over states of 2^n per
Trotter step), the roofline of the dominant pass kernel from HIP events
around every pass kernel of the timed runs (direct launches on the kernels'
stream; a HIP-graph replay is timed beside them), the plain complex128
per-point throughput on the same GPU, and the FP64 oracle timed on the host
cores.

Also measured (legs of their own, outside the timed region): a device copy
and an in-place elementwise kernel of 2 GiB (reference points; the copy also
scales the rocprofv3 traffic counters), the same scan as one complex128
batch, the 4x4 torus (32 link qubits, 32 GiB complex64 and 64 GiB complex128
states) ramped to (0.25, 0.25) in 200 steps with the event-timed GB/s of
every pass kind, the adjoint, the mixed batch, the exact solvers, the
gate-level circuit and the paper's protocol paths.

Usage: python bench.py [--steps K] [--warmup W] [--gpus 1]
       python bench.py --pmc-summary FETCH_CSV WRITE_CSV   (host only: turns two
           rocprofv3 --pmc counter files of this benchmark into the traffic
           record read by later runs)
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0     # MI355X HBM3E, GB/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_scan_3x3_c64.json")
# schedules chosen by the autotuner on an MI355X (lines: n c128 batch-class schedule)
SHIPPED_TABLE = os.path.join(ROOT, "paper_2108_13410_amd", "tuned_mi355x.txt")
# sources the scan's pass kernels are compiled from (the traffic record is
# keyed by their hash)
EXACT_4X4_SPLIT = "split=12:4:12:0/10:4:13:3:h7@22/10:4:13:3,xcd=7"
KERNEL_SRCS = [os.path.join(ROOT, "paper_2108_13410_amd", "csrc", f)
               for f in ("z2h_kernels.hip", "z2h_tile.h", "z2h_kernels.h", "z2h_internal.h")]


def kernel_hash():
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def ensure_built():
    from paper_2108_13410_amd import z2h
    if not os.path.exists(z2h.LIB_PATH):
        from paper_2108_13410_amd import build as b
        b.build()


def make_batch(jobs, dtype, z2h):
    scheds, Lx, Ly, H = [], [], [], []
    for j in jobs:
        scheds.append(z2h.schedule(j["c0"], j["c1"], j["M"], j["T"] / j["M"],
                                   renorm=1 if dtype == z2h.Z2H_C64 else 0))
        Lx.append(j["Lx"])
        Ly.append(j["Ly"])
        H.append(j["c1"])
    return z2h.z2h_batch_create(Lx, Ly, scheds, [z2h.Z2H_INIT_PSI1] * len(jobs), H, dtype)


def plain_c128(jobs, z2h, torch, npoints):
    """Per-point complex128 runs (the plain method) on a sample of the grid."""
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C128)
    sz = z2h.z2h_plan_sizes(plan)
    psi = z2h.alloc_state(plan)
    ws = z2h.alloc_bytes(max(sz["ws_evolve"], sz["ws_observe"]))
    out = torch.zeros(z2h.Z2H_OBS_DOUBLES, dtype=torch.float64, device="cuda")
    zl, xl = z2h.z2h_loop_masks(3, 3)
    step = max(1, len(jobs) // npoints)
    picks = list(range(0, len(jobs), step))[:npoints]

    def run(j):
        job = jobs[j]
        z2h.z2h_state_init(plan, psi, z2h.Z2H_INIT_PSI1)
        z2h.z2h_evolve(plan, psi, ws, z2h.schedule(job["c0"], job["c1"], job["M"], job["T"] / job["M"]))
        z2h.z2h_observe(plan, psi, ws, job["c1"], zl, xl, d_out=out, host=False)

    run(picks[0])
    torch.cuda.synchronize()
    res = {}
    t0 = time.perf_counter()
    for j in picks:
        run(j)
        torch.cuda.synchronize()
        res[j] = out.cpu().numpy().copy()
    dt = time.perf_counter() - t0
    return dt / len(picks), res


def copy_ceiling(torch, nbytes=1 << 31, reps=5):
    """Achievable HBM rate on this device: torch's device-to-device copy of
    nbytes (nbytes read + nbytes written) and an in-place elementwise kernel
    over the same buffer, timed with events on the current stream."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    a.neg_()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    ev[0].record()
    for _ in range(reps):
        b.copy_(a)
    ev[1].record()
    ev[2].record()
    for _ in range(reps):
        a.neg_()
    ev[3].record()
    torch.cuda.synchronize()
    copy_ms = ev[0].elapsed_time(ev[1]) / reps
    inpl_ms = ev[2].elapsed_time(ev[3]) / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_each_way": nbytes,
            "copy_GBps": 2 * nbytes / (copy_ms * 1e-3) / 1e9,
            "inplace_GBps": 2 * nbytes / (inpl_ms * 1e-3) / 1e9}


def cache_has(path, n, c128):
    """Whether a schedule cache written by the autotuner has an entry for n
    qubits in this precision (lines: n c128 batch-class schedule)."""
    if not path or not os.path.exists(path):
        return False
    with open(path) as f:
        for ln in f:
            p = ln.split()
            if len(p) >= 4 and p[0] == str(n) and p[1] == ("1" if c128 else "0"):
                return True
    return False


def four_by_four(z2h, torch, tune=True, tune_cache=None, steps=None, schedules=None, precisions=("c64", "c128")):
    """The 4x4 torus (32 link qubits): ramp from the toric code to
    (0.25, 0.25), T = 20, M = 200, in complex64 (renormalised every step)
    and complex128; event-timed GB/s per pass kind, energies, norm drift.
    steps (profiling runs): fewer steps at the same dt; schedules: explicit
    schedule string per precision instead of the tuned table's."""
    from paper_2108_13410_amd import workloads
    job = workloads.point_4x4()
    if steps:
        job = dict(job, M=int(steps), T=job["T"] * int(steps) / job["M"])
    M, n = job["M"], 32
    zl, xl = z2h.z2h_loop_masks(4, 4)
    res = {}
    schedules = schedules or {}
    for name, dtype in (("c64", z2h.Z2H_C64), ("c128", z2h.Z2H_C128)):
        if name not in precisions:
            continue
        b = 8 if dtype == z2h.Z2H_C64 else 16
        tuned = None
        if schedules.get(name):
            pass
        elif tune:
            if cache_has(tune_cache, 32, dtype == z2h.Z2H_C128):
                z2h.z2h_tune_load(tune_cache)
            else:
                tuned = z2h.z2h_autotune(4, 4, dtype, 1, None if tune_cache == SHIPPED_TABLE else tune_cache)
                print(f"4x4 {name} autotuned: {tuned}", file=sys.stderr, flush=True)
        if schedules.get(name):
            plan = z2h.z2h_plan_create_config(4, 4, dtype, schedules[name])
        else:
            plan = z2h.z2h_plan_create(4, 4, dtype)
        sz = z2h.z2h_plan_sizes(plan)
        info = z2h.z2h_plan_info(plan)
        psi = z2h.alloc_state(plan)
        ws = z2h.alloc_bytes(max(sz["ws_evolve"], sz["ws_observe"]))
        norms = torch.zeros(M, dtype=torch.float64, device="cuda")
        sched = z2h.schedule(job["c0"], job["c1"], M, job["T"] / M,
                             renorm=1 if dtype == z2h.Z2H_C64 else 0)
        z2h.z2h_state_init(plan, psi, z2h.Z2H_INIT_PSI1)
        torch.cuda.synchronize()
        z2h.z2h_timing_read()
        z2h.z2h_timing_enable(True)
        t0 = time.perf_counter()
        z2h.z2h_evolve(plan, psi, ws, sched, norms=norms)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        counts, ms = z2h.z2h_timing_read()
        z2h.z2h_timing_enable(False)
        ob = z2h.z2h_observe(plan, psi, ws, job["c1"], zl, xl)
        nrm = norms.cpu().numpy()
        per_pass = 2 * (1 << n) * b
        kinds = {}
        for k, kname in enumerate(("z", "x", "plain")):
            if counts[k]:
                avg = ms[k] / counts[k]
                kinds[kname] = {"launches": int(counts[k]), "avg_ms": avg,
                                "GBps": per_pass / (avg * 1e-3) / 1e9}
        res[name] = {
            "schedule": z2h.z2h_plan_describe(plan), "passes_per_step": info["passes_per_step"],
            "autotuned": None if tuned is None else {"config": tuned[0], "ms_per_trotter_step": tuned[1]},
            "seconds": el, "amp_updates_per_s": (1 << n) * M / el,
            "bytes_per_pass": per_pass, "pass": kinds,
            "energy": ob["energy"], "norm": ob["norm"], "mx": ob["mx"], "mz": ob["mz"],
            "wilson_1x3": ob["zloop"][0],
            "max_step_norm_drift": float(abs(nrm - 1).max()),
        }
        del psi, ws, norms
        z2h.z2h_plan_destroy(plan)
        torch.cuda.empty_cache()
        print(f"4x4 {name}: {el:.2f} s", file=sys.stderr, flush=True)
    if "c64" not in res or "c128" not in res:
        return res
    res["c64_vs_c128"] = {"energy_per_link": abs(res["c64"]["energy"] - res["c128"]["energy"]) / n,
                          "mx": abs(res["c64"]["mx"] - res["c128"]["mx"]),
                          "mz": abs(res["c64"]["mz"] - res["c128"]["mz"])}
    return res


def pass_kernel_names(z2h, schedule):
    """Template instance of the z pass (group 0) and the x pass (top group)
    kernels of the 3x3 complex64 scan schedule."""
    if not schedule:
        return {}
    plan = z2h.z2h_plan_create_config(3, 3, z2h.Z2H_C64, schedule)
    d = z2h.z2h_plan_describe(plan)
    z2h.z2h_plan_destroy(plan)
    g = d["groups"]

    def name(gr):
        return f"level_kernel_full<float, {gr['R']}, {gr['full']}, 2, {gr['pair']}>"
    return {"z": name(g[0]), "x": name(g[-1])}


def pmc_summary(fetch_csv, write_csv):
    """Reduce two rocprofv3 --pmc runs of this benchmark (FETCH_SIZE, then
    WRITE_SIZE; KiB per dispatch) to bytes per scan pass launch.  Each counter
    is scaled by what it reads for the calibration copy of known size (the
    largest device-to-device copy dispatch: bytes_each_way read and written)."""
    import csv
    import numpy as np

    def load(path, counter):
        rows = [r for r in csv.DictReader(open(path)) if r["Counter_Name"] == counter]
        per = {}
        for r in rows:
            per.setdefault((r["Kernel_Name"], int(r["Grid_Size"])), []).append(float(r["Counter_Value"]))
        return per

    out = {"kernel_source_sha256_16": kernel_hash()}
    scale = {}
    for key, path, counter in (("fetch", fetch_csv, "FETCH_SIZE"), ("write", write_csv, "WRITE_SIZE")):
        per = load(path, counter)
        copies = {k: v for k, v in per.items() if "copyBuffer" in k[0]}
        ck = max(copies, key=lambda k: k[1])
        copy_kib = float(np.median(copies[ck]))
        expect = 1 << 31
        scale[key] = expect / (copy_kib * 1024.0)
        passes = {k: v for k, v in per.items() if "level_kernel" in k[0] and k[1] >= (1 << 23)}
        vals = [x for v in passes.values() for x in v]
        if not vals:
            raise SystemExit(f"{path}: no scan pass dispatches (level_kernel, grid >= 2^23) found")
        out[key] = {"copy_kernel": ck[0], "copy_grid": ck[1], "copy_kib_per_dispatch": copy_kib,
                    "copy_bytes_expected": expect, "scale": scale[key],
                    "pass_dispatches": len(vals), "pass_kib_per_dispatch": float(np.mean(vals)),
                    "per_kernel": {f"{k[0][:80]} grid={k[1]}": float(np.mean(v)) for k, v in passes.items()}}
    fb = out["fetch"]["pass_kib_per_dispatch"] * 1024 * scale["fetch"]
    wb = out["write"]["pass_kib_per_dispatch"] * 1024 * scale["write"]
    # per pass kernel (template instance and grid): scaled fetch + write bytes
    out["per_kernel_bytes"] = {}
    for k, v in out["fetch"]["per_kernel"].items():
        if k in out["write"]["per_kernel"]:
            out["per_kernel_bytes"][k] = v * 1024 * scale["fetch"] + out["write"]["per_kernel"][k] * 1024 * scale["write"]
    out["bytes_per_launch"] = fb + wb
    out["fetch_bytes_per_launch"] = fb
    out["write_bytes_per_launch"] = wb
    out["algorithmic_bytes_per_launch"] = 2 * 1024 * (1 << 18) * 8
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps({k: out[k] for k in ("bytes_per_launch", "fetch_bytes_per_launch",
                                          "write_bytes_per_launch", "algorithmic_bytes_per_launch")}))


def paper_protocol(z2h, torch):
    """The paper's protocol on the 3x3 torus (complex128, J = 1/2, dg = 1e-5
    and dt = 0.02 per step): the dual-line path and the three red paths run
    together (one pass launch serves all four), with energies traced every
    100 steps; extrema of d2E/dg2 from local quadratic fits, beside the
    values the paper prints (Figs. dual_evo, sec_order)."""
    import numpy as np
    from paper_2108_13410_amd import protocols as pr
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C128)
    runs = [("dual line", pr.dual_path(0.5), 0.1798)] + \
           [(f"red r={r}", pr.red_path(0.5, r), paper) for r, paper in ((0.05, 0.1920), (0.15, 0.1916), (0.25, 0.2489))]
    inits = [{"psi1": z2h.Z2H_INIT_PSI1, "psi1p": z2h.Z2H_INIT_PSI1P}[init] for _, (init, _, _), _ in runs]
    paths = [z2h.make_path(verts, steps, pr.DT, sampling=1, every=100) for _, (_, verts, steps), _ in runs]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, trace = z2h.z2h_paths_evolve(plan, paths, inits=inits)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    tr = trace[:, :, 1].cpu().numpy()
    out, steps_total = [], 0
    for j, (name, (init, verts, steps), paper) in enumerate(runs):
        n = steps[-1] // 100               # the last leg (g from 0.5 to 0) has equal length on every path
        E = tr[-n - 1:, j][::-1]
        g = np.linspace(0.0, 0.5, n + 1)
        x, d2 = pr.second_derivative(g, E, 10)
        gx, _ = pr.extremum_in(x, d2, 0.05, 0.45, "min")
        out.append({"path": name, "steps": int(sum(steps)), "d2E_extremum_g": gx, "paper": paper})
        steps_total += sum(steps)
    return {"runs": out, "seconds": el, "trotter_steps_per_s": steps_total / el,
            "amp_updates_per_s": steps_total * (1 << 18) / el, "precision": "complex128",
            "launch": "four paths per pass launch (z2h_paths_evolve)",
            "traces": "observables every 100 steps (every 1e-3 in g)"}


def dos_leg(z2h, torch):
    """Figs. dos_sec and dos_dual (Sec. V) on the 3x3 torus, complex128, paper
    protocol: the distribution of |psi|^2 over Ztilde = 2w - n on the red
    paths (r = 0.01 .. 0.19, run together) at g = 0.19, and on the dual line
    at g = 0.65 and 0.30, with the maxima of each (peaks of at least 1 % of
    the largest bin; "interior" leaves out the ends of the occupied range)."""
    from paper_2108_13410_amd import protocols as pr
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C128)
    t0 = time.perf_counter()
    red, dual = pr.dos_study(z2h, plan)
    el = time.perf_counter() - t0
    n = plan.n
    row = lambda d: {"maxima_at_Ztilde": pr.dos_maxima(d, n), "interior_maxima": pr.dos_maxima(d, n, True),
                     "dos": [round(float(x), 6) for x in d]}
    return {"seconds": el, "red_g0.19": {str(r): row(d) for r, d in red.items()},
            "dual_line": {str(g): row(d) for g, d in dual.items()},
            "paper": "single maximum for r < 0.16 (Fig. dos_sec); on the dual line two maxima at g = 0.30 with "
                     "one at Ztilde = -10, one maximum at g = 0.65 (Fig. dos_dual)"}


def blue_leg(z2h, torch, ps=(0.36, 0.32, 0.28, 0.24)):
    """Fig. 3maxima (Sec. V): psi_1 along the g axis to P(p, 0), then the blue
    line to P'(0, p), for four p, run together (3x3, complex128, paper
    protocol, energies every 100 steps).  On the blue leg, d2E/dg2 from
    local quadratic fits; its largest and smallest values and all its local
    extrema, beside the dual point lambda = p/2."""
    import numpy as np
    from paper_2108_13410_amd import protocols as pr
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C128)
    paths = []
    for p in ps:
        _, verts, steps = pr.topo_paths(p)["E"]
        paths.append(z2h.make_path(verts, steps, pr.DT, sampling=1, every=100))
    t0 = time.perf_counter()
    _, tr = z2h.z2h_paths_evolve(plan, paths)
    tr = tr.cpu().numpy()
    el = time.perf_counter() - t0
    out = {}
    for j, p in enumerate(ps):
        nb = paths[j].steps[1] // 100
        lam = np.linspace(0, p, nb + 1)
        x, d2 = pr.second_derivative(lam, tr[-nb - 1:, j, 1], 10)
        ext = [round(float(x[i]), 3) for i in range(1, len(d2) - 1) if (d2[i] - d2[i - 1]) * (d2[i + 1] - d2[i]) < 0]
        out[str(p)] = {"dual_point_lambda": p / 2, "d2_max_at": float(x[np.argmax(d2)]),
                       "d2_min_at": float(x[np.argmin(d2)]), "local_extrema_at": ext}
    return {"seconds": el, "paths": out}


def refinement_leg(z2h, torch, ns=(10, 200, 500, 800)):
    """Table contrast_tab (Sec. VI): the red path to R(0.5, 0.05) and on to
    R'(0, 0.05) with dg = 1e-4/n and dt = 0.2/n per step, n = 10 (the
    protocol), 200, 500, 800; E_n(g) on the last leg at the n = 10 grid
    (every 1e-5 in g, 50001 points); delta_n = sum |E_10 - E_n|, alpha_n =
    max.  3x3, complex128; the four paths run concurrently, one stream each."""
    import threading
    import numpy as np
    from paper_2108_13410_amd import protocols as pr
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C128)
    sz = z2h.z2h_plan_sizes(plan)
    runs = {}

    def one(n):
        init, verts, steps, dt = pr.refined_red_path(0.5, 0.05, n)
        stream = torch.cuda.Stream()
        with torch.cuda.stream(stream):
            psi = z2h.alloc_state(plan)
            ws = z2h.alloc_bytes(max(sz["ws_evolve"], sz["ws_observe"]))
            z2h.z2h_state_init(plan, psi, z2h.Z2H_INIT_PSI1, stream=stream.cuda_stream)
            t0 = time.perf_counter()
            E = {}
            for i in range(3):
                # one leg per call; energies every 1e-5 in g on the two legs that vary g
                every = n // 10 if i != 1 else 0
                tr = z2h.z2h_path_evolve(plan, psi, ws, z2h.make_path(verts[i:i + 2], steps[i:i + 1], dt, sampling=1,
                                                                      every=every), stream=stream.cuda_stream)
                stream.synchronize()
                E[i] = tr[:, 1].cpu().numpy()
                print(f"refinement n={n}: leg {i + 1} of 3 done ({steps[i]} steps) after "
                      f"{time.perf_counter() - t0:.0f} s", file=sys.stderr, flush=True)
            runs[n] = (E[0], E[2], sum(steps), time.perf_counter() - t0)

    threads = [threading.Thread(target=one, args=(n,)) for n in ns]
    t0 = time.perf_counter()
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    wall = time.perf_counter() - t0
    paper = {200: (0.03982, 4.79e-5), 500: (0.04009, 4.99e-5), 800: (0.04075, 4.98e-5)}
    rows = []
    for n in ns:
        d1, a1 = pr.refinement_metrics(runs[ns[0]][0], runs[n][0])
        d3, a3 = pr.refinement_metrics(runs[ns[0]][1], runs[n][1])
        rows.append({"n": n, "steps": runs[n][2], "seconds": runs[n][3],
                     "delta_n": d3, "alpha_n": a3, "delta_n_g_axis": d1, "alpha_n_g_axis": a1,
                     "paper_delta_n": paper.get(n, (0.0, 0.0))[0], "paper_alpha_n": paper.get(n, (0.0, 0.0))[1]})
    return {"rows": rows, "wall_seconds": wall, "grid_points": int(len(runs[ns[0]][1])),
            "reading": "delta_n, alpha_n: E_n(g) on the leg R(0.5, 0.05) -> R'(0, 0.05); *_g_axis: on the leg "
                       "O(0, 0) -> P(0.5, 0); every leg refined; 50001 points every 1e-5 in g"}


def adjoint_leg(z2h, torch):
    """Gradient of the final energy (3x3, complex128, M = 200, T = 20, loss at
    (1, 1, 0.3, 0.3)) with respect to the 400 per-step schedule values, by
    the adjoint sweep through torch.autograd; timed beside the forward ramp."""
    from paper_2108_13410_amd import workloads
    from paper_2108_13410_amd.autograd import EvolveEnergy
    M, T = 200, 20.0
    c0, c1 = workloads.TORIC, workloads.point(0.3, 0.3)
    sZ0, sX0 = workloads.adjoint_angles(M)
    plan = z2h.z2h_plan_create(3, 3, z2h.Z2H_C128)
    times = []
    for _ in range(3):
        sZ = torch.tensor(sZ0, dtype=torch.float64, requires_grad=True)
        sX = torch.tensor(sX0, dtype=torch.float64, requires_grad=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L = EvolveEnergy.apply(sZ, sX, plan, c0, c1, T / M, c1)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        L.backward()
        torch.cuda.synchronize()
        times.append((t1 - t0, time.perf_counter() - t1))
    fwd, bwd = min(t[0] for t in times), min(t[1] for t in times)
    return {"lattice": "3x3", "steps": M, "precision": "complex128", "parameters": 2 * M,
            "loss": float(L.detach()), "forward_ms": fwd * 1e3, "backward_ms": bwd * 1e3,
            "backward_over_forward": bwd / fwd, "grad_norm": float(torch.cat([sZ.grad, sX.grad]).norm())}


def scan_c128_leg(z2h, torch, jobs, obs64):
    """The same 1024-point scan in complex128 (the paper's precision, 4 GiB of
    states) as one batch run with event-timed pass kernels: throughput, the
    roofline of each pass kind, and the complex64 scan's distance to it."""
    nj, n, M = len(jobs), 18, jobs[0]["M"]
    batch = make_batch(jobs, z2h.Z2H_C128, z2h)
    states = torch.empty(batch.states_bytes, dtype=torch.uint8, device="cuda")
    ws = torch.empty(batch.ws_bytes, dtype=torch.uint8, device="cuda")
    obs = torch.zeros(nj * z2h.Z2H_OBS_DOUBLES, dtype=torch.float64, device="cuda")
    z2h.z2h_batch_run(batch, states, ws, obs)  # graph recorded
    z2h.z2h_timing_enable(True)
    z2h.z2h_batch_run(batch, states, ws, obs)  # timed mode warmed
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    z2h.z2h_batch_run(batch, states, ws, obs)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    counts, ms = z2h.z2h_batch_timing(batch)
    z2h.z2h_timing_enable(False)
    t0 = time.perf_counter()
    z2h.z2h_batch_run(batch, states, ws, obs)
    torch.cuda.synchronize()
    graph_s = time.perf_counter() - t0
    bytes_per_launch = 2 * nj * (1 << n) * 16
    per_kind = {}
    for kind, idx in (("z", 0), ("x", 1)):
        if counts[idx]:
            avg = float(ms[idx]) / int(counts[idx])
            ach = bytes_per_launch / (avg * 1e-3) / 1e9
            per_kind[kind] = {"launches": int(counts[idx]), "avg_launch_ms": avg, "achieved_GBps": ach,
                              "frac": ach / HBM_PEAK_GBS}
    o128 = obs.cpu().numpy().reshape(nj, -1)
    del states, ws, obs, batch
    torch.cuda.empty_cache()
    return {"seconds": el, "graph_seconds": graph_s, "amp_updates_per_s": nj * (1 << n) * M / el,
            "bytes_per_pass_launch": bytes_per_launch, "pass": per_kind,
            "c64_scan_vs_c128_scan": {
                "max_abs_err_energy_per_link": float(abs(o128[:, 1] - obs64[:, 1]).max() / n),
                "max_abs_err_wilson": float(max(abs(o128[:, 6] - obs64[:, 6]).max(),
                                                abs(o128[:, 7] - obs64[:, 7]).max()))},
            "c64_scan_speedup": None}


def mixed_leg(z2h, torch):
    """The mixed batch (32 each of 2x2, 2x3 and 3x3 tori, (hx, hz) ~ U[0, 0.6]^2,
    M ~ U{200..1000}, T = 20, seeded) in complex64 as one batch run."""
    from paper_2108_13410_amd import workloads
    jobs = workloads.mixed()
    batch = make_batch(jobs, z2h.Z2H_C64, z2h)
    states = torch.empty(batch.states_bytes, dtype=torch.uint8, device="cuda")
    ws = torch.empty(batch.ws_bytes, dtype=torch.uint8, device="cuda")
    obs = torch.zeros(len(jobs) * z2h.Z2H_OBS_DOUBLES, dtype=torch.float64, device="cuda")
    z2h.z2h_batch_run(batch, states, ws, obs)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        z2h.z2h_batch_run(batch, states, ws, obs)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / 3
    amp = sum((1 << (2 * j["Lx"] * j["Ly"])) * j["M"] for j in jobs)
    return {"jobs": len(jobs), "lattices": "32 x 2x2, 32 x 2x3, 32 x 3x3", "ms_per_run": el * 1e3,
            "amp_updates_per_s": amp / el, "launch": "HIP graph (resident small lattices on a side stream)"}


def exact_leg(z2h, torch):
    """Exact solvers on the GPU.
    - 4x4 torus, complex128 (2^32 amplitudes; start vector plus two Lanczos
      vectors = 192 GiB): Lanczos ground energy of H at the paper's point
      P(g = 0.5, lambda = 0), J = 1/2, from |+...+>, and one H x.
      Algorithmic bytes: an H x is 2 (2K - 1) + 1 state passes (read + write
      per pass, x read again by the last); a fused Lanczos iteration is 4K
      (the last pass reads y, u and the previous vector and writes the next).
    - 3x3, complex128: the stepwise exact evolution of a 200-step ramp with a
      16-dimensional Krylov basis per step."""
    torch.cuda.empty_cache()
    out = {}
    c = (0.5, 0.5, 0.5, 0.0)
    # H x makes 2K - 1 passes over K transform groups: a three-group split
    # (12 + 10 + 10 links, the strided groups in two runs of qubits: 12-14 +
    # 22-28 and 15-21 + 29-31), not a Trotter-tuned schedule with more groups
    plan = z2h.z2h_plan_create_config(4, 4, z2h.Z2H_C128, EXACT_4X4_SPLIT)
    K = len(z2h.z2h_plan_describe(plan)["groups"])
    V = 16 << 32
    v = z2h.alloc_state(plan)
    ws = z2h.alloc_bytes(z2h.z2h_lanczos_sizes(plan, 64))
    y = ws[:V].view(torch.complex128)
    z2h.z2h_state_init(plan, v, z2h.Z2H_INIT_PLUS)
    z2h.z2h_hamiltonian_apply(plan, v, y, c)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(2):
        z2h.z2h_hamiltonian_apply(plan, v, y, c)
    torch.cuda.synchronize()
    t_hx = (time.perf_counter() - t0) / 2
    del y
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0, it, _, beta = z2h.z2h_lanczos_ground(plan, v, ws, c, max_iter=64, tol=1e-11)
    t_l = time.perf_counter() - t0
    hx_bytes = (2 * (2 * K - 1) + 1) * V
    it_bytes = 4 * K * V
    out["lanczos_4x4"] = {
        "couplings": c, "precision": "complex128", "groups": K, "E0": e0, "iterations": it,
        "last_beta": float(beta[-1]) if len(beta) else None,
        "seconds": t_l, "ms_per_iteration": t_l / it * 1e3,
        "iteration_GBps_algorithmic": it_bytes / (t_l / it) / 1e9,
        "hx_ms": t_hx * 1e3, "hx_GBps_algorithmic": hx_bytes / t_hx / 1e9,
        "hx_frac_of_hbm_peak": hx_bytes / t_hx / 1e9 / HBM_PEAK_GBS,
    }
    del v, ws
    torch.cuda.empty_cache()
    plan3 = z2h.z2h_plan_create(3, 3, z2h.Z2H_C128)
    psi = z2h.alloc_state(plan3)
    ws3 = z2h.alloc_bytes(z2h.z2h_exact_sizes(plan3, 16))
    M = 200
    sched = z2h.schedule((0.5, 0.5, 0.0, 0.0), (0.5, 0.5, 0.3, 0.2), M, 0.02)
    z2h.z2h_state_init(plan3, psi, z2h.Z2H_INIT_PSI1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    err = z2h.z2h_exact_evolve(plan3, psi, ws3, sched, krylov_dim=16)
    torch.cuda.synchronize()
    t_e = time.perf_counter() - t0
    out["exact_evolve_3x3"] = {"steps": M, "krylov_dim": 16, "ms_per_step": t_e / M * 1e3,
                               "krylov_error_estimate": err}
    return out


def circuit_leg(z2h, torch, with_4x4=False):
    """The paper's circuit at gate level (Sec. III; n links + 1 ancilla) beside
    the fused Trotter path, per Trotter step: 3x3 in complex128 gate by gate
    (522 launches), in tile groups and in register groups; optionally 4x4 (33 qubits,
    complex64, 64 GiB) in fused passes."""
    out = {}
    c0, c1, M, dt = (0.5, 0.5, 0.0, 0.0), (0.5, 0.5, 0.3, 0.2), 100, 0.02

    def gate_level(Lx, Ly, dtype, fuse, steps):
        n = 2 * Lx * Ly
        psi = torch.zeros(1 << (n + 1), dtype=torch.complex128 if dtype == z2h.Z2H_C128 else torch.complex64,
                          device="cuda")
        psi[0] = 1
        ws = z2h.alloc_bytes(z2h.z2h_gates_ws_bytes(n + 1))
        z2h.z2h_circuit_evolve(Lx, Ly, dtype, psi, ws, z2h.schedule(c0, c1, M, dt, k_end=1), fuse=fuse)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        z2h.z2h_circuit_evolve(Lx, Ly, dtype, psi, ws, z2h.schedule(c0, c1, M, dt, k_begin=1, k_end=1 + steps),
                               fuse=fuse)
        torch.cuda.synchronize()
        del psi
        torch.cuda.empty_cache()
        return (time.perf_counter() - t0) / steps

    def trotter_path(Lx, Ly, dtype, steps):
        plan = z2h.z2h_plan_create(Lx, Ly, dtype)
        phi = z2h.alloc_state(plan)
        z2h.z2h_state_init(plan, phi, z2h.Z2H_INIT_PSI1)
        ws = z2h.alloc_bytes(z2h.z2h_plan_sizes(plan)["ws_evolve"])
        z2h.z2h_evolve(plan, phi, ws, z2h.schedule(c0, c1, steps, dt))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        z2h.z2h_evolve(plan, phi, ws, z2h.schedule(c0, c1, steps, dt))
        torch.cuda.synchronize()
        del phi
        torch.cuda.empty_cache()
        return (time.perf_counter() - t0) / steps

    ng = z2h.z2h_circuit_step(3, 3, c0, c0, dt)[1]
    a, b, r, c = gate_level(3, 3, z2h.Z2H_C128, 0, 10), gate_level(3, 3, z2h.Z2H_C128, 1, 20), \
        gate_level(3, 3, z2h.Z2H_C128, 2, 20), trotter_path(3, 3, z2h.Z2H_C128, 200)
    arr3 = z2h.z2h_circuit_step(3, 3, c0, c0, dt)[0]
    passes3 = {f: z2h.z2h_gates_schedule(19, z2h.Z2H_C128, arr3, ng, f)[1] for f in (1, 2)}
    out["3x3_c128"] = {"gates_per_step": ng, "tile_passes_per_step": passes3[1],
                       "register_passes_per_step": passes3[2],
                       "gate_by_gate_ms_per_step": a * 1e3, "lds_groups_ms_per_step": b * 1e3,
                       "register_groups_ms_per_step": r * 1e3, "trotter_path_ms_per_step": c * 1e3,
                       "trotter_path_speedup_over_best_gates": min(b, r) / c}
    if with_4x4:
        ng4 = z2h.z2h_circuit_step(4, 4, c0, c0, dt)[1]
        b4, r4, c4 = gate_level(4, 4, z2h.Z2H_C64, 1, 1), gate_level(4, 4, z2h.Z2H_C64, 2, 1), \
            trotter_path(4, 4, z2h.Z2H_C64, 3)
        arr4 = z2h.z2h_circuit_step(4, 4, c0, c0, dt)[0]
        passes4 = {f: z2h.z2h_gates_schedule(33, z2h.Z2H_C64, arr4, ng4, f)[1] for f in (1, 2)}
        out["4x4_c64"] = {"gates_per_step": ng4, "tile_passes_per_step": passes4[1],
                          "register_passes_per_step": passes4[2], "lds_groups_ms_per_step": b4 * 1e3,
                          "register_groups_ms_per_step": r4 * 1e3, "trotter_path_ms_per_step": c4 * 1e3,
                          "trotter_path_speedup_over_best_gates": min(b4, r4) / c4}
    return out


def cpu_baseline(seconds_hint):
    """The FP64 oracle (test infrastructure, untuned) on a bounded sample of
    the scan: a few of its points, every Trotter step of each."""
    import oracle
    from paper_2108_13410_amd import workloads
    jobs = workloads.scan_3x3()
    npts = int(os.environ.get("Z2H_CPU_POINTS", "4"))
    steps = int(os.environ.get("Z2H_CPU_STEPS", "1000"))
    picks = [jobs[(len(jobs) - 1) * i // max(npts - 1, 1)] for i in range(npts)]
    states = [oracle.init_psi1(3, 3) for _ in picks]
    t0 = time.perf_counter()
    for job, psi in zip(picks, states):
        oracle.evolve(3, 3, psi, job["c0"], job["c1"], steps, job["T"] / job["M"])
    dt = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    where = ", ".join(f"({j['c1'][2]:.2f}, {j['c1'][3]:.2f})" for j in picks)
    return {
        "value": (1 << 18) * steps * npts / dt, "unit": "amplitude-updates/s", "cores": threads,
        "kind": "oracle",
        "sample": f"{npts} of the scan's 1024 3x3 points (hx, hz) = {where}, {steps} of their 1000 Trotter "
                  f"steps each, FP64 gate-by-gate, {dt:.1f} s on {threads} OpenMP threads",
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--plain-points", type=int, default=16)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-tune", action="store_true")
    ap.add_argument("--no-4x4", action="store_true")
    ap.add_argument("--no-scan-c128", action="store_true", help="skip the complex128 scan leg")
    ap.add_argument("--only-4x4", default=None, metavar="PRECISIONS",
                    help="profiling: run only the 4x4 leg for these precisions (c64,c128) and print it")
    ap.add_argument("--steps-4x4", type=int, default=None, help="profiling: Trotter steps of the 4x4 leg")
    ap.add_argument("--schedule-4x4", action="append", default=[], metavar="PRECISION=SCHEDULE",
                    help="profiling: explicit 4x4 schedule string, e.g. c128=split=12:4:12:0/10:4:13:3/10:4:13:3")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--no-protocol", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint and mixed-batch legs")
    ap.add_argument("--no-exact", action="store_true", help="skip the exact-solver leg (Lanczos, Krylov)")
    ap.add_argument("--no-circuit", action="store_true", help="skip the gate-level circuit leg")
    ap.add_argument("--dos", action="store_true", help="add the Ztilde distributions of Figs. dos_sec, dos_dual")
    ap.add_argument("--blue", action="store_true", help="add the blue paths of Fig. 3maxima")
    ap.add_argument("--refinement", action="store_true",
                    help="add Table contrast_tab's refinement study (1.6e7 Trotter steps, a few minutes)")
    ap.add_argument("--circuit-4x4", action="store_true", help="add the 33-qubit gate-level step (about 10 s)")
    ap.add_argument("--tune-cache", default=None,
                    help="schedule cache: loaded if it has the needed entries, else written by the autotuner "
                         "(default: the table shipped with the package, never written)")
    ap.add_argument("--retune", action="store_true", help="run the autotuner instead of loading a table")
    ap.add_argument("--pmc-summary", nargs=2, default=None, metavar=("FETCH_CSV", "WRITE_CSV"))
    args = ap.parse_args()
    if args.tune_cache is None and not args.retune and os.path.exists(SHIPPED_TABLE):
        args.tune_cache = SHIPPED_TABLE
    if args.pmc_summary:
        pmc_summary(*args.pmc_summary)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the batched scan shards by job with no communication, "
              "and multi-GPU runs are not implemented; use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    ensure_built()
    from paper_2108_13410_amd import workloads, z2h

    torch.cuda.set_device(0)
    if args.only_4x4:
        if args.tune_cache and os.path.exists(args.tune_cache):
            z2h.z2h_tune_load(args.tune_cache)
        scheds = dict(x.split("=", 1) for x in args.schedule_4x4)
        if not args.no_copy:
            # the 2 GiB device copy that scales rocprofv3's traffic counters
            print(f"copy reference: {copy_ceiling(torch)}", file=sys.stderr, flush=True)
        out = four_by_four(z2h, torch, not args.no_tune, args.tune_cache, steps=args.steps_4x4,
                           schedules=scheds, precisions=tuple(args.only_4x4.split(",")))
        print(json.dumps({"torus_4x4": out}))
        return
    jobs = workloads.scan_3x3()
    nj = len(jobs)
    M = jobs[0]["M"]
    n = 18
    # the project's autotuner picks the pass schedule for this batch size
    # (and for single complex128 states) before anything is created
    tuned = {}
    tuned_from = "autotuned in this run" if not args.no_tune else "planner default"
    if cache_has(args.tune_cache, 18, False) and cache_has(args.tune_cache, 18, True):
        z2h.z2h_tune_load(args.tune_cache)
        tuned_from = os.path.relpath(args.tune_cache, ROOT)
        # the table's entries the scan (18 qubits, complex64, batch class 64)
        # and the single complex128 states (batch class 1) run with
        # ("qubits precision batch-class config")
        with open(args.tune_cache) as fh:
            for line in fh:
                f = line.split()
                if len(f) == 4 and (f[0], f[1], f[2]) == ("18", "0", "64"):
                    tuned["scan_c64"] = (f[3], None)
                elif len(f) == 4 and (f[0], f[1], f[2]) == ("18", "1", "1"):
                    tuned["plain_c128"] = (f[3], None)
        print(f"schedules loaded from {args.tune_cache}", file=sys.stderr, flush=True)
    elif not args.no_tune:
        out = None if args.tune_cache == SHIPPED_TABLE else args.tune_cache
        tuned["scan_c64"] = z2h.z2h_autotune(3, 3, z2h.Z2H_C64, nj, out)
        tuned["plain_c128"] = z2h.z2h_autotune(3, 3, z2h.Z2H_C128, 1, out)
        print(f"autotuned: {tuned}", file=sys.stderr, flush=True)
    batch = make_batch(jobs, z2h.Z2H_C64, z2h)
    states = torch.empty(batch.states_bytes, dtype=torch.uint8, device="cuda")
    ws = torch.empty(batch.ws_bytes, dtype=torch.uint8, device="cuda")
    obs = torch.zeros(nj * z2h.Z2H_OBS_DOUBLES, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    # Warm both launch modes: the HIP-graph replay and the timed mode, which
    # issues the same launch sequence with an event pair around every pass
    # kernel (graph-recorded events carry no timestamps).
    for _ in range(args.warmup):
        z2h.z2h_batch_run(batch, states, ws, obs)
    z2h.z2h_timing_enable(True)
    z2h.z2h_batch_run(batch, states, ws, obs)
    torch.cuda.synchronize()
    print(f"warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)

    # timed region: K steps, per-kernel HIP events live
    t0 = time.perf_counter()
    for _ in range(args.steps):
        z2h.z2h_batch_run(batch, states, ws, obs)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    counts, ms = z2h.z2h_batch_timing(batch)  # pass kernels of the last timed step
    z2h.z2h_timing_enable(False)
    ms_step = 1000.0 * elapsed / args.steps
    amp_updates = nj * (1 << n) * M
    value = amp_updates / (elapsed / args.steps)
    print(f"timed {args.steps} steps: {ms_step:.1f} ms/step", file=sys.stderr, flush=True)

    # the same steps replayed from the HIP graph
    t0 = time.perf_counter()
    for _ in range(args.steps):
        z2h.z2h_batch_run(batch, states, ws, obs)
    torch.cuda.synchronize()
    graph_ms = 1000.0 * (time.perf_counter() - t0) / args.steps

    # Per pass kind (z: group 0 with the Z phase, x: top group with the X
    # phase, plain: transform only), each a level_kernel_full instance; the
    # roofline is reported for the kind with the largest total time.
    bytes_per_launch = 2 * nj * (1 << n) * 8  # every amplitude read once and written once
    traffic = None
    if os.path.exists(TRAFFIC_FILE):
        with open(TRAFFIC_FILE) as f:
            tr = json.load(f)
        if tr.get("kernel_source_sha256_16") == kernel_hash():
            traffic = {}
            names = pass_kernel_names(z2h, tuned.get("scan_c64", (None,))[0])
            for kind, name in names.items():
                for k, v in tr.get("per_kernel_bytes", {}).items():
                    if k.startswith(f"void z2h::{name}(") and k.endswith(f"grid={nj << 14}"):
                        traffic[kind] = v
    per_kind = {}
    for kind, idx in (("z", 0), ("x", 1), ("plain", 2)):
        if counts[idx] == 0:
            continue
        avg = float(ms[idx]) / int(counts[idx])
        ach = bytes_per_launch / (avg * 1e-3) / 1e9
        per_kind[kind] = {"launches": int(counts[idx]), "total_ms": float(ms[idx]), "avg_launch_ms": avg,
                          "achieved_GBps": ach, "frac": ach / HBM_PEAK_GBS,
                          "traffic": None if traffic is None else traffic.get(kind)}
    dom = max(("z", "x"), key=lambda k: per_kind[k]["total_ms"])
    obs_np = obs.cpu().numpy().reshape(nj, -1)

    line = {
        "metric": "amplitude-updates/s per Trotter step & % of HBM peak; batched c64 vs plain c128",
        "value": value,
        "unit": "amplitude-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "scan_3x3_32x32_c64", "lattice": "3x3 torus", "qubits": n,
                   "states": nj, "trotter_steps": M, "T": jobs[0]["T"],
                   "grid": "(hx, hz) in linspace(0, 0.6, 32)^2", "storage": "complex64",
                   "parallelism": "1 GPU", "launch": "timed: direct launches with per-kernel events"},
        "graph_ms_per_step": graph_ms,
        "schedule": {k: {"config": v[0], "ms_per_trotter_step": v[1]} for k, v in tuned.items()},
        "schedule_source": tuned_from,
        "roofline": {"bound": "hbm", "achieved": per_kind[dom]["achieved_GBps"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": per_kind[dom]["frac"], "traffic": per_kind[dom]["traffic"],
                     "kernel": f"level_kernel_full, {dom} pass (largest total time)",
                     "launches_timed": per_kind[dom]["launches"], "avg_launch_ms": per_kind[dom]["avg_launch_ms"],
                     "bytes_per_launch": bytes_per_launch},
        "roofline_by_pass": per_kind,
    }
    if not args.no_copy:
        line["copy_reference"] = copy_ceiling(torch)
        print(f"copy reference: {line['copy_reference']}", file=sys.stderr, flush=True)
    if not args.no_plain:
        per_point, res = plain_c128(jobs, z2h, torch, args.plain_points)
        err_e = max(abs(res[j][1] - obs_np[j][1]) / n for j in res)
        err_w = max(max(abs(res[j][6] - obs_np[j][6]), abs(res[j][7] - obs_np[j][7])) for j in res)
        line["plain_c128"] = {
            "ms_per_point": per_point * 1e3,
            "value": (1 << n) * M / per_point,
            "scan_seconds": per_point * nj,
            "batched_speedup": per_point * nj / (elapsed / args.steps),
            "points_compared": len(res),
            "max_abs_err_energy_per_link": err_e,
            "max_abs_err_wilson": err_w,
        }
        print(f"plain c128: {per_point*1e3:.2f} ms/point", file=sys.stderr, flush=True)
    if not args.no_scan_c128:
        line["scan_c128"] = scan_c128_leg(z2h, torch, jobs, obs_np)
        line["scan_c128"]["c64_scan_speedup"] = line["scan_c128"]["seconds"] / (elapsed / args.steps)
        sc = line["scan_c128"]
        print(f"scan c128: {sc['seconds']:.3f} s, {sc['amp_updates_per_s']:.3e} amplitude-updates/s, passes "
              + ", ".join(f"{k} {v['achieved_GBps']:.0f} GB/s" for k, v in sc["pass"].items()),
              file=sys.stderr, flush=True)
    if not args.no_4x4:
        line["torus_4x4"] = four_by_four(z2h, torch, not args.no_tune, args.tune_cache)
    if not args.no_adjoint:
        line["adjoint"] = adjoint_leg(z2h, torch)
        line["mixed_batch"] = mixed_leg(z2h, torch)
        print(f"adjoint: {line['adjoint']['backward_ms']:.1f} ms, mixed batch: {line['mixed_batch']['ms_per_run']:.1f} ms",
              file=sys.stderr, flush=True)
    if not args.no_exact:
        line["exact"] = exact_leg(z2h, torch)
        lz = line["exact"]["lanczos_4x4"]
        print(f"exact: 4x4 E0 = {lz['E0']:.10f} ({lz['iterations']} it, {lz['ms_per_iteration']:.0f} ms/it), "
              f"H x {lz['hx_GBps_algorithmic']:.0f} GB/s", file=sys.stderr, flush=True)
    if not args.no_circuit:
        line["gate_level"] = circuit_leg(z2h, torch, args.circuit_4x4)
        g3 = line["gate_level"]["3x3_c128"]
        print(f"gate level 3x3: {g3['gate_by_gate_ms_per_step']:.2f} / {g3['lds_groups_ms_per_step']:.2f} / "
              f"{g3['register_groups_ms_per_step']:.2f} ms per step (Trotter path {g3['trotter_path_ms_per_step']:.3f})",
              file=sys.stderr, flush=True)
    if not args.no_protocol:
        line["paper_protocol"] = paper_protocol(z2h, torch)
        print(f"paper protocol: {line['paper_protocol']['trotter_steps_per_s']:.0f} steps/s", file=sys.stderr, flush=True)
    if args.dos:
        line["dos"] = dos_leg(z2h, torch)
        for r, v in line["dos"]["red_g0.19"].items():
            print(f"dos red r={r} g=0.19: maxima at Ztilde {v['maxima_at_Ztilde']} (interior {v['interior_maxima']})",
                  file=sys.stderr, flush=True)
        for g, v in line["dos"]["dual_line"].items():
            print(f"dos dual line g={g}: maxima at Ztilde {v['maxima_at_Ztilde']}", file=sys.stderr, flush=True)
    if args.blue:
        line["blue_paths"] = blue_leg(z2h, torch)
        for p, v in line["blue_paths"]["paths"].items():
            print(f"blue p={p}: d2E max at {v['d2_max_at']:.3f}, min at {v['d2_min_at']:.3f}, dual point "
                  f"{v['dual_point_lambda']:.3f}", file=sys.stderr, flush=True)
    if args.refinement:
        line["refinement"] = refinement_leg(z2h, torch)
        for r in line["refinement"]["rows"]:
            print(f"refinement n={r['n']}: R->R' delta {r['delta_n']:.5f} alpha {r['alpha_n']:.3g}; "
                  f"O->P delta {r['delta_n_g_axis']:.5f} alpha {r['alpha_n_g_axis']:.3g} "
                  f"(paper {r['paper_delta_n']}, {r['paper_alpha_n']}), {r['seconds']:.0f} s", file=sys.stderr, flush=True)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(15)
    line["paper_context"] = {"rtx3090_c128_19q": ">= 0.8e7-1.8e7 link-amplitude-updates/s, derived from "
                             "the wall time per red path the paper states for its RTX 3090 runs (Sec. VII)"}
    print(json.dumps(line))


if __name__ == "__main__":
    main()
