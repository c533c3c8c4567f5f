#!/usr/bin/env python
"""Benchmark of the multigrid hot path on one MI355X.

A step is one whole solve to 1e-10 (relative max-norm residual) of the
256^3 homogeneous-Dirichlet Poisson problem split into 512 boxes of 32^3
(1 ghost cell), FP64, V(2,2) red-black Gauss-Seidel down to a 2^3 CG bottom,
right-hand side i.i.d. uniform[-1, 1] (seed 2), inputs resident in HBM.

value = fine-cell V-cycle updates per second = 256^3 * cycles / solve time.

The JSON line also carries
  roofline     : the level-0 Gauss-Seidel colour kernel (the dominant one),
                 algorithmic bytes per launch / its mean duration from HIP
                 events recorded around each of its launches in the timed
                 steps, against the 8 TB/s HBM peak; traffic = HBM bytes per
                 launch from rocprofv3 counters (FETCH_SIZE + WRITE_SIZE,
                 scaled by the same counters on a copy of known size), when a
                 summary taken on the current kernel source is committed;
  cpu_baseline : the FP64 oracle on the machine's host, one thread, on a bounded
                 sample (two V-cycles of the same problem).

After the headline the same line carries, unless --sections says otherwise:
  c1              : 32^3 periodic sine problem in one box, FP64: time per
                    V-cycle (latency-bound; no roofline claim)
  mixed_precision : 512^3 variable coefficient in 512 boxes of 64^3, FP64
                    V-cycles vs FP32 V-cycles inside FP64 refinement vs
                    conjugate gradients preconditioned by the FP32 V-cycle
  heat            : backward-Euler heat steps on the headline geometry, each
                    a Helmholtz solve started from the previous state
  nodal           : the nodal Poisson solver on the 257^3 nodes of the
                    headline domain
  composite       : two-level composite Poisson (256^3 coarse cells, the
                    central half refined by 2: 256^3 fine cells in 512
                    boxes), time per solve and per cycle
  batched         : 256 periodic problems of edges 32..128, batch engine vs
                    plain FP64 solves one at a time
  serving         : an open-loop trace of 2000 requests (200/s), continuous
                    batching vs plain FP64 first-come-first-served, p50/p99
                    latency, and a sweep of the arrival rate (x0.5 .. x4)
                    for the largest sustainable solves/s
The CPU leg (the oracle, on the host's cores; --no-cpu-baseline skips it)
adds to those rows: the oracle's time per cycle (C1, and the 512^3 problem
in a background process started before the GPU work), its solves/s on the
host's cores for a sample of the batch, and, per result of each row, the
relative residual recomputed with the oracle's FP64 operator and the error
against the oracle's solution (against the GPU's FP64 solution at 512^3,
where an oracle solve would take hours).

Other modes (not the benchmark line):
  --calibrate-copy          also run one elementwise kernel that reads and
                            writes 1 GiB (scales the counters)
  --summarize-counters DIR  turn the rocprofv3 --pmc outputs under
                            DIR/<shape>/{fetch,write} into
                            profiles/counters_gs_level0_256c512.json
  --no-headline             run only the sections (for profiling them)
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import os
import platform
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N = 256
MAX_BOX = 32
SEED = 2
TOL = 1e-10
PEAK_GBPS = 8000.0
# the sources that decide what the counted launches do: the kernels, and the
# host code that lays out the levels and picks their tiles
KERNEL_SRCS = [os.path.join(ROOT, "paper_2403_12179_amd", "csrc", f)
               for f in ("bxmg_kernels.hip", "bxmg_host.cpp", "bxmg_host.h")]
COUNTERS = os.path.join(ROOT, "profiles", "counters_gs_level0_256c512.json")
GS_KERNEL = "k_gs<double, 0>"
GS_MATCH = "k_gs<double, 0"
COPY_BYTES = 1 << 30

# Compulsory bytes per fine cell per V(2,2) cycle, FP64 (s = 8 B), per level
# l with N_l cells: 8 half-sweeps x 1.5 s N_l + residual/restriction
# (2 + 1/8) s N_l + zeroing the coarse guess s N_l / 8 + prolongation
# (2 + 1/8) s N_l = 16.375 s N_l; sum over levels 8/7 N_0; plus the level-0
# convergence residual 2 s N_0.
BYTES_PER_CELL_CYCLE = 8.0 * (16.375 * 8.0 / 7.0 + 2.0)
GS_BYTES_PER_CELL = 1.5 * 8.0  # one colour: read other colour, rhs of this colour, write this colour


def src_sha():
    h = hashlib.sha256()
    for f in KERNEL_SRCS:
        h.update(open(f, "rb").read())
    return h.hexdigest()[:16]


def cpu_info():
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        model = [l.split(":", 1)[1].strip() for l in out.splitlines() if l.startswith("Model name")]
        return (model[0] if model else platform.processor()), os.cpu_count()
    except Exception:
        return platform.processor(), os.cpu_count()


def make_problem(bx, W):
    ba = bx.BoxArray.chop((0, 0, 0), (N - 1,) * 3, MAX_BOX, bc=(bx.DIRICHLET0,) * 3)
    f = W.uniform_rhs((N, N, N), SEED)
    phi = bx.MultiFab(ba).set_val(0.0)
    rhs = bx.MultiFab(ba).set_val(0.0).from_global(f)
    return ba, f, phi, rhs


def shape_key(z, r, ly):
    return "%d,%d,%d" % (z, r, ly)


def traffic_from_counters(key):
    """HBM bytes per level-0 GS launch for launch shape `key` (planes per
    thread, buffer addressing, log2 tile-row cap), from the committed counter
    summary, if it was taken on the current kernel source and that shape."""
    if not os.path.exists(COUNTERS):
        return None
    c = json.load(open(COUNTERS))
    if c.get("kernel_src_sha") != src_sha():
        return None
    e = c.get("shapes", {}).get(key)
    return e.get("hbm_bytes_per_launch") if e else None


def summarize_counters(d):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the level-0 GS launches
    and of the 1 GiB elementwise calibration kernel, from the rocprofv3 --pmc
    databases under d/<shape>/fetch and d/<shape>/write (shape directories
    named z<Z>_r<R>_l<L>, one pair of runs per launch shape); writes the
    committed summary."""
    import sqlite3

    def rows(sub, counter):
        dbs = glob.glob(os.path.join(sub, "**", "*.db"), recursive=True)
        if not dbs:
            raise SystemExit("no rocprofv3 database under %s" % sub)
        out = []
        for db in dbs:
            con = sqlite3.connect(db)
            out += list(con.execute("select dispatch_id, kernel_name, grid_size, value from counters_collection "
                                    "where counter_name = ?", (counter,)))
        return out

    def per_dispatch(rs, match, largest_only):
        vals, grids = {}, {}
        for disp, name, grid, value in rs:
            if match in name:
                vals[disp] = vals.get(disp, 0.0) + float(value)
                grids[disp] = grid
        if largest_only:  # the level-0 launches are the largest of the kernel
            top = max(grids.values(), default=0)
            return [v for d, v in vals.items() if grids[d] == top]
        return list(vals.values())

    out = {"kernel": GS_KERNEL, "workload": "256^3 in 512 boxes of 32^3, FP64", "kernel_src_sha": src_sha(),
           "command_per_shape": ["cd /tmp && timeout -s KILL 300 rocprofv3 --pmc %s -d $REPO/%s/z<Z>_r<R>_l<L>/%s "
                                 "-o c2 -- python3 $REPO/bench.py --steps 1 --warmup 0 --no-cpu-baseline "
                                 "--sections '' --knobs <Z>,<R>,<L> --calibrate-copy"
                                 % (c, os.path.relpath(d, ROOT), sub) for c, sub in (("FETCH_SIZE", "fetch"),
                                                                                 ("WRITE_SIZE", "write"))],
           "shapes": {}}
    scales = []
    for sd in sorted(x for x in glob.glob(os.path.join(d, "z*_r*_l*")) if os.path.isdir(x)):
        z, r, ly = (int(x[1:]) for x in os.path.basename(sd).split("_"))
        e = {}
        for counter, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
            rs = rows(os.path.join(sd, sub), counter)
            gs = per_dispatch(rs, GS_MATCH, True)
            cp = per_dispatch(rs, "MulFunctor", False)
            if not gs or not cp:
                raise SystemExit("missing dispatches for %s in %s (gs %d, copy %d)" % (counter, sd, len(gs), len(cp)))
            e[counter.lower() + "_kib_per_launch"] = sum(gs) / len(gs)
            e[counter.lower() + "_copy_kib"] = max(cp)
            e[counter.lower() + "_launches"] = len(gs)
        # the calibration kernel reads 1 GiB and writes 1 GiB
        fscale = (COPY_BYTES / 1024.0) / e["fetch_size_copy_kib"]
        wscale = (COPY_BYTES / 1024.0) / e["write_size_copy_kib"]
        e["fetch_scale"], e["write_scale"] = fscale, wscale
        e["hbm_bytes_per_launch"] = 1024.0 * (e["fetch_size_kib_per_launch"] * fscale +
                                              e["write_size_kib_per_launch"] * wscale)
        e["traffic_over_algorithmic"] = e["hbm_bytes_per_launch"] / (GS_BYTES_PER_CELL * N ** 3)
        out["shapes"][shape_key(z, r, ly)] = e
        scales.append((fscale, wscale))
    if not out["shapes"]:
        raise SystemExit("no shape directories z<Z>_r<R>_l<L> under %s" % d)
    out["algorithmic_bytes_per_launch"] = GS_BYTES_PER_CELL * N ** 3
    os.makedirs(os.path.dirname(COUNTERS), exist_ok=True)
    json.dump(out, open(COUNTERS, "w"), indent=1)
    print(json.dumps(out, indent=1))


# C3 (512^3, cell beta): level-0 kernels whose HBM bytes the counters check,
# with their algorithmic bytes per fine cell (one colour of a half-sweep
# writes half the cells; beta is read at every cell once)
C3_N = 512
C3_KERNELS = [
    ("FP64 GS, cell beta (one colour)", "k_gs<double, 1", 20.0),
    ("FP32 GS, cell beta (one colour)", "k_gs<float, 1", 10.0),
    ("FP64 residual with the float cast", "k_resid<double, 1, float", 28.0),
    ("FP64 residual+restriction", "k_resid_restrict<double, 1>", 25.0),
]
C3_COUNTERS = os.path.join(ROOT, "profiles", "counters_c3_level0_512c512_varcoef.json")


def summarize_counters_c3(d):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the C3 level-0 launches
    in C3_KERNELS (the largest launches of each) and of the 1 GiB calibration
    kernel, from the rocprofv3 --pmc databases under d/fetch and d/write;
    writes the committed summary."""
    import sqlite3

    def rows(sub, counter):
        dbs = glob.glob(os.path.join(sub, "**", "*.db"), recursive=True)
        if not dbs:
            raise SystemExit("no rocprofv3 database under %s" % sub)
        out = []
        for db in dbs:
            con = sqlite3.connect(db)
            out += list(con.execute("select dispatch_id, kernel_name, grid_size, value from counters_collection "
                                    "where counter_name = ?", (counter,)))
        return out

    def largest(rs, match):
        vals, grids = {}, {}
        for disp, name, grid, value in rs:
            if match in name:
                vals[disp] = vals.get(disp, 0.0) + float(value)
                grids[disp] = grid
        top = max(grids.values(), default=0)
        return [v for k, v in vals.items() if grids[k] == top]

    cells = float(C3_N) ** 3
    out = {"workload": "512^3 in 512 boxes of 64^3, cell beta, FP64 / FP32-in-FP64 / PCG solves to 1e-10",
           "kernel_src_sha": src_sha(),
           "commands": ["cd /tmp && timeout -s KILL 300 rocprofv3 --pmc %s -d $REPO/%s/%s -o c3 -- python3 "
                        "$REPO/bench.py --no-headline --sections mixed --no-cpu-baseline --calibrate-copy"
                        % (c, os.path.relpath(d, ROOT), sub) for c, sub in (("FETCH_SIZE", "fetch"),
                                                                         ("WRITE_SIZE", "write"))],
           "kernels": {}}
    scale = {}
    data = {}
    for counter, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        rs = rows(os.path.join(d, sub), counter)
        cp = largest(rs, "MulFunctor")
        if not cp:
            raise SystemExit("no calibration dispatch for %s" % counter)
        scale[counter] = (COPY_BYTES / 1024.0) / max(cp)
        data[counter] = rs
    out["fetch_scale"], out["write_scale"] = scale["FETCH_SIZE"], scale["WRITE_SIZE"]
    for label, match, bpc in C3_KERNELS:
        e = {"match": match, "algorithmic_bytes_per_launch": bpc * cells}
        for counter in ("FETCH_SIZE", "WRITE_SIZE"):
            v = largest(data[counter], match)
            if not v:
                raise SystemExit("no dispatches of %s for %s" % (match, counter))
            e[counter.lower() + "_kib_per_launch"] = sum(v) / len(v)
            e[counter.lower() + "_launches"] = len(v)
        e["hbm_bytes_per_launch"] = 1024.0 * (e["fetch_size_kib_per_launch"] * scale["FETCH_SIZE"] +
                                              e["write_size_kib_per_launch"] * scale["WRITE_SIZE"])
        e["traffic_over_algorithmic"] = e["hbm_bytes_per_launch"] / e["algorithmic_bytes_per_launch"]
        out["kernels"][label] = e
    json.dump(out, open(C3_COUNTERS, "w"), indent=1)
    print(json.dumps(out, indent=1))


# ------------------------------------------------------------ other rows
def host(t):
    return np.asfortranarray(t.double().cpu().numpy())


def section_c1(bx, W, reps=20):
    """32^3 periodic, one box, f = -3 (2 pi)^2 sin sin sin, FP64, to 1e-10:
    time per V-cycle (the whole problem fits in the caches: latency-bound)."""
    import torch
    n = 32
    f, _ = W.sine_rhs(n, periodic=True)
    ba = bx.BoxArray.chop((0, 0, 0), (n - 1,) * 3, 32, bc=(bx.PERIODIC,) * 3)
    phi = bx.MultiFab(ba).set_val(0.0)
    rhs = bx.MultiFab(ba).set_val(0.0).from_global(f)
    for _ in range(3):
        phi.set_val(0.0)
        bx.mlmg_solve(phi, rhs, rel_tol=TOL)
    times = []
    for _ in range(reps):
        phi.set_val(0.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = bx.mlmg_solve(phi, rhs, rel_tol=TOL)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    times.sort()
    med = times[len(times) // 2]
    out = {"workload": "poisson_periodic_32c_1box_sine_fp64_tol1e-10", "cycles": res.cycles, "ok": res.ok,
           "ms_per_solve_median": 1000.0 * med, "us_per_cycle": 1e6 * med / max(res.cycles, 1),
           "final_rel_resid_inf": res.rel_resid_inf}
    keep = {"f": f, "u": phi.to_global(), "n": n}
    return out, keep


def section_mixed(bx, W, reps=3):
    """512^3 in 512 boxes of 64^3, Dirichlet, beta = exp(g) (g: 3 box-filter
    passes, std 1), f ~ U[-1,1]: FP64 V-cycles vs FP32 V-cycles inside FP64
    refinement vs conjugate gradients preconditioned by the FP32 V-cycle, all
    to 1e-10.  Fields drawn on the device (seeds 3 and 33)."""
    import torch
    n = 512
    ba = bx.BoxArray.chop((0, 0, 0), (n - 1,) * 3, 64, bc=(bx.DIRICHLET0,) * 3)
    f = W.uniform_rhs_device((n, n, n), 3)
    beta = W.smooth_gaussian_beta_device((n, n, n), 33)
    rhs = bx.MultiFab(ba).set_val(0.0).from_tensor(f)
    bmf = bx.MultiFab(ba).set_val(1.0).from_tensor(beta)
    keep = {"n": n, "f": host(f), "beta": host(beta), "u": {}}
    del f, beta
    phi = bx.MultiFab(ba)
    out = {"workload": "poisson_varcoef_512c_512x64c_dirichlet_tol1e-10", "boxes": len(ba)}
    for key, prec, kr in (("fp64", 0, 0), ("fp32_in_fp64_ir", 1, 0), ("pcg_fp32_vcycle", 1, 1)):
        times, res = [], None
        for r in range(reps + 1):
            phi.set_val(0.0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = bx.mlmg_solve(phi, rhs, bmf, rel_tol=TOL, precision=prec, krylov=kr)
            torch.cuda.synchronize()
            if r > 0:
                times.append(time.perf_counter() - t0)
            if not res.ok:
                raise SystemExit("mixed-precision section: solve failed: %s" % res)
        ms = 1000.0 * min(times)
        out[key] = {"ms_per_solve": ms, "solves_per_s": 1000.0 / ms, "cycles": res.cycles,
                    "final_rel_resid_inf": res.rel_resid_inf}
        keep["u"][key] = phi.to_global()
    u64 = keep["u"]["fp64"]
    for key in ("fp32_in_fp64_ir", "pcg_fp32_vcycle"):
        out[key]["rel_max_diff_vs_gpu_fp64"] = float(np.max(np.abs(keep["u"][key] - u64)) / np.max(np.abs(u64)))
    out["speedup_mixed_over_fp64"] = out["fp64"]["ms_per_solve"] / out["fp32_in_fp64_ir"]["ms_per_solve"]
    out["speedup_pcg_over_fp64"] = out["fp64"]["ms_per_solve"] / out["pcg_fp32_vcycle"]["ms_per_solve"]
    del phi, rhs, bmf
    torch.cuda.empty_cache()
    return out, keep


def section_heat(bx, W, steps=20, dt=1e-4):
    """Backward-Euler heat steps u_t = lap u + s on the headline geometry
    (256^3 in 512 boxes of 32^3, Dirichlet), s ~ U[-1,1] (seed 6), u0 = 0,
    each step a Helmholtz solve (alpha = 1/dt, alpha h^2 = 0.15) to 1e-10
    started from the previous state, FP64 V-cycles; the state stays on the
    device.  Reported: time per step, cycles per step, fine-cell V-cycle
    updates per second."""
    import torch
    n = N
    ba = bx.BoxArray.chop((0, 0, 0), (n - 1,) * 3, MAX_BOX, bc=(bx.DIRICHLET0,) * 3)
    src_t = W.uniform_rhs_device((n, n, n), 6)
    src = bx.MultiFab(ba, nghost=0).from_tensor(src_t)
    keep = {"n": n, "dt": dt, "src": host(src_t)}
    del src_t
    u = bx.MultiFab(ba).set_val(0.0)
    bx.heat_run(u, dt, 2, source=src, rel_tol=TOL)
    u.set_val(0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = []
    for k in range(steps):
        if k == steps - 1:
            torch.cuda.synchronize()
            t_last = time.perf_counter()
            keep["u_prev"] = u.to_global()
            t_skip = time.perf_counter() - t_last
        res.append(bx.heat_step(u, dt, source=src, rel_tol=TOL))
    torch.cuda.synchronize()
    dt_run = time.perf_counter() - t0 - t_skip
    keep["u"] = u.to_global()
    cyc = [r.cycles for r in res]
    out = {"workload": "heat_backward_euler_256c_512x32c_dirichlet_dt1e-4_tol1e-10", "steps": steps,
           "ok": all(r.ok for r in res), "ms_per_step": 1000.0 * dt_run / steps,
           "cycles_per_step_mean": sum(cyc) / len(cyc), "cycles_per_step": cyc,
           "cell_updates_per_s": n ** 3 * sum(cyc) / dt_run, "alpha_h2": 1.0 / dt / n / n}
    del u, src
    torch.cuda.empty_cache()
    return out, keep


def section_nodal(bx, W, reps=3):
    """Nodal Poisson on the nodes of the 256^3 domain (257^3 values),
    homogeneous Dirichlet, f ~ U[-1,1] (seed 7, drawn on the device), FP64
    V(2,2) to 1e-10."""
    import torch
    n = N
    ba = bx.BoxArray.chop((0, 0, 0), (n - 1,) * 3, MAX_BOX, bc=(bx.DIRICHLET0,) * 3)
    g = torch.Generator(device="cuda")
    g.manual_seed(7)
    rhs = torch.rand((n + 1,) * 3, generator=g, device="cuda", dtype=torch.float64) * 2.0 - 1.0
    phi = torch.zeros_like(rhs)
    bx.nodal_solve(ba, phi, rhs, rel_tol=TOL)
    times = []
    for _ in range(reps):
        phi.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = bx.nodal_solve(ba, phi, rhs, rel_tol=TOL)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ms = 1000.0 * min(times)
    out = {"workload": "nodal_poisson_257^3_nodes_dirichlet_fp64_tol1e-10", "ok": res.ok, "cycles": res.cycles,
           "ms_per_solve": ms, "node_updates_per_s": (n - 1) ** 3 * res.cycles / (ms / 1000.0),
           "final_rel_resid_inf": res.rel_resid_inf}
    keep = {"n": n, "f": np.asfortranarray(rhs.cpu().numpy().transpose(2, 1, 0)),
            "u": np.asfortranarray(phi.cpu().numpy().transpose(2, 1, 0))}
    del phi, rhs
    torch.cuda.empty_cache()
    return out, keep


def section_composite(bx, W, reps=3):
    """Two-level composite Poisson: 256^3 coarse cells (h0 = 1/256), the
    central half refined by 2 (256^3 fine cells in 512 boxes of 32^3),
    homogeneous Dirichlet, f ~ U[-1,1] on both levels (coarse seed 71 drawn
    on the host, fine seed 72 drawn on the device), FP64 to 1e-10."""
    import torch
    n = N
    cb, fb = W.composite_layout(n, "centre", max_box=MAX_BOX)
    cba = bx.BoxArray.from_boxes((0, 0, 0), (n - 1,) * 3, cb, bc=(bx.DIRICHLET0,) * 3)
    fba = bx.BoxArray.from_boxes((0, 0, 0), (2 * n - 1,) * 3, fb, bc=(bx.DIRICHLET0,) * 3)
    fc = W.uniform_rhs((n, n, n), seed=71)
    pc = bx.MultiFab(cba, nghost=1)
    rc = bx.MultiFab(cba, nghost=0).from_global(fc)
    g = torch.Generator(device="cuda")
    g.manual_seed(72)
    ffd = torch.zeros((2 * n,) * 3, device="cuda", dtype=torch.float64)
    lo, hi = n // 2, 3 * n // 2
    ffd[lo:hi, lo:hi, lo:hi] = torch.rand((n,) * 3, generator=g, device="cuda", dtype=torch.float64) * 2.0 - 1.0
    pf = bx.MultiFab(fba, nghost=1)
    rf = bx.MultiFab(fba, nghost=0).from_tensor(ffd)
    bx.composite_solve(pc, rc, pf, rf, rel_tol=TOL)
    times = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = bx.composite_solve(pc, rc, pf, rf, rel_tol=TOL)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
    ms = 1000.0 * min(times)
    ncov = (n // 2) ** 3
    unknowns = n ** 3 - ncov + n ** 3
    out = {"workload": "composite_poisson_256^3_coarse_+_256^3_fine_in_512_boxes_dirichlet_fp64_tol1e-10",
           "ok": res.ok, "cycles": res.cycles, "ms_per_solve": ms, "ms_per_cycle": ms / max(res.cycles, 1),
           "unknowns": unknowns, "unknown_updates_per_s": unknowns * res.cycles / (ms / 1000.0),
           "final_rel_resid_inf": res.rel_resid_inf, "levels": res.levels}
    keep = {"n": n, "cb": cb, "fb": fb, "fc": fc, "ff": np.asfortranarray(ffd.cpu().numpy()),
            "uc": pc.to_global(), "uf": pf.to_global()}
    del pc, rc, pf, rf, ffd
    torch.cuda.empty_cache()
    return out, keep


def make_batch_problems(bx, W, nprob=256, seed=4, ctx=None):
    edges = W.batch_edges(nprob, seed)
    probs = []
    for p, e in enumerate(edges):
        ba = bx.BoxArray.chop((0, 0, 0), (e - 1,) * 3, 32, bc=(bx.PERIODIC,) * 3)
        f = W.uniform_rhs_device((e, e, e), 4000 + p, mean_zero=True)
        probs.append(dict(e=e, ba=ba, f=f, phi=bx.MultiFab(ba, ctx=ctx).set_val(0.0),
                          rhs=bx.MultiFab(ba, ctx=ctx).set_val(0.0).from_tensor(f)))
    return probs


def section_batched(bx, W, nsample=4, tune_cache=None):
    """256 periodic problems, edges uniform over {32,48,64,96,128} (seed 4),
    max box 32, f ~ U[-1,1] minus its mean (seed 4000+p): the batch engine
    (FP32 V-cycles inside FP64 refinement, one launch per stage over all
    problems, hipGraph) vs plain FP64 solves one at a time, both to 1e-10.
    The batch runs on a context of its own whose launch shape is tuned on
    this batch (tune_cache False: the default shape, no tuning)."""
    import torch
    from paper_2403_12179_amd import tuning
    ctx = bx.Context(0)
    probs = make_batch_problems(bx, W, ctx=ctx)
    cells = sum(p["e"] ** 3 for p in probs)
    out = {"workload": "batch_256_periodic_edges_32-128_maxbox32_tol1e-10", "problems": len(probs),
           "cells": cells, "boxes": sum(len(p["ba"]) for p in probs)}
    if tune_cache is False:
        tuned = dict(tuning.DEFAULT_SHAPE, source="default")
        tuning.apply(ctx, tuned)
    else:
        tuned = tuning.tune_batch(ctx, [(p["phi"], p["rhs"], None, TOL) for p in probs], 12 << 30, 512,
                                  cache=tune_cache, precision=1)
    out["launch_shape"] = {k: v for k, v in tuned.items() if k != "format"}
    # warm-up on a few problems (builds, graph capture)
    b = bx.Batch(ctx, 12 << 30, 512, precision=1)
    for p in probs[:4]:
        b.add(p["phi"], p["rhs"], rel_tol=TOL)
    b.run(2)
    for p in probs:
        p["phi"].set_val(0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ids = {}
    for q, p in enumerate(probs):
        pid = b.add(p["phi"], p["rhs"], rel_tol=TOL)
        if pid is None:
            raise SystemExit("batched section: arena too small")
        ids[pid] = q
    t_add = time.perf_counter() - t0
    done = b.run(2)
    t_batch = time.perf_counter() - t0
    ok = all(r.ok for _, r in done) and len(done) == len(probs)
    cyc = [r.cycles for _, r in done]
    worst = max(r.rel_resid_inf for _, r in done)
    b.close()
    # the sampled problems' batched results, for the oracle's check
    rng = np.random.default_rng(44)
    sample = sorted(int(q) for q in rng.choice(len(probs), size=nsample, replace=False))
    by_q = {ids[i]: r for i, r in done}
    keep = [dict(q=q, e=probs[q]["e"], f=host(probs[q]["f"]), u=probs[q]["phi"].to_global(),
                 cycles=by_q[q].cycles, per=(1, 1, 1), beta=None, tol=TOL) for q in sample]
    # plain FP64, one problem after another, in the default launch shape
    tuning.apply(ctx, tuning.DEFAULT_SHAPE)
    for p in probs[:4]:
        p["phi"].set_val(0.0)
        bx.mlmg_solve(p["phi"], p["rhs"], rel_tol=TOL)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cyc64 = []
    for p in probs:
        p["phi"].set_val(0.0)
        r = bx.mlmg_solve(p["phi"], p["rhs"], rel_tol=TOL)
        cyc64.append(r.cycles)
        ok = ok and r.ok
    torch.cuda.synchronize()
    t_one = time.perf_counter() - t0
    out.update({"ok": ok, "batched_solves_per_s": len(probs) / t_batch, "batched_seconds": t_batch,
                "batched_admission_seconds": t_add, "batched_cycles_mean": sum(cyc) / len(cyc),
                "batched_worst_rel_resid_inf": worst,
                "fp64_one_at_a_time_solves_per_s": len(probs) / t_one, "fp64_one_at_a_time_seconds": t_one,
                "fp64_cycles_mean": sum(cyc64) / len(cyc64),
                "speedup_batched_over_fp64": t_one / t_batch,
                "batched_cell_updates_per_s": sum(p["e"] ** 3 * c for p, c in zip(probs, cyc)) / t_batch})
    edges = [p["e"] for p in probs]
    del probs
    torch.cuda.empty_cache()
    return out, keep, edges


def stage_requests(bx, W, trace):
    reqs = []
    for q in trace:
        e = q["edge"]
        ba = bx.BoxArray.chop((0, 0, 0), (e - 1,) * 3, 32, bc=(bx.DIRICHLET0,) * 3)
        f = W.uniform_rhs_device((e, e, e), q["seed"])
        rhs = bx.MultiFab(ba).set_val(0.0).from_tensor(f)
        bmf = None
        if q["kind"]:
            bmf = bx.MultiFab(ba).set_val(1.0).from_tensor(W.smooth_gaussian_beta_device((e, e, e), q["seed"] + 1))
        reqs.append(dict(q=q, ba=ba, phi=bx.MultiFab(ba).set_val(0.0), rhs=rhs, beta=bmf))
        del f
    return reqs


def latency_stats(lat, t_first, t_last):
    a = np.asarray(lat)
    return {"p50_ms": 1000.0 * float(np.percentile(a, 50)), "p99_ms": 1000.0 * float(np.percentile(a, 99)),
            "mean_ms": 1000.0 * float(a.mean()), "solves_per_s": len(a) / (t_last - t_first)}


def run_served(bx, ctx, reqs, speed):
    """One open-loop pass of the trace through a fresh server, arrivals at
    `speed` times the trace's rate; returns (stats, per-request results)."""
    import torch
    for r in reqs:
        r["phi"].set_val(0.0)
    srv = bx.Server(ctx, 24 << 30, max_problems=512, chunk=2, precision=1)
    torch.cuda.synchronize()
    nreq = len(reqs)
    lat, res_of, ok, nxt = {}, {}, True, 0
    t0 = time.perf_counter()
    while len(lat) + len(srv.rejected) < nreq:
        now = (time.perf_counter() - t0) * speed
        while nxt < nreq and reqs[nxt]["q"]["t"] <= now:
            r = reqs[nxt]
            srv.submit(nxt, r["phi"], r["rhs"], r["beta"], r["q"]["tol"])
            nxt += 1
        if srv.idle():
            continue
        for tag, res, t_done in srv.pump():
            lat[tag] = (t_done - t0) - reqs[tag]["q"]["t"] / speed
            res_of[tag] = res
            ok = ok and res.ok and res.rel_resid_inf <= reqs[tag]["q"]["tol"]
    t_end = max(lat[k] + reqs[k]["q"]["t"] / speed for k in lat)
    st = latency_stats(list(lat.values()), reqs[0]["q"]["t"] / speed, t_end)
    st["ok"] = ok and not srv.rejected
    st["offered_per_s"] = nreq / ((reqs[-1]["q"]["t"] - reqs[0]["q"]["t"]) / speed)
    srv.close()
    return st, res_of


def section_serving(bx, W, nreq, sweep=(0.5, 2.0, 4.0), nsample=4):
    """Open-loop trace: exponential inter-arrivals of mean 5 ms (seed 5),
    edge = clamp(16 round(exp(U(ln 32, ln 256)) / 16), 32, 256), Dirichlet,
    beta constant or lognormal (1/2 each), tol 10^U(-10,-8), f ~ U[-1,1]
    (seed 5000+q); inputs staged in HBM before the clock starts.  Served:
    continuous batching (FP32 V-cycles inside FP64 refinement, admission by
    footprint, two cycles per pump); baseline: plain FP64 solves one at a
    time in arrival order.  Latency = completion - arrival.  The sweep
    replays the trace with the arrival times scaled (x0.5 .. x4 the rate)
    through the server: a rate is sustained when the served solves/s keep
    within 5% of the offered rate."""
    import torch
    trace = W.serving_trace(nreq, 5)
    reqs = stage_requests(bx, W, trace)
    ctx = reqs[0]["phi"].ctx
    torch.cuda.synchronize()
    out = {"workload": "serving_trace_%d_req_200per_s_edges_32-256_dirichlet_tol1e-8..1e-10" % nreq,
           "requests": nreq, "mean_cells": sum(r["q"]["edge"] ** 3 for r in reqs) / nreq,
           "lognormal_share": sum(r["q"]["kind"] for r in reqs) / nreq}
    # warm-up: a few requests of each kind through a server
    srv = bx.Server(ctx, 24 << 30, max_problems=512, chunk=2, precision=1)
    for r in reqs[:4]:
        srv.submit(-1, r["phi"], r["rhs"], r["beta"], r["q"]["tol"])
    while not srv.idle():
        srv.pump()
    srv.close()
    out["served"], res_of = run_served(bx, ctx, reqs, 1.0)
    # the sampled requests' served results, for the oracle's check (edges
    # up to 128, where an oracle solve takes seconds)
    small = [q for q in range(nreq) if reqs[q]["q"]["edge"] <= 128]
    rng = np.random.default_rng(55)
    sample = sorted(int(q) for q in rng.choice(small, size=min(nsample, len(small)), replace=False))
    keep = []
    for q in sample:
        r = reqs[q]
        keep.append(dict(q=q, e=r["q"]["edge"], f=r["rhs"].to_global(), u=r["phi"].to_global(),
                         beta=r["beta"].to_global() if r["beta"] is not None else None, per=(0, 0, 0),
                         tol=r["q"]["tol"], cycles=res_of[q].cycles))
    sw = {}
    for speed in sweep:
        st, _ = run_served(bx, ctx, reqs, speed)
        sw["x%g" % speed] = st
    sw["x1"] = out["served"]
    sustained = [v["offered_per_s"] for v in sw.values() if v["solves_per_s"] >= 0.95 * v["offered_per_s"]]
    out["rate_sweep"] = dict(sorted(sw.items(), key=lambda kv: kv[1]["offered_per_s"]))
    out["max_sustained_offered_per_s"] = max(sustained) if sustained else None
    out["max_served_solves_per_s"] = max(v["solves_per_s"] for v in sw.values())
    # baseline: FP64 solves one at a time, first come first served
    for r in reqs:
        r["phi"].set_val(0.0)
    torch.cuda.synchronize()
    lat1 = []
    ok1 = True
    t0 = time.perf_counter()
    for r in reqs:
        while time.perf_counter() - t0 < r["q"]["t"]:
            pass
        res = bx.mlmg_solve(r["phi"], r["rhs"], r["beta"], rel_tol=r["q"]["tol"])
        lat1.append(time.perf_counter() - t0 - r["q"]["t"])
        ok1 = ok1 and res.ok
    t_end1 = max(l + r["q"]["t"] for l, r in zip(lat1, reqs))
    out["fp64_fcfs"] = latency_stats(lat1, reqs[0]["q"]["t"], t_end1)
    out["fp64_fcfs"]["ok"] = ok1
    out["p99_ratio_fcfs_over_served"] = out["fp64_fcfs"]["p99_ms"] / out["served"]["p99_ms"]
    del reqs
    torch.cuda.empty_cache()
    return out, keep


# ------------------------------------------------- CPU leg (the oracle)
# Everything below runs the oracle: the baseline timings on the host's cores
# and the check of sampled GPU results against the oracle's operator and
# solutions.  Worker processes are started as children that never touch the
# GPU.


def cpu_baseline(f, cycles=(1, 3)):
    """The oracle, as it stands, on the headline problem: solves of 1 and of 3
    fixed V-cycles, so the per-cycle time (their difference over 2) and the
    setup (hierarchy, ghost plans, first residual) are stated apart; value is
    the per-cycle rate."""
    from oracle import pyoracle as orc
    orc.build()
    boxes = orc.chop((0, 0, 0), (N - 1,) * 3, MAX_BOX)
    t = {}
    for c in cycles:
        t0 = time.perf_counter()
        orc.solve((0, 0, 0), (N - 1,) * 3, (0, 0, 0), boxes, f, fixed_cycles=c)
        t[c] = time.perf_counter() - t0
    c0, c1 = cycles
    per_cycle = (t[c1] - t[c0]) / (c1 - c0)
    setup = t[c0] - c0 * per_cycle
    model, ncpu = cpu_info()
    return {"value": N ** 3 / per_cycle, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "s_per_cycle": per_cycle, "setup_s": setup,
            "sample": "solves of %d and %d fixed V(2,2) cycles of the 256^3 / 512-box FP64 problem, 1 thread, "
                      "%.1f s and %.1f s: per cycle their difference over %d, setup the rest; host %s, "
                      "%s logical CPUs" % (c0, c1, t[c0], t[c1], c1 - c0, model, ncpu),
            "seconds": t[c0] + t[c1]}


def cpu_c1():
    """The oracle's C1 solve: time per V-cycle, one thread."""
    import workloads as W
    from oracle import pyoracle as orc
    orc.build()
    n = 32
    f, s = W.sine_rhs(n, periodic=True)
    t0 = time.perf_counter()
    u, info = orc.solve((0, 0, 0), (n - 1,) * 3, (1, 1, 1), orc.chop((0, 0, 0), (n - 1,) * 3, 32), f)
    dt = time.perf_counter() - t0
    return {"us_per_cycle": 1e6 * dt / max(info["cycles"], 1), "cycles": info["cycles"], "cores": 1,
            "sample": "the whole 32^3 solve incl. setup, 1 thread"}, u


def cpu_rows(orc, W, keep):
    """The oracle, as it stands, beside the heat, nodal and composite rows
    (one thread each, bounded samples, setup included)."""
    out = {}
    model, ncpu = cpu_info()
    host_s = "host %s, %s logical CPUs" % (model, ncpu)
    if "heat" in keep:
        k = keep["heat"]
        n, dt = k["n"], k["dt"]
        boxes = orc.chop((0, 0, 0), (n - 1,) * 3, MAX_BOX)
        t0 = time.perf_counter()
        orc.heat_step((0, 0, 0), (n - 1,) * 3, (0, 0, 0), boxes, k["u_prev"], dt, source=k["src"], fixed_cycles=2)
        t = time.perf_counter() - t0
        out["heat"] = {"value": n ** 3 * 2 / t, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
                       "sample": "one backward-Euler step of the same problem cut to 2 V-cycles, 1 thread, %.1f s; %s"
                                 % (t, host_s)}
    if "nodal" in keep:
        n = keep["nodal"]["n"]
        t0 = time.perf_counter()
        orc.nodal_solve((n, n, n), (0, 0, 0), keep["nodal"]["f"], fixed_cycles=2)
        t = time.perf_counter() - t0
        out["nodal"] = {"value": n ** 3 * 2 / t, "unit": "node-updates/s", "cores": 1, "kind": "oracle",
                        "sample": "2 V-cycles of the same 257^3-node problem, 1 thread, %.1f s; %s" % (t, host_s)}
    if "composite" in keep:
        n = 128  # the same layout rule at half the size: ~2 s per cycle
        cb, fb = W.composite_layout(n, "centre", max_box=MAX_BOX)
        fc = W.uniform_rhs((n, n, n), seed=71)
        ff = np.zeros((2 * n,) * 3, order="F")
        lo, hi = n // 2, 3 * n // 2
        ff[lo:hi, lo:hi, lo:hi] = W.uniform_rhs((n, n, n), seed=72)
        t0 = time.perf_counter()
        orc.composite_solve(n, (0, 0, 0), cb, fb, fc, ff, fixed_cycles=2)
        t = time.perf_counter() - t0
        unknowns = n ** 3 - (n // 2) ** 3 + n ** 3
        out["composite"] = {"value": unknowns * 2 / t, "unit": "unknown-updates/s", "cores": 1, "kind": "oracle",
                            "sample": "2 composite cycles of the 128^3 + 128^3 problem (central half refined), "
                                      "1 thread, %.1f s; %s" % (t, host_s)}
    return out


def cpu_leg_c3(out_path):
    """Child process: the oracle on the 512^3 variable-coefficient problem
    (host draws of the same recipe, seeds 3 and 33), one thread: setup plus
    the first residual, then the same plus one V-cycle; the difference is
    the time per cycle."""
    import workloads as W
    from oracle import pyoracle as orc
    orc.build()
    n = 512
    f = W.uniform_rhs((n, n, n), 3)
    beta = W.smooth_gaussian_beta((n, n, n), 33)
    boxes = orc.chop((0, 0, 0), (n - 1,) * 3, 64)
    t0 = time.perf_counter()
    orc.solve((0, 0, 0), (n - 1,) * 3, (0, 0, 0), boxes, f, beta, max_cycles=0, rel_tol=0.0)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    orc.solve((0, 0, 0), (n - 1,) * 3, (0, 0, 0), boxes, f, beta, fixed_cycles=1)
    t_one = time.perf_counter() - t0
    json.dump({"setup_and_residual_s": t_setup, "seconds_per_cycle": t_one - t_setup, "cores": 1,
               "sample": "512^3 / 512 boxes of 64^3, variable beta, FP64: one V(2,2) cycle (plus its residual), "
                         "timed as the difference of a 1-cycle and a 0-cycle solve, 1 thread"},
              open(out_path, "w"))


def cpu_leg_c4(problems, out_path):
    """Child process: oracle FP64 solves (to 1e-10) of the given batch
    problems, one after another, one thread (host draws of the same recipe)."""
    import workloads as W
    from oracle import pyoracle as orc
    orc.build()
    res = []
    for q, e in problems:
        f = W.uniform_rhs((e, e, e), 4000 + q, mean_zero=True)
        t0 = time.perf_counter()
        _, info = orc.solve((0, 0, 0), (e - 1,) * 3, (1, 1, 1), orc.chop((0, 0, 0), (e - 1,) * 3, 32), f,
                            rel_tol=TOL)
        res.append({"q": q, "e": e, "seconds": time.perf_counter() - t0, "cycles": info["cycles"]})
    json.dump(res, open(out_path, "w"))


def spawn_cpu_leg(args):
    """Start `python bench.py --cpu-leg ...` as a child process (it never
    initialises the GPU)."""
    return subprocess.Popen([sys.executable, os.path.abspath(__file__)] + args, cwd=ROOT,
                            stdout=subprocess.DEVNULL, stderr=subprocess.PIPE, text=True)


def cpu_c4(edges, tmpdir, budget_s=20.0):
    """The batch on the host's cores: P worker processes (P = min(16,
    logical CPUs)), each solving its share of a sample of the problems with
    the oracle; CPU solves/s = solves / wall time."""
    ncpu = os.cpu_count() or 1
    P = max(1, min(16, ncpu))
    # a sample of the batch in the batch's own edge mix: the first problems,
    # sized so that the whole run stays near budget_s
    per_cell_s = 1.2e-7 * 10  # ~10 cycles at the oracle's ~0.12 us per cell-cycle
    take, cost = [], 0.0
    for q, e in enumerate(edges):
        cost += per_cell_s * e ** 3
        take.append((q, e))
        if cost >= budget_s * P or len(take) == len(edges):
            break
    shares = [take[i::P] for i in range(P)]
    procs = []
    t0 = time.perf_counter()
    for i, sh in enumerate(shares):
        if not sh:
            continue
        path = os.path.join(tmpdir, "c4_%d.json" % i)
        arg = ";".join("%d,%d" % qe for qe in sh)
        procs.append((spawn_cpu_leg(["--cpu-leg", "c4", "--cpu-problems", arg, "--cpu-out", path]), path))
    results = []
    for pr, path in procs:
        pr.wait()
        if pr.returncode != 0:
            raise SystemExit("oracle worker failed: %s" % pr.stderr.read())
        results += json.load(open(path))
    wall = time.perf_counter() - t0
    return {"solves_per_s": len(results) / wall, "solves": len(results), "cores": len(procs), "wall_s": wall,
            "cycles_mean": sum(r["cycles"] for r in results) / len(results),
            "sample": "the first %d of the 256 batch problems (edges %s), FP64 oracle solves to 1e-10 on %d "
                      "processes of 1 thread" % (len(results), sorted({e for _, e in take}), len(procs))}


def oracle_check(orc, n, per, f, beta, u, tol, solve_oracle=True, u_ref=None):
    """P9: the relative residual of u by the oracle's FP64 operator, and the
    relative error against the oracle's solution (or against u_ref)."""
    dlo, dhi = (0, 0, 0), (n - 1,) * 3
    r = f - orc.apply_op(dlo, dhi, per, 1.0 / n, u, beta)
    out = {"oracle_rel_resid_inf": float(np.max(np.abs(r)) / np.max(np.abs(f))), "tol": tol}
    out["meets_tol"] = out["oracle_rel_resid_inf"] <= tol
    if solve_oracle:
        uo, io = orc.solve(dlo, dhi, per, orc.chop(dlo, dhi, 32), f, beta, rel_tol=tol)
        out["e_rel_vs_oracle"] = float(np.max(np.abs(u - uo)) / np.max(np.abs(uo)))
        out["oracle_cycles"] = io["cycles"]
    elif u_ref is not None:
        out["e_rel_vs_gpu_fp64"] = float(np.max(np.abs(u - u_ref)) / np.max(np.abs(u_ref)))
    return out


def summarize_trace(csv_path, out_path, command):
    """The rocprofv3 --stats kernel table (csv) as a short text summary, and,
    from the kernel trace next to it, the same kernels split by launch size
    (the largest grids of the level kernels are the finest level's)."""
    import csv
    rows = list(csv.DictReader(open(csv_path)))
    trace = csv_path.replace("kernel_stats.csv", "kernel_trace.csv")
    by_grid = {}
    if os.path.exists(trace):
        for r in csv.DictReader(open(trace)):
            key = (r["Kernel_Name"], int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"]))
            d = int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
            n, t = by_grid.get(key, (0, 0))
            by_grid[key] = (n + 1, t + d)
    tot = sum(float(r["TotalDurationNs"]) for r in rows)
    lines = ["# rocprofv3 --kernel-trace --stats summary", "# command: " + command,
             "# %d kernels, %.3f ms total GPU time" % (len(rows), tot / 1e6),
             "%-90s %8s %12s %12s %7s" % ("kernel", "calls", "total_us", "avg_us", "pct")]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        name = r["Name"] if len(r["Name"]) <= 90 else r["Name"][:87] + "..."
        lines.append("%-90s %8d %12.1f %12.2f %7.2f" % (name, int(r["Calls"]), float(r["TotalDurationNs"]) / 1e3,
                                                        float(r["AverageNs"]) / 1e3, 100.0 * float(r["TotalDurationNs"]) / tot))
    if by_grid:
        lines += ["", "# by launch size (threads per launch), kernels above 1% of the time",
                  "%-90s %12s %8s %12s" % ("kernel", "threads", "calls", "avg_us")]
        big = {r["Name"] for r in rows if 100.0 * float(r["TotalDurationNs"]) / tot >= 1.0}
        for (name, g), (n, t) in sorted(by_grid.items(), key=lambda kv: (kv[0][0], -kv[0][1])):
            if name in big:
                short = name if len(name) <= 90 else name[:87] + "..."
                lines.append("%-90s %12d %8d %12.2f" % (short, g, n, t / n / 1e3))
    open(out_path, "w").write("\n".join(lines) + "\n")
    print("\n".join(lines[:25]))


def calibrate_copy():
    """An elementwise kernel that reads 1 GiB and writes 1 GiB (the scale of
    the HBM byte counters)."""
    import torch
    a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.mul(a, 1.0, out=b)
    torch.cuda.synchronize()
    del a, b


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--summarize-counters", metavar="DIR")
    ap.add_argument("--summarize-counters-c3", metavar="DIR")
    ap.add_argument("--sections", default="c1,mixed,heat,nodal,composite,batched,serving",
                    help="other rows to measure after the headline (comma list; '' for none)")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--no-autotune", action="store_true", help="default launch shapes, no tuning")
    ap.add_argument("--tune-cache", metavar="PATH",
                    help="launch-shape cache file (default: BXMG_TUNE_CACHE or ~/.cache/bxmg/tune.json; "
                         "'none' to time without a cache)")
    ap.add_argument("--no-headline", action="store_true", help="run only the sections (profiling)")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("CSV", "OUT", "COMMAND"),
                    help="write a text summary of a rocprofv3 kernel_stats.csv")
    ap.add_argument("--knobs", metavar="Z,R,L", help="planes per thread, buffer addressing (0/1), log2 tile-row cap")
    ap.add_argument("--cpu-leg", choices=("c3", "c4"), help=argparse.SUPPRESS)
    ap.add_argument("--cpu-problems", default="", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-out", help=argparse.SUPPRESS)
    args = ap.parse_args()

    if args.cpu_leg == "c3":
        cpu_leg_c3(args.cpu_out)
        return 0
    if args.cpu_leg == "c4":
        probs = [tuple(int(v) for v in x.split(",")) for x in args.cpu_problems.split(";") if x]
        cpu_leg_c4(probs, args.cpu_out)
        return 0
    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
        return 0
    if args.summarize_counters_c3:
        summarize_counters_c3(args.summarize_counters_c3)
        return 0
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return 0
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported (the batched and served forms "
              "shard by problem across GPUs)" % args.gpus, file=sys.stderr)
        return 3

    import tempfile
    secs = [x for x in args.sections.split(",") if x]
    cpu = not args.no_cpu_baseline and not args.no_headline
    tmpdir = tempfile.mkdtemp(prefix="bxmg_bench_")
    c3_proc = None
    if cpu and "mixed" in secs:
        # the oracle on the 512^3 problem takes minutes: in a child process
        # on its own core while the GPU rows run
        c3_proc = spawn_cpu_leg(["--cpu-leg", "c3", "--cpu-out", os.path.join(tmpdir, "c3.json")])

    import torch
    import paper_2403_12179_amd as bx
    from paper_2403_12179_amd import tuning
    import workloads as W

    if args.no_autotune:
        tune_cache = False
    elif args.tune_cache:
        tune_cache = False if args.tune_cache == "none" else tuning.TuneCache(args.tune_cache)
    else:
        tune_cache = None
    line = {}
    keep = {}
    if not args.no_headline:
        ba, f, phi, rhs = make_problem(bx, W)
        ctx = phi.ctx
        lib = bx.lib()
        tuned = None
        if args.knobs:
            # launch shapes given explicitly (e.g. for a profiled run)
            z, r, ly = (int(x) for x in args.knobs.split(","))
            tuned = {"planes_per_thread": z, "buffer_addressing": r, "tile_rows_log2_cap": ly, "source": "--knobs"}
        elif not args.no_autotune:
            # the project autotuner picks the launch shapes on this workload
            # (or takes them from its cache)
            tuned = tuning.tune_solve(bx.MultiFab(ba), rhs, cache=tune_cache, cycles=6)
            tuned.pop("format", None)
            z, r, ly = tuned["planes_per_thread"], tuned["buffer_addressing"], tuned["tile_rows_log2_cap"]
        else:
            z, r, ly = 4, 1, 8
        for param, value in ((0, z), (1, z), (2, r), (3, ly)):
            bx._lib.check(lib.bxmg_ctx_tune(ctx._h, param, value))
        for _ in range(args.warmup):
            phi.set_val(0.0)
            res = bx.mlmg_solve(phi, rhs, rel_tol=TOL)
            assert res.ok, res
        import ctypes as C
        bx._lib.check(lib.bxmg_profile_stage(ctx._h, 0))
        bx._lib.check(lib.bxmg_profile_read(ctx._h, None, None, 1))
        cycles = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for step in range(args.steps):
            phi.set_val(0.0)
            res = bx.mlmg_solve(phi, rhs, rel_tol=TOL)
            cycles.append(res.cycles)
            if step == 0:
                # the level-0 GS launches of the first timed step carry the
                # event brackets; the later steps run without them
                bx._lib.check(lib.bxmg_profile_stage(ctx._h, -1))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        launches = C.c_int64()
        gs_ms = C.c_double()
        bx._lib.check(lib.bxmg_profile_read(ctx._h, C.byref(launches), C.byref(gs_ms), 1))
        bx._lib.check(lib.bxmg_profile_stage(ctx._h, -1))
        if not res.ok:
            raise SystemExit("solve failed: %s" % res)
        if args.calibrate_copy:
            calibrate_copy()

        # the same solve with the 512 boxes kept as boxes (one launch per stage
        # over every box's tiles, ghost exchanges between boxes): the fused
        # multi-box launch without merging the level into one box; outside
        # the timed region, and not in the profiling runs
        boxes_kept = None
        if not args.calibrate_copy and not args.knobs:
            bx._lib.check(lib.bxmg_ctx_tune(ctx._h, 5, 0))
            phi.set_val(0.0)
            bx.mlmg_solve(phi, rhs, rel_tol=TOL)
            tb = []
            for _ in range(3):
                phi.set_val(0.0)
                torch.cuda.synchronize()
                tm = time.perf_counter()
                rb = bx.mlmg_solve(phi, rhs, rel_tol=TOL)
                torch.cuda.synchronize()
                tb.append(time.perf_counter() - tm)
            bx._lib.check(lib.bxmg_ctx_tune(ctx._h, 5, 1))
            boxes_kept = {"ms_per_solve": 1000.0 * min(tb), "cycles": rb.cycles, "ok": rb.ok,
                          "note": "the caller's 512 boxes as the execution boxes (knob 5 off): one launch per "
                                  "stage over all boxes' tiles, ghost exchanges between boxes"}
        ms_per_step = (t1 - t0) * 1000.0 / args.steps
        mean_cycles = sum(cycles) / len(cycles)
        value = N ** 3 * mean_cycles / (ms_per_step / 1000.0)
        gs_avg_ms = gs_ms.value / max(launches.value, 1)
        gs_bytes = GS_BYTES_PER_CELL * N ** 3
        achieved = gs_bytes / (gs_avg_ms / 1000.0) / 1e9
        key = shape_key(z, r, ly)
        traffic = traffic_from_counters(key)
        line = {
            "metric": "V-cycle cell-updates/s + HBM GB/s; batched solves/s & p99 latency at 1e-10",
            "value": value,
            "unit": "cell-updates/s",
            "n_gpus": 1,
            "steps": args.steps,
            "warmup": args.warmup,
            "ms_per_step": ms_per_step,
            "higher_is_better": True,
            "scaling": "weak",
            "vs_baseline": None,
            "dtype": "f64",
            "data": "synthetic",
            "config": {"workload": "poisson_dirichlet_256c_512x32c_fp64_vcycle22_tol1e-10", "domain": [N, N, N],
                       "boxes": len(ba), "box": [MAX_BOX] * 3, "nghost": 1, "levels": res.levels,
                       "cycles_per_solve": mean_cycles, "rhs": "uniform[-1,1] seed 2"},
            "vcycle_effective_GBps": BYTES_PER_CELL_CYCLE * N ** 3 * mean_cycles / (ms_per_step / 1000.0) / 1e9,
            "vcycle_model_bytes_per_cell": BYTES_PER_CELL_CYCLE,
            "solves_per_s": 1000.0 / ms_per_step,
            "autotuned_launch_shape": tuned,
            "final_rel_resid_inf": res.rel_resid_inf,
            "boxes_kept": boxes_kept,
            "roofline": {"bound": "hbm", "kernel": GS_KERNEL + " (level 0, one colour)", "achieved": achieved,
                         "peak": PEAK_GBPS, "unit": "GB/s", "frac": achieved / PEAK_GBPS, "traffic": traffic,
                         "algorithmic_bytes_per_launch": gs_bytes, "avg_launch_ms": gs_avg_ms,
                         "launches_timed": launches.value, "launch_shape": key},
        }
        del phi, rhs
        torch.cuda.empty_cache()
    if args.no_headline and args.calibrate_copy:
        calibrate_copy()
    for name in secs:
        print("bench: section %s" % name, file=sys.stderr, flush=True)
        if name == "c1":
            line["c1"], keep["c1"] = section_c1(bx, W)
        elif name == "mixed":
            line["mixed_precision"], keep["mixed"] = section_mixed(bx, W)
        elif name == "heat":
            line["heat"], keep["heat"] = section_heat(bx, W)
        elif name == "nodal":
            line["nodal"], keep["nodal"] = section_nodal(bx, W)
        elif name == "composite":
            line["composite"], keep["composite"] = section_composite(bx, W)
        elif name == "batched":
            line["batched"], keep["batched"], keep["edges"] = section_batched(bx, W, tune_cache=tune_cache)
        elif name == "serving":
            line["serving"], keep["serving"] = section_serving(bx, W, args.serving_requests)
        else:
            raise SystemExit("unknown section %r" % name)
    if cpu:
        print("bench: cpu leg", file=sys.stderr, flush=True)
        cb = cpu_baseline(f)
        cb.pop("seconds", None)
        line["cpu_baseline"] = cb
        from oracle import pyoracle as orc
        if "c1" in keep:
            c1, uo = cpu_c1()
            k = keep["c1"]
            c1["e_rel_gpu_vs_oracle"] = float(np.max(np.abs(k["u"] - uo)) / np.max(np.abs(uo)))
            line["c1"]["cpu_oracle"] = c1
        if "mixed" in keep:
            k = keep.pop("mixed")
            chk = {}
            for key, u in k["u"].items():
                chk[key] = oracle_check(orc, k["n"], (0, 0, 0), k["f"], k["beta"], u, TOL, solve_oracle=False,
                                        u_ref=None if key == "fp64" else k["u"]["fp64"])
            line["mixed_precision"]["error_vs_oracle"] = chk
            del k
        for row, cb_row in cpu_rows(orc, W, keep).items():
            line[row]["cpu_oracle"] = cb_row
        if "heat" in keep:
            k = keep.pop("heat")
            n, dt = k["n"], k["dt"]
            f = -(k["u_prev"] * (1.0 / dt) + k["src"])
            r = f - orc.apply_op((0, 0, 0), (n - 1,) * 3, (0, 0, 0), 1.0 / n, k["u"], None, 1.0 / dt)
            line["heat"]["error_vs_oracle"] = {
                "last_step_oracle_rel_resid_inf": float(np.max(np.abs(r)) / np.max(np.abs(f))), "tol": TOL}
            del k, f, r
        if "nodal" in keep:
            k = keep.pop("nodal")
            n = k["n"]
            r = (k["f"] - orc.nodal_apply((n, n, n), (0, 0, 0), 1.0 / n, k["u"]))[1:-1, 1:-1, 1:-1]
            line["nodal"]["error_vs_oracle"] = {
                "oracle_rel_resid_inf": float(np.max(np.abs(r)) / np.max(np.abs(k["f"][1:-1, 1:-1, 1:-1]))),
                "tol": TOL}
            del k, r
        if "composite" in keep:
            k = keep.pop("composite")
            n, fb = k["n"], k["fb"]
            fm = W.fine_mask(n, fb)
            cov = fm.reshape(n, 2, n, 2, n, 2).any(axis=(1, 3, 5))
            uf = np.where(fm, k["uf"], 0.0)
            Lc, Lf = orc.composite_apply(n, (0, 0, 0), k["cb"], fb, 1.0 / n, k["uc"], uf)
            fnorm = max(np.abs(k["fc"][~cov]).max(), np.abs(k["ff"][fm]).max())
            r = max(np.abs(k["fc"] - Lc)[~cov].max(), np.abs(k["ff"] - Lf)[fm].max())
            line["composite"]["error_vs_oracle"] = {"oracle_rel_resid_inf": float(r / fnorm), "tol": TOL}
            del k, uf, Lc, Lf
        if "batched" in keep:
            line["batched"]["error_vs_oracle"] = [
                dict(problem=s["q"], edge=s["e"], gpu_cycles=s["cycles"],
                     **oracle_check(orc, s["e"], s["per"], s["f"], s["beta"], s["u"], s["tol"]))
                for s in keep.pop("batched")]
            line["batched"]["cpu_oracle"] = cpu_c4(keep["edges"], tmpdir)
        if "serving" in keep:
            line["serving"]["error_vs_oracle"] = [
                dict(request=s["q"], edge=s["e"], lognormal_beta=s["beta"] is not None, gpu_cycles=s["cycles"],
                     **oracle_check(orc, s["e"], s["per"], s["f"], s["beta"], s["u"], s["tol"]))
                for s in keep.pop("serving")]
        if c3_proc is not None:
            try:
                c3_proc.wait(timeout=600)
            except subprocess.TimeoutExpired:
                c3_proc.kill()
            path = os.path.join(tmpdir, "c3.json")
            if c3_proc.returncode == 0 and os.path.exists(path):
                line["mixed_precision"]["cpu_oracle"] = json.load(open(path))
            else:
                line["mixed_precision"]["cpu_oracle"] = {"error": "oracle child failed or timed out"}
    elif c3_proc is not None:
        c3_proc.kill()
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
