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
  mixed_precision : 512^3 variable coefficient in 512 boxes of 64^3, FP64
                    V-cycles vs FP32 V-cycles inside FP64 refinement
  batched         : 256 periodic problems of edges 32..128, batch engine vs
                    plain FP64 solves one at a time
  serving         : an open-loop request trace (200/s), continuous batching
                    vs plain FP64 first-come-first-served, p50/p99 latency

Other modes (not the benchmark line):
  --calibrate-copy          also run one elementwise kernel that reads and
                            writes 1 GiB (scales the counters)
  --summarize-counters DIR  turn two rocprofv3 --pmc outputs into
                            profiles/counters_gs_level0_256c512.json
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


def cpu_baseline(f, cycles=2):
    """The oracle, as it stands, on two V-cycles of the same problem."""
    from oracle import pyoracle as orc
    orc.build()
    boxes = orc.chop((0, 0, 0), (N - 1,) * 3, MAX_BOX)
    t0 = time.perf_counter()
    u, info = orc.solve((0, 0, 0), (N - 1,) * 3, (0, 0, 0), boxes, f, fixed_cycles=cycles)
    dt = time.perf_counter() - t0
    model, ncpu = cpu_info()
    return {"value": N ** 3 * cycles / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": "%d V(2,2) cycles of the 256^3 / 512-box FP64 problem incl. setup, 1 thread, %.1f s; host %s, "
                      "%s logical CPUs" % (cycles, dt, model, ncpu),
            "seconds": dt}


def traffic_from_counters():
    if not os.path.exists(COUNTERS):
        return None
    c = json.load(open(COUNTERS))
    if c.get("kernel_src_sha") != src_sha():
        return None
    return c.get("hbm_bytes_per_launch")


def summarize_counters(d, knobs=""):
    """Per-dispatch FETCH_SIZE / WRITE_SIZE (KiB) of the level-0 GS launches
    and of the 1 GiB elementwise calibration kernel, from the rocprofv3 --pmc
    databases under d/fetch and d/write; writes the committed summary."""
    import sqlite3

    def rows(sub, counter):
        dbs = glob.glob(os.path.join(d, sub, "**", "*.db"), recursive=True)
        if not dbs:
            raise SystemExit("no rocprofv3 database under %s" % os.path.join(d, sub))
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
           "commands": ["cd /tmp && timeout -s KILL 300 rocprofv3 --pmc %s -d $REPO/%s/%s -o c2 -- python3 "
                        "$REPO/bench.py --steps 1 --warmup 0 --no-cpu-baseline --sections '' --knobs %s "
                        "--calibrate-copy" % (c, os.path.normpath(d), sub, knobs or "<autotuned>")
                        for c, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write"))]}
    for counter, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        rs = rows(sub, counter)
        gs = per_dispatch(rs, GS_MATCH, True)
        cp = per_dispatch(rs, "MulFunctor", False)
        if not gs or not cp:
            raise SystemExit("missing dispatches for %s (gs %d, copy %d)" % (counter, len(gs), len(cp)))
        out[counter.lower() + "_kib_per_launch"] = sum(gs) / len(gs)
        out[counter.lower() + "_copy_kib"] = max(cp)
        out[counter.lower() + "_launches"] = len(gs)
    # the calibration kernel reads 1 GiB and writes 1 GiB
    fscale = (COPY_BYTES / 1024.0) / out["fetch_size_copy_kib"]
    wscale = (COPY_BYTES / 1024.0) / out["write_size_copy_kib"]
    out["fetch_scale"], out["write_scale"] = fscale, wscale
    out["hbm_bytes_per_launch"] = 1024.0 * (out["fetch_size_kib_per_launch"] * fscale +
                                            out["write_size_kib_per_launch"] * wscale)
    out["algorithmic_bytes_per_launch"] = GS_BYTES_PER_CELL * N ** 3
    os.makedirs(os.path.dirname(COUNTERS), exist_ok=True)
    json.dump(out, open(COUNTERS, "w"), indent=1)
    print(json.dumps(out, indent=1))


# ------------------------------------------------------------ other rows
def section_mixed(bx, W, reps=3):
    """512^3 in 512 boxes of 64^3, Dirichlet, beta = exp(g) (g: 3 box-filter
    passes, std 1), f ~ U[-1,1]: FP64 V-cycles vs FP32 V-cycles inside FP64
    refinement, both to 1e-10; error of the mixed solution against the FP64
    one.  Fields drawn on the device (seeds 3 and 33)."""
    import torch
    n = 512
    ba = bx.BoxArray.chop((0, 0, 0), (n - 1,) * 3, 64, bc=(bx.DIRICHLET0,) * 3)
    f = W.uniform_rhs_device((n, n, n), 3)
    beta = W.smooth_gaussian_beta_device((n, n, n), 33)
    rhs = bx.MultiFab(ba).set_val(0.0).from_tensor(f)
    bmf = bx.MultiFab(ba).set_val(1.0).from_tensor(beta)
    del f, beta
    phi = bx.MultiFab(ba)
    out = {"workload": "poisson_varcoef_512c_512x64c_dirichlet_tol1e-10", "boxes": len(ba)}
    sols = {}
    for prec in (0, 1):
        times, res = [], None
        for r in range(reps + 1):
            phi.set_val(0.0)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = bx.mlmg_solve(phi, rhs, bmf, rel_tol=TOL, precision=prec)
            torch.cuda.synchronize()
            if r > 0:
                times.append(time.perf_counter() - t0)
            if not res.ok:
                raise SystemExit("mixed-precision section: solve failed: %s" % res)
        key = "fp64" if prec == 0 else "fp32_in_fp64_ir"
        ms = 1000.0 * min(times)
        out[key] = {"ms_per_solve": ms, "solves_per_s": 1000.0 / ms, "cycles": res.cycles,
                    "final_rel_resid_inf": res.rel_resid_inf}
        sols[prec] = phi.slab.clone()
    d = (sols[1] - sols[0]).abs().max().item() / sols[0].abs().max().item()
    out["mixed_vs_fp64_rel_max_diff"] = d
    out["speedup_mixed_over_fp64"] = out["fp64"]["ms_per_solve"] / out["fp32_in_fp64_ir"]["ms_per_solve"]
    del sols, phi, rhs, bmf
    torch.cuda.empty_cache()
    return out


def make_batch_problems(bx, W, nprob=256, seed=4):
    edges = W.batch_edges(nprob, seed)
    probs = []
    for p, e in enumerate(edges):
        ba = bx.BoxArray.chop((0, 0, 0), (e - 1,) * 3, 32, bc=(bx.PERIODIC,) * 3)
        f = W.uniform_rhs_device((e, e, e), 4000 + p, mean_zero=True)
        probs.append(dict(e=e, ba=ba, phi=bx.MultiFab(ba).set_val(0.0), rhs=bx.MultiFab(ba).set_val(0.0).from_tensor(f)))
    return probs


def section_batched(bx, W):
    """256 periodic problems, edges uniform over {32,48,64,96,128} (seed 4),
    max box 32, f ~ U[-1,1] minus its mean (seed 4000+p): the batch engine
    (FP32 V-cycles inside FP64 refinement, one launch per stage over all
    problems, hipGraph) vs plain FP64 solves one at a time, both to 1e-10."""
    import torch
    probs = make_batch_problems(bx, W)
    cells = sum(p["e"] ** 3 for p in probs)
    ctx = probs[0]["phi"].ctx
    out = {"workload": "batch_256_periodic_edges_32-128_maxbox32_tol1e-10", "problems": len(probs),
           "cells": cells, "boxes": sum(len(p["ba"]) for p in probs)}
    # warm-up of both paths on a few problems (builds, graph capture)
    b = bx.Batch(ctx, 12 << 30, 512, precision=1)
    for p in probs[:4]:
        b.add(p["phi"], p["rhs"], rel_tol=TOL)
    b.run(2)
    for p in probs[:4]:
        p["phi"].set_val(0.0)
        bx.mlmg_solve(p["phi"], p["rhs"], rel_tol=TOL)
    for p in probs:
        p["phi"].set_val(0.0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for p in probs:
        if b.add(p["phi"], p["rhs"], rel_tol=TOL) is None:
            raise SystemExit("batched section: arena too small")
    t_add = time.perf_counter() - t0
    done = b.run(2)
    t_batch = time.perf_counter() - t0
    ok = all(r.ok for _, r in done) and len(done) == len(probs)
    cyc = [r.cycles for _, r in done]
    worst = max(r.rel_resid_inf for _, r in done)
    b.close()
    # plain FP64, one problem after another
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
    del probs
    torch.cuda.empty_cache()
    return out


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
    return reqs


def latency_stats(lat, t_first, t_last):
    import numpy as np
    a = np.asarray(lat)
    return {"p50_ms": 1000.0 * float(np.percentile(a, 50)), "p99_ms": 1000.0 * float(np.percentile(a, 99)),
            "mean_ms": 1000.0 * float(a.mean()), "solves_per_s": len(a) / (t_last - t_first)}


def section_serving(bx, W, nreq):
    """Open-loop trace: exponential inter-arrivals of mean 5 ms (seed 5),
    edge = clamp(16 round(exp(U(ln 32, ln 256)) / 16), 32, 256), Dirichlet,
    beta constant or lognormal (1/2 each), tol 10^U(-10,-8), f ~ U[-1,1]
    (seed 5000+q); inputs staged in HBM before the clock starts.  Served:
    continuous batching (FP32 V-cycles inside FP64 refinement, admission by
    footprint, one cycle per pump); baseline: plain FP64 solves one at a
    time in arrival order.  Latency = completion - arrival."""
    import torch
    trace = W.serving_trace(nreq, 5)
    reqs = stage_requests(bx, W, trace)
    ctx = reqs[0]["phi"].ctx
    torch.cuda.synchronize()
    out = {"workload": "serving_trace_%d_req_200per_s_edges_32-256_dirichlet_tol1e-8..1e-10" % nreq,
           "requests": nreq, "mean_cells": sum(r["q"]["edge"] ** 3 for r in reqs) / nreq,
           "lognormal_share": sum(r["q"]["kind"] for r in reqs) / nreq}
    srv = bx.Server(ctx, 24 << 30, max_problems=512, chunk=2, precision=1)
    # warm-up: one request of each kind through the server
    for r in reqs[:2]:
        srv.submit(-1, r["phi"], r["rhs"], r["beta"], r["q"]["tol"])
    while not srv.idle():
        srv.pump()
    for r in reqs:
        r["phi"].set_val(0.0)
    torch.cuda.synchronize()
    lat, ok, nxt = {}, True, 0
    t0 = time.perf_counter()
    while len(lat) + len(srv.rejected) < nreq:
        now = time.perf_counter() - t0
        while nxt < nreq and reqs[nxt]["q"]["t"] <= now:
            r = reqs[nxt]
            srv.submit(nxt, r["phi"], r["rhs"], r["beta"], r["q"]["tol"])
            nxt += 1
        if srv.idle():
            continue
        for tag, res, t_done in srv.pump():
            lat[tag] = (t_done - t0) - reqs[tag]["q"]["t"]
            ok = ok and res.ok and res.rel_resid_inf <= reqs[tag]["q"]["tol"]
    t_end = max(lat[k] + reqs[k]["q"]["t"] for k in lat)
    out["served"] = latency_stats(list(lat.values()), reqs[0]["q"]["t"], t_end)
    out["served"]["ok"] = ok and not srv.rejected
    srv.close()
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--summarize-counters", metavar="DIR")
    ap.add_argument("--knobs-used", default="",
                    help="launch shape the counter runs used (recorded with --summarize-counters)")
    ap.add_argument("--sections", default="mixed,batched,serving",
                    help="other rows to measure after the headline (comma list; '' for none)")
    ap.add_argument("--serving-requests", type=int, default=400)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("CSV", "OUT", "COMMAND"),
                    help="write a text summary of a rocprofv3 kernel_stats.csv")
    ap.add_argument("--knobs", metavar="Z,R,L", help="planes per thread, buffer addressing (0/1), log2 tile-row cap")
    args = ap.parse_args()

    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.knobs_used)
        return 0
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return 0
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported (the batched and served forms "
              "shard by problem across GPUs)" % args.gpus, file=sys.stderr)
        return 3

    import torch
    import paper_2403_12179_amd as bx
    import workloads as W

    ba, f, phi, rhs = make_problem(bx, W)
    ctx = phi.ctx
    lib = bx.lib()
    tuned = None
    if args.knobs:
        # launch shapes given explicitly (e.g. the autotuner's choice of an
        # earlier run, so that a profiled run times exactly those launches)
        z, r, ly = (int(x) for x in args.knobs.split(","))
        for param, value in ((0, z), (1, z), (2, r), (3, ly)):
            bx._lib.check(lib.bxmg_ctx_tune(ctx._h, param, value))
        tuned = {"planes_per_thread": z, "buffer_addressing": r, "tile_rows_log2_cap": ly, "source": "--knobs"}
    elif not args.no_autotune:
        # the project autotuner picks the launch shapes on this workload
        tuned = bx.autotune(bx.MultiFab(ba), rhs, cycles=6)
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
            # the level-0 GS launches of the first timed step carry the event
            # brackets; the later steps run without them
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
        # an elementwise kernel that reads 1 GiB and writes 1 GiB
        a = torch.empty(COPY_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        torch.mul(a, 1.0, out=b)
        torch.cuda.synchronize()

    ms_per_step = (t1 - t0) * 1000.0 / args.steps
    mean_cycles = sum(cycles) / len(cycles)
    value = N ** 3 * mean_cycles / (ms_per_step / 1000.0)
    gs_avg_ms = gs_ms.value / max(launches.value, 1)
    gs_bytes = GS_BYTES_PER_CELL * N ** 3
    achieved = gs_bytes / (gs_avg_ms / 1000.0) / 1e9
    traffic = traffic_from_counters()
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
        "roofline": {"bound": "hbm", "kernel": GS_KERNEL + " (level 0, one colour)", "achieved": achieved,
                     "peak": PEAK_GBPS, "unit": "GB/s", "frac": achieved / PEAK_GBPS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": gs_bytes, "avg_launch_ms": gs_avg_ms,
                     "launches_timed": launches.value},
    }
    del phi, rhs
    torch.cuda.empty_cache()
    secs = [x for x in args.sections.split(",") if x]
    for name in secs:
        print("bench: section %s" % name, file=sys.stderr, flush=True)
        if name == "mixed":
            line["mixed_precision"] = section_mixed(bx, W)
        elif name == "batched":
            line["batched"] = section_batched(bx, W)
        elif name == "serving":
            line["serving"] = section_serving(bx, W, args.serving_requests)
        else:
            raise SystemExit("unknown section %r" % name)
    if not args.no_cpu_baseline:
        cb = cpu_baseline(f)
        cb.pop("seconds", None)
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
