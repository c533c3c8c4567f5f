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
KERNEL_SRC = os.path.join(ROOT, "paper_2403_12179_amd", "csrc", "bxmg_kernels.hip")
COUNTERS = os.path.join(ROOT, "profiles", "counters_gs_level0_256c512.json")
GS_KERNEL = "k_gs<double, 0>"
COPY_BYTES = 1 << 30

# Compulsory bytes per fine cell per V(2,2) cycle, FP64 (s = 8 B), per level
# l with N_l cells: 8 half-sweeps x 1.5 s N_l + residual/restriction
# (2 + 1/8) s N_l + zeroing the coarse guess s N_l / 8 + prolongation
# (2 + 1/8) s N_l = 16.375 s N_l; sum over levels 8/7 N_0; plus the level-0
# convergence residual 2 s N_0.
BYTES_PER_CELL_CYCLE = 8.0 * (16.375 * 8.0 / 7.0 + 2.0)
GS_BYTES_PER_CELL = 1.5 * 8.0  # one colour: read other colour, rhs of this colour, write this colour


def src_sha():
    return hashlib.sha256(open(KERNEL_SRC, "rb").read()).hexdigest()[:16]


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


def summarize_counters(d):
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

    def per_dispatch(rs, match, min_grid):
        vals = {}
        for disp, name, grid, value in rs:
            if match in name and grid >= min_grid:
                vals[disp] = vals.get(disp, 0.0) + float(value)
        return list(vals.values())

    level0_threads = (N ** 3) // 2 // 4  # one colour of level 0, >= 1 cell per thread
    out = {"kernel": GS_KERNEL, "workload": "256^3 in 512 boxes of 32^3, FP64", "kernel_src_sha": src_sha()}
    for counter, sub in (("FETCH_SIZE", "fetch"), ("WRITE_SIZE", "write")):
        rs = rows(sub, counter)
        gs = per_dispatch(rs, "k_gs", level0_threads)
        cp = per_dispatch(rs, "MulFunctor", 0)
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--summarize-counters", metavar="DIR")
    args = ap.parse_args()

    if args.summarize_counters:
        summarize_counters(args.summarize_counters)
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
    for _ in range(args.steps):
        phi.set_val(0.0)
        res = bx.mlmg_solve(phi, rhs, rel_tol=TOL)
        cycles.append(res.cycles)
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
        "final_rel_resid_inf": res.rel_resid_inf,
        "roofline": {"bound": "hbm", "kernel": GS_KERNEL + " (level 0, one colour)", "achieved": achieved,
                     "peak": PEAK_GBPS, "unit": "GB/s", "frac": achieved / PEAK_GBPS, "traffic": traffic,
                     "algorithmic_bytes_per_launch": gs_bytes, "avg_launch_ms": gs_avg_ms,
                     "launches_timed": launches.value},
    }
    if not args.no_cpu_baseline:
        cb = cpu_baseline(f)
        cb.pop("seconds", None)
        line["cpu_baseline"] = cb
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
