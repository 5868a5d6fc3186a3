"""Benchmark: cell-updates/s of the per-cycle grid update on one MI355X.

Workload: 1000 x 1000 cells + 50-cell PML (1050 x 1050 = 1,102,500 cells),
two materials with pressure-dependent strength, R = 50 cells, 15 km/s,
plain FP64 (the scale configuration). One step = one full cycle of the hot
path over the whole grid. W warm-up cycles, then K timed cycles, bracketed by
stream synchronisation; inputs are resident in HBM throughout.

Prints one JSON line. `roofline` reports the whole cycle's algorithmic bytes
per cell-update (state read + written once, PML auxiliaries in layer cells)
over the measured device time, against the 8 TB/s HBM peak.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def algorithmic_bytes_per_cell(pb) -> float:
    """State read + written once per cycle (FP64): rho, I, f per material,
    three deviatoric stresses when strength is on, two node velocities per
    cell; plus the PML auxiliaries (3 cell + 4 node values per damped
    direction, read + written; corner cells count twice; the reference
    density and the sink read / written once) averaged over all cells."""
    g = pb.grid
    nmat = g.nmat
    strength = any(m.strength for m in pb.mats[:nmat])
    per_cell = 2 + nmat + (3 if strength else 0) + 2
    state = 2 * 8 * per_cell
    NR, NZ = g.NR, g.NZ
    ncell = NR * NZ
    bottom = g.pml_b * NR
    right = g.pml_r * NZ
    union = bottom + g.n_z * g.pml_r
    aux = 2 * 8 * 7 * (bottom + right) + 8 * 3 * union  # rho_ref read, msink r+w
    return state + aux / ncell if pb.pml.enabled else state


def cpu_baseline(pb, budget_s=12.0):
    from oracle import oracle as O
    from oracle.oracle import Oracle
    threads = O.set_threads(os.cpu_count() or 1)
    o = Oracle(pb)
    cells = pb.grid.ncells
    n, t0 = 0, time.perf_counter()
    while True:
        o.step(5)
        n += 5
        el = time.perf_counter() - t0
        if el >= budget_s or n >= 2000:
            break
    return {"value": cells * n / el, "unit": "cell-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} cycles of the same 1050x1050 workload from its initial state"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--tune", type=int, default=2, metavar="K",
                    help="time every tile shape over K cycles during warm-up and keep the fastest (0: off)")
    ap.add_argument("--variant", type=int, default=-1, help="force a tile shape (disables --tune)")
    ap.add_argument("--grid", type=int, default=0, help="workgroups per launch with --variant (0: one per tile)")
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB mebibytes (3 launches) and exit; "
                         "profiling it gives the HBM counter scale factors")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on exactly one GPU; --gpus must be 1"}))
        sys.exit(2)
    import torch
    if args.copy_calibrate:
        n = args.copy_calibrate * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8}), flush=True)
        return
    from paper_2403_04267_amd import inputs
    from paper_2403_04267_amd.salec import Salec

    pb = inputs.config_scale()
    ctx = Salec(pb, "cuda:0")
    if args.variant >= 0:
        ctx.set_schedule(args.variant, args.grid)
    elif args.tune > 0:
        ctx.tune(args.tune)  # advances the run; counted as warm-up
    if args.warmup:
        ctx.step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(args.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev_ms = ctx.last_step_ms()
    cells = pb.grid.ncells
    cu = cells * args.steps
    value = cu / (dev_ms / 1e3)
    bpc = algorithmic_bytes_per_cell(pb)
    achieved = bpc * value / 1e9
    d = ctx.diag()
    out = {
        "metric": "cell-updates/s", "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": dev_ms / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "impact-1050x1050-2mat-strength-pml50-fp64", "cells": cells,
                   "cycles": args.steps, "precision": "fp64"},
        "wall_ms_per_step": wall * 1e3 / args.steps,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_cell_update": bpc, "scope": "whole cycle"},
        "sim": {"t": d["t"], "dt": d["dt"], "cycle": d["cycle"]},
        "schedule": ctx.schedule(),
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(pb)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
