"""Benchmark: cell-updates/s of the per-cycle grid update on one MI355X.

Headline workload: 1000 x 1000 cells + 50-cell PML (1050 x 1050 =
1,102,500 cells), two materials with pressure-dependent strength, R = 50
cells, 15 km/s, plain FP64. One step = one full cycle of the hot path over
the whole grid (one launch of the cycle kernel). The tile shape is chosen by
the library's tuner during warm-up; W warm-up cycles, then K timed cycles
bracketed by stream synchronisation, inputs resident in HBM throughout. The
device time comes from HIP events the library records on its own stream
around the replayed graphs (the timed cycles run as 5 consecutive calls; the
median call is reported beside the total). Right after them, the cycle
kernel's own mean duration is measured over further cycles launched between
HIP events; the roofline uses it.

Also measured (the "extensions" object; skipped with --headline-only):
  mixed_scale    the same workload in the mixed-precision mode (with its error
                 against a plain-FP64 GPU run: conserved densities at cycle 200,
                 crater level at cycle 2000, also for a run started in FP64
                 and handed to the mixed mode at cycle 40; likewise for
                 mixed_large, and the per-member crater level of 64 sampled
                 members for batched_mixed)
  mixed_large    4000 x 4000 + 100 PML (4100^2 cells), mixed precision
  batched_fp64   256 seeded uneven impacts (sides 200-800), plain FP64
  batched_mixed  1024 seeded uneven impacts (sides 200-1200), mixed
  layered_fp64   the 1050^2 workload as a two-layer target under gravity
                 (400 m cells, lithostatic initial pressure), plain FP64
  paper_layout_fp64  the impact on Table 2's stretched 512 x 532 grid (two
                 layers, gravity), plain FP64
  three_layer_fp64   the 1050^2 workload as Sec. 4's three-layer target
                 (calcite, granite, dunite; 400 m cells, gravity), plain FP64
  paper_layers_fp64  Sec. 4's three-layer setting on Table 2's grid, FP64
  three_layer_pm_fp64  the three-layer 1050^2 target with the per-material
                 closure (each material's own density and energy), FP64
  pml_payoff     the same small impact with a PML, with plain walls and on a
                 10x larger domain, each to the same time (interior error,
                 reflected energy, crater geometry, device time)
  pml_payoff_table2  the same comparison on Table 2's grid with Sec. 4's three
                 layers and gravity, to 30 s, against ~200 km longer extension
                 zones; Sec. 3's layers and the stress-damping extension
  paper_layers_damage_fp64  paper_layers_fp64 with Table 1's damage and
                 block-model constants (the damage kernels), FP64
  damage_table2  the PML run of that setting against the reference to 60 s:
                 crater and crust-base profile differences, crust-base uplift
Each but the last three is init + tune + warm-up, then a short timed run.

Prints one JSON line. `roofline` is the cycle kernel's algorithmic HBM
bytes per launch (state read and written once, PML auxiliaries) over the
cycle kernel's mean duration, against the 8 TB/s HBM peak and against the
device-to-device copy rate measured in the same run; `traffic` is the
kernel's measured HBM bytes per launch (committed counter summary) over the
same time, in GB/s, or null when the kernel sources or the schedule differ
from those the counters were taken with.
"""
import argparse
import dataclasses
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_cycle_fp64_1050x1050_hbm_traffic.json")


def kernel_sources_sha() -> str:
    """Hash of the sources that define the cycle kernel's memory traffic."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2403_04267_amd", "csrc")
    for name in ("salec_cycle.hpp", "salec_device.hpp", "salec_cycle.hip", "salec_cycle_f64.hip"):
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def algorithmic_bytes_per_cell(pb) -> float:
    """State read + written once per cycle (FP64): rho, I, f per material,
    three deviatoric stresses when strength is on, two node velocities per
    cell; plus the PML auxiliaries (3 cell + 4 node values per damped
    direction, read + written; corner cells count twice; the reference
    density read and the sink read + written) averaged over all cells.
    Mixed precision: stress and velocity are 4-byte values. The per-material
    closure adds each material's partial density and specific energy; damage
    adds D and the vibration speed (FP64)."""
    g = pb.grid
    nmat = g.nmat
    strength = any(m.strength for m in pb.mats[:nmat])
    damage = any(int(getattr(m, "damage", 0)) for m in pb.mats[:nmat])
    wide = 8 * (2 + nmat + (2 * nmat if g.closure else 0) + (2 if damage else 0))
    narrow = (8 if pb.precision == "fp64" else 4) * ((3 if strength else 0) + 2)
    state = 2 * (wide + narrow)
    NR, NZ = g.NR, g.NZ
    ncell = NR * NZ
    bottom = g.pml_b * NR
    right = g.pml_r * NZ
    union = bottom + g.n_z * g.pml_r
    aux = 2 * 8 * 7 * (bottom + right) + 8 * 3 * union
    return state + aux / ncell if pb.pml.enabled else state


def traffic_per_launch(schedule, workload="scale"):
    """Measured HBM bytes per cycle-kernel launch (FETCH_SIZE + WRITE_SIZE,
    each scaled by the reading for a plain copy of known size), if the
    recorded counters were taken from the current kernel sources, the
    workload and the schedule being timed."""
    try:
        with open(TRAFFIC_FILE) as fh:
            recs = json.load(fh).get("records", [])
    except (OSError, ValueError, AttributeError):
        return None
    sha = kernel_sources_sha()
    for rec in recs:
        want = rec.get("schedule", {})
        if rec.get("workload", "scale") != workload:
            continue
        if rec.get("kernel_sources_sha256") == sha and all(schedule.get(k) == v for k, v in want.items()):
            return rec.get("hbm_bytes_per_launch")
    return None


# VALU issue peak of the chip: 256 CUs x 4 SIMDs, one wave64 FP64/FP32 VALU
# instruction per SIMD every 4 cycles at 2.4 GHz, 64 lanes each (the FMA of
# the published 78.6 TFLOP/s FP64 vector peak counts as 2 of its flops).
VALU_LANE_OPS_PEAK = 256 * 4 * 2.4e9 / 4 * 64


def valu_per_launch(schedule, workload="scale"):
    """VALU instructions per cycle-kernel launch (SQ_INSTS_VALU, wave64
    instructions, recorded with the traffic records, one record or a list),
    if taken from the current kernel sources and the schedule being timed."""
    try:
        with open(TRAFFIC_FILE) as fh:
            recs = json.load(fh).get("valu")
    except (OSError, ValueError, AttributeError):
        return None
    if isinstance(recs, dict):
        recs = [recs]
    sha = kernel_sources_sha()
    for rec in recs or []:
        if rec.get("kernel_sources_sha256") != sha or rec.get("workload", "scale") != workload:
            continue
        if all(schedule.get(k) == v for k, v in rec.get("schedule", {}).items()):
            return rec.get("sq_insts_valu_per_dispatch")
    return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def host_threads() -> int:
    """The host cores this process may use (the OpenMP limit if one is set,
    else the CPU affinity set)."""
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        return int(env)
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:
        return os.cpu_count() or 1


def cpu_baseline(pb, budget_s=12.0, budget_1_s=8.0):
    """The oracle as it stands (plain FP64 C, -O2, OpenMP over rows) on the
    same workload from its initial state: all usable host cores for about
    budget_s seconds, then one thread for about budget_1_s seconds."""
    from oracle import oracle as O
    from oracle.oracle import Oracle

    def timed(threads, budget):
        used = O.set_threads(threads)
        o = Oracle(pb)
        n, t0 = 0, time.perf_counter()
        while True:
            o.step(5 if threads > 1 else 1)
            n += 5 if threads > 1 else 1
            el = time.perf_counter() - t0
            if el >= budget or n >= 2000:
                break
        return pb.grid.ncells * n / el, used, n, el

    rate, used, n, el = timed(host_threads(), budget_s)
    rate1, _, n1, el1 = timed(1, budget_1_s)
    O.set_threads(host_threads())
    return {"value": rate, "unit": "cell-updates/s", "cores": used, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{n} cycles of the same 1050x1050 FP64 workload from its initial state on {used} threads "
                      f"({el:.1f} s); {n1} cycles on one thread ({el1:.1f} s)",
            "one_thread": {"value": rate1, "unit": "cell-updates/s", "cores": 1, "cycles": n1, "seconds": el1},
            "parallel_speedup": rate / rate1}


def copy_bandwidth(mib=2048, reps=5):
    """Device-to-device copy rate (bytes read + written per second, GB/s):
    the attainable HBM bandwidth on this device, next to the 8 TB/s peak."""
    import torch
    n = mib * (1 << 20)
    src = torch.ones(n, dtype=torch.uint8, device="cuda:0")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    best = float("inf")
    for _ in range(reps):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    del src, dst
    torch.cuda.empty_cache()
    return 2 * n / (best / 1e3) / 1e9


def run(problems, steps, warmup, tune, variant=-1, grid=0, parts=1):
    """Times `steps` cycles of a context in `parts` consecutive calls; returns
    (cell-updates/s over all of them, ms per cycle, schedule, context, rate
    of each call)."""
    from paper_2403_04267_amd.salec import Salec
    ctx = Salec(problems, "cuda:0")
    if variant >= 0:
        ctx.set_schedule(variant, grid)
    elif tune > 0:
        ctx.tune(tune)
    if warmup:
        ctx.step(warmup)
    probs = problems if isinstance(problems, list) else [problems]
    cells = sum(p.grid.ncells for p in probs)
    ms, rates, done = 0.0, [], 0
    for q in range(parts):
        n = steps * (q + 1) // parts - done
        ctx.step(n)
        m = ctx.last_step_ms()
        ms += m
        rates.append(cells * n / (m / 1e3))
        done += n
    return cells * steps / (ms / 1e3), ms / steps, ctx.schedule(), ctx, rates


def extension(name, problems, steps, warmup, tune, fp64_rate=None):
    import torch
    t0 = time.perf_counter()
    rate, ms, sch, ctx, _ = run(problems, steps, warmup, tune)
    probs = problems if isinstance(problems, list) else [problems]
    out = {"value": rate, "unit": "cell-updates/s", "ms_per_cycle": ms, "cycles": steps,
           "instances": len(probs), "cells": sum(p.grid.ncells for p in probs),
           "precision": probs[0].precision, "schedule": {k: sch[k] for k in ("tile_r", "tile_z", "threads")},
           "bytes_per_cell_update": sum(algorithmic_bytes_per_cell(p) * p.grid.ncells for p in probs) /
           sum(p.grid.ncells for p in probs)}
    out["hbm_frac"] = out["bytes_per_cell_update"] * rate / 1e9 / HBM_PEAK_GBS
    if fp64_rate:
        out["speedup_vs_fp64"] = rate / fp64_rate
    del ctx
    torch.cuda.empty_cache()
    out["wall_s"] = time.perf_counter() - t0
    print(f"[bench] {name}: {rate:.3e} cu/s, {ms * 1e3:.1f} us/cycle", file=sys.stderr, flush=True)
    return out


def mixed_accuracy(pb64, early=200, late=2000, hand=40):
    """The mixed mode against the plain-FP64 GPU run of the same problem from
    the same start, per field: relative L2 of rho, p, I, v_r, v_z over all
    cells (nodes) and over those holding matter, the conserved densities,
    crater depth and radius (cells), at cycles `early` and `late`. Beside it
    the FP64 conditioning floor measured the same way (an FP64 run whose
    initial velocities are one ulp up), and the hand-over path: FP64 for the
    first `hand` cycles, then the mixed mode (fields, PML auxiliaries and
    clock handed over between contexts)."""
    import numpy as np
    import torch
    from paper_2403_04267_amd.salec import Salec
    from tests.crater import per_field
    a, b, p = Salec(pb64), Salec(pb64.replace(precision="mixed")), Salec(pb64)
    F0 = p.fields(eos=False)
    p.set_fields(F0["rho"], F0["I"], F0["f"], np.nextafter(F0["v"], np.inf), F0["s"])
    del F0
    for x in (a, b, p):
        x.step(hand)
    c = Salec(pb64.replace(precision="mixed"))
    c.continue_from(a)
    sj = pb64.scene.surface_j
    out = {"against": "plain-FP64 GPU run (bit for bit the oracle at every size the oracle runs)",
           "hand_over_cycle": hand}
    done = hand
    for cyc in (early, late):
        for x in (a, b, c, p):
            x.step(cyc - done)
        done = cyc
        Fa = a.fields()
        out[str(cyc)] = {name: per_field(x.fields(), Fa, pb64.grid, sj)
                         for name, x in (("mixed", b), ("fp64_start", c), ("fp64_floor", p))}
        del Fa
    del a, b, c, p
    torch.cuda.empty_cache()
    return out


def handover(ext, fp64_rate, cycles, hand=40):
    """The rate of the path that meets the accuracy bar: the first `hand`
    cycles in FP64, the rest of the workload's cycles in the mixed mode."""
    rm = ext["value"]
    rate = cycles / (hand / fp64_rate + (cycles - hand) / rm)
    ext["value_plain_mixed"] = rm
    ext["value"] = rate
    ext["path"] = f"FP64 for {hand} cycles, then mixed, over {cycles} cycles"
    ext["speedup_vs_fp64"] = rate / fp64_rate


def ensemble_accuracy(cycles=1000):
    """64 members sampled (every 16th) from the 1024-member ensemble, mixed
    against plain FP64 after `cycles` cycles: per-member difference of the
    crater level on the axis, in cells."""
    import numpy as np
    import torch
    from paper_2403_04267_amd import inputs
    from paper_2403_04267_amd.salec import Salec
    from tests.crater import crater_depth
    sample = inputs.ensemble(4267, 1024, 200, 1200)[::16]
    a, b = Salec(sample), Salec([p.replace(precision="mixed") for p in sample])
    a.step(cycles)
    b.step(cycles)
    d = []
    for k, pb in enumerate(sample):
        sj = pb.scene.surface_j
        d.append(abs(crater_depth(a.fields(eos=False, k=k)["f"], pb.grid, sj) -
                     crater_depth(b.fields(eos=False, k=k)["f"], pb.grid, sj)) / pb.grid.dz)
    del a, b
    torch.cuda.empty_cache()
    d = np.array(d)
    return {"against": "plain-FP64 GPU batch", "members": len(d), "cycles": cycles,
            "crater_level_diff_cells": {"max": float(d.max()), "mean": float(d.mean()),
                                        "median": float(np.median(d)), "within_1": int((d <= 1).sum())}}


def pml_payoff():
    """The PML payoff study: the 100x100 hydrodynamic impact (R = 10 cells,
    10 km/s) with a 20-cell PML, with plain walls, and on a 1000x1000 domain,
    each to t = 0.08 s; interior differences against the large domain,
    crater geometry, cells and device time."""
    from paper_2403_04267_amd.pml_study import Setup, run
    t0 = time.perf_counter()
    r = run(Setup())
    r["wall_s"] = time.perf_counter() - t0
    print(f"[bench] pml payoff: pml {r['pml']['err_vs_big']}, bare {r['bare']['err_vs_big']}",
          file=sys.stderr, flush=True)
    return r


def pml_payoff_table2():
    """The PML comparison in the paper's setting: Table 2's grid with Sec. 4's
    three layers (calcite, granite, dunite; gravity) with its PML, with plain
    walls, and with extension zones ~200 km longer, each to 30 s (the shock
    has turned at the bottom boundary); once with Sec. 3's layers and once
    with the extension that also relaxes the deviatoric stress in them."""
    from paper_2403_04267_amd.pml_study import PaperSetup, paper_run
    t0 = time.perf_counter()
    r = paper_run(PaperSetup(t_end=30.0))
    d = paper_run(PaperSetup(t_end=30.0, damp_stress=1))
    r["pml_damp_stress"] = d["pml"]
    r["wall_s"] = time.perf_counter() - t0
    print(f"[bench] pml payoff (Table 2, far field): pml {r['pml']['err_vs_ref_far']}, with stress damping "
          f"{d['pml']['err_vs_ref_far']}, bare {r['bare']['err_vs_ref_far']}", file=sys.stderr, flush=True)
    return r


def paper_layers_damage():
    """Sec. 4's three-layer setting on Table 2's grid with Table 1's damage
    and block-model constants on every layer (block size the projectile
    radius)."""
    from paper_2403_04267_amd import inputs
    pb = inputs.config_paper_layers()
    h = pb.scene.radius
    keys = ("calcite", "granite", "dunite")
    return pb.replace(mats=[inputs.with_damage(m, **inputs.TABLE1_DAMAGE[k], af_h=h) for m, k in zip(pb.mats, keys)],
                      name="paper-layers-damage")


def damage_table2():
    """The PML run of Sec. 4's three-layer setting with damage and the block
    model against the reference with ~200 km longer extension zones, at 60 s:
    crater surface and crust base profile differences, crust-base uplift and
    crater depth of both, the time and cycles each run reached."""
    from paper_2403_04267_amd.pml_study import paper_profiles
    t0 = time.perf_counter()
    r = paper_profiles(times=(60.0,), damage=1)
    r["wall_s"] = time.perf_counter() - t0
    p = r["60s"]["pml"]
    print(f"[bench] damage, Table 2, 60 s: crater median {p['crater']['median_m']:.0f} m, crust base max "
          f"{p['moho']['max_m']:.0f} m", file=sys.stderr, flush=True)
    return r


WORKLOADS = ("scale", "large", "ens256", "ens1024", "paper_layers_damage", "three_layer", "three_layer_pm")


def workload(name):
    """The headline workload (scale) or one of the workloads the extensions
    time, by name (for profiling runs)."""
    from paper_2403_04267_amd import inputs
    return {"scale": inputs.config_scale, "large": lambda: inputs.config_large("mixed"),
            "ens256": lambda: inputs.ensemble(2403, 256, 200, 800),
            "ens1024": lambda: inputs.ensemble(4267, 1024, 200, 1200, precision="mixed"),
            "paper_layers_damage": paper_layers_damage,
            "three_layer": lambda: inputs.three_layer_impact(1000, 50, 50, 15e3, 7, 75, name="three"),
            "three_layer_pm": lambda: three_layer_pm(inputs)}[name]()


def three_layer_pm(inputs):
    """The three-layer 1050^2 target under the per-material closure."""
    three = inputs.three_layer_impact(1000, 50, 50, 15e3, 7, 75, name="three-pm")
    return three.replace(grid=dataclasses.replace(three.grid, closure=1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--headline-only", action="store_true", help="skip the mixed and batched measurements")
    ap.add_argument("--mixed", action="store_true",
                    help="time the headline workload in the mixed-precision mode (profiling; not the headline)")
    ap.add_argument("--tune", type=int, default=32, metavar="K",
                    help="time every tile shape over K cycles during warm-up and keep the fastest (0: off)")
    ap.add_argument("--variant", type=int, default=-1, help="force a tile shape (disables --tune)")
    ap.add_argument("--grid", type=int, default=0, help="workgroups per launch with --variant (0: one per tile)")
    ap.add_argument("--kernel-cycles", type=int, default=200,
                    help="cycles after the timed ones over which the cycle kernel's own duration is measured")
    ap.add_argument("--workload", default="scale", choices=sorted(WORKLOADS),
                    help="profiling only: time another workload in place of the headline's")
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB mebibytes (3 launches) and exit; "
                         "profiling it gives the HBM counter scale factors")
    args = ap.parse_args()
    if args.workload != "scale":  # a profiling run: the workload alone
        args.headline_only, args.no_cpu = True, True
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; --gpus must be 1"}))
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

    pb = workload(args.workload)
    if args.mixed:
        pb = [p.replace(precision="mixed") for p in pb] if isinstance(pb, list) else pb.replace(precision="mixed")
    probs = pb if isinstance(pb, list) else [pb]
    ncells = sum(p.grid.ncells for p in probs)
    precision = probs[0].precision
    t_wall = time.perf_counter()
    value, ms_cycle, sch, ctx, rates = run(pb, args.steps, args.warmup, args.tune, args.variant, args.grid, parts=5)
    wall = time.perf_counter() - t_wall
    rates.sort()
    # the cycle kernel's own mean duration, right after the timed cycles, same
    # context and schedule (launched between HIP events instead of in graphs)
    k_ms, f_ms = ctx.time_kernels(args.kernel_cycles)
    bpc = sum(algorithmic_bytes_per_cell(p) * p.grid.ncells for p in probs) / ncells
    achieved = bpc * ncells / (k_ms / 1e3) / 1e9
    traffic_b = traffic_per_launch(sch, args.workload)
    traffic = traffic_b / (k_ms / 1e3) / 1e9 if traffic_b else None
    valu = valu_per_launch(sch, args.workload)
    d = ctx.diag()
    del ctx
    torch.cuda.empty_cache()
    copy_gbs = copy_bandwidth()
    out = {
        "metric": "cell-updates/s", "value": value, "unit": "cell-updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_cycle,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32+f64" if precision == "mixed" else "f64", "data": "synthetic",
        "config": {"workload": (f"impact-1050x1050-2mat-strength-pml50-{precision}" if args.workload == "scale"
                                else f"{args.workload}-{precision} (profiling run, not the headline)"),
                   "cells": ncells, "instances": len(probs), "cycles": args.steps, "precision": precision},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_bytes_per_launch": traffic_b,
                     "copy_gbs": copy_gbs, "frac_of_copy": achieved / copy_gbs,
                     "traffic_frac_of_copy": traffic / copy_gbs if traffic else None,
                     "kernel": "k_cycle (one launch = one cycle of the whole grid)",
                     "kernel_ms": k_ms, "kernel_timing_cycles": args.kernel_cycles,
                     "finalize_ms": f_ms, "bytes_per_cell_update": bpc,
                     # what bounds this kernel in practice: VALU issue (counted
                     # instructions, halo recomputation included) and latency
                     "valu_issue": None if not valu else {
                         "lane_ops_per_cell_update": valu * 64 / ncells,
                         "achieved_lane_ops_per_s": valu * 64 / (k_ms / 1e3),
                         "peak_lane_ops_per_s": VALU_LANE_OPS_PEAK,
                         "frac": valu * 64 / (k_ms / 1e3) / VALU_LANE_OPS_PEAK}},
        "schedule": sch,
        "median_of_5": {"value": rates[2], "min": rates[0], "max": rates[4],
                        "note": "the timed cycles as 5 consecutive calls; value is over all of them"},
        "sim": {"t": d["t"], "dt": d["dt"], "cycle": d["cycle"]},
        "wall_s": wall,
    }
    torch.cuda.empty_cache()
    if not args.headline_only:
        ext = {}
        ext["mixed_scale"] = extension("mixed 1050^2", pb.replace(precision="mixed"), args.steps,
                                       args.warmup, args.tune, value)
        ext["mixed_scale"]["accuracy"] = mixed_accuracy(pb.replace(precision="fp64"))
        handover(ext["mixed_scale"], value, pb.cycles)
        ext["mixed_large"] = extension("mixed 4100^2", inputs.config_large("mixed"), 200, 10, 1)
        large64 = extension("fp64 4100^2", inputs.config_large("fp64"), 100, 10, 1)
        ext["mixed_large"]["fp64_value"] = large64["value"]
        ext["mixed_large"]["accuracy"] = mixed_accuracy(inputs.config_large("fp64"))
        handover(ext["mixed_large"], large64["value"], inputs.config_large().cycles)
        ext["batched_fp64"] = extension("batched 256 fp64", inputs.ensemble(2403, 256, 200, 800), 40, 2, 1)
        ext["batched_mixed"] = extension("batched 1024 mixed",
                                         inputs.ensemble(4267, 1024, 200, 1200, precision="mixed"), 10, 1, 1)
        ext["batched_mixed"]["accuracy"] = ensemble_accuracy()
        ext["layered_fp64"] = extension("layered 1050^2 fp64",
                                        inputs.layered_impact(1000, 50, 50, 15e3, 70, name="layered"), 500, 20,
                                        args.tune, value)
        ext["paper_layout_fp64"] = extension("Table 2 grid 512x532 fp64", inputs.config_paper(), 300, 20,
                                             args.tune, value)
        ext["three_layer_fp64"] = extension("three-layer 1050^2 fp64",
                                            inputs.three_layer_impact(1000, 50, 50, 15e3, 7, 75, name="three"),
                                            500, 20, args.tune, value)
        ext["paper_layers_fp64"] = extension("Table 2 grid 512x532 three layers fp64",
                                             inputs.config_paper_layers(), 300, 20, args.tune, value)
        ext["three_layer_pm_fp64"] = extension("three-layer 1050^2 per-material fp64", three_layer_pm(inputs),
                                               500, 20, args.tune, value)
        ext["paper_layers_damage_fp64"] = extension("Table 2 grid three layers, damage fp64",
                                                    paper_layers_damage(), 300, 20, args.tune, value)
        ext["pml_payoff"] = pml_payoff()
        ext["pml_payoff_table2"] = pml_payoff_table2()
        ext["damage_table2"] = damage_table2()
        out["extensions"] = ext
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(probs[0])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
