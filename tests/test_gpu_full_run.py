"""The 1050 x 1050 strength impact (two materials, R = 50 cells, 15 km/s,
50-cell PML) run for its whole 5000 cycles in the launch configuration the
benchmark times (the tuned schedule), in FP64 and in the mixed mode.

The oracle cannot follow 5.5e9 cell-updates in a test, so the checks are what
holds at any length: no device error, the cycle count, a strictly positive
finite step, the mass budget closing (matter in the grid plus what left
through the outer faces plus what the PML sink removed equals the initial
mass, to the rounding of FP64 sums), and the crater on the axis in both modes
within one cell of each other. The first 10 cycles of the same schedule equal
the oracle bit for bit (the full-size parity test).
"""
import numpy as np
import pytest

from paper_2403_04267_amd import inputs

from .crater import crater_depth

pytestmark = pytest.mark.gpu

CYCLES = 5000


@pytest.fixture(scope="module")
def runs():
    from paper_2403_04267_amd.salec import Salec
    pb = inputs.config_scale()
    out = {}
    for prec in ("fp64", "mixed"):
        c = Salec(pb.replace(precision=prec))
        d0 = c.diag()
        c.tune(2)
        done = int(c.diag()["cycle"])
        c.step(CYCLES - done)
        out[prec] = {"d0": d0, "d": c.diag(), "f": c.fields(eos=False)["f"], "sched": c.schedule()}
        del c
    out["pb"] = pb
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_whole_run_completes_with_a_closed_mass_budget(runs, prec):
    r = runs[prec]
    d0, d = r["d0"], r["d"]
    s = r["sched"]
    print(f"[{prec}, {CYCLES} cycles, {s['tile_r']}x{s['tile_z']}/{s['threads']} grid {s['grid']}] "
          f"t = {d['t']:.4e} s, dt = {d['dt']:.3e} s, mass out {d['mass_out']:.3e}, "
          f"PML sink {d['mass_pml']:.3e} of {d0['mass']:.4e} kg", flush=True)
    assert int(d["cycle"]) == CYCLES and d["err"] == 0
    assert np.isfinite(d["dt"]) and d["dt"] > 0
    total = d["mass"] + d["mass_out"] + d["mass_pml"]
    assert abs(total - d0["mass"]) <= 1e-12 * d0["mass"]


def test_crater_levels_of_both_modes_agree(runs):
    pb = runs["pb"]
    sj = pb.scene.surface_j
    da = crater_depth(runs["fp64"]["f"], pb.grid, sj)
    db = crater_depth(runs["mixed"]["f"], pb.grid, sj)
    print(f"[{CYCLES} cycles] crater level on the axis: fp64 {da:.3f} m, mixed {db:.3f} m", flush=True)
    assert abs(da - db) <= pb.grid.dz
