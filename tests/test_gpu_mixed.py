"""GPU checks of the mixed-precision mode (FP32 bulk arithmetic; FP64
density, volume fractions, internal energy, flux sums and time step) against
the FP64 oracle and the FP64 GPU path, through the C ABI.

Bars. Errors are relative L2 norms of the conserved volume densities (see
tests/crater.py: rho, rho I, phi p, f, phi s, node momentum). While the runs
are still deterministic in the ejecta (first 100 cycles) every one is
<= 1e-4. Later the method's own amplification of rounding in the ejecta
takes over: two FP64 runs that differ by one ulp in the initial velocities
drift apart to 1e-4 - 1e-2 by cycle 500 (test_fp64_sensitivity_floor in
tests/test_oracle_physics.py). The floor is measured on each problem with
the oracle (initial velocities one ulp up) and printed, per field over the
cells holding matter, beside the mixed run's. In the hydrodynamic impact the
floor is of the mixed error's size, and each conserved density is held to
max(1e-4, 10 x floor). The strength impact is not chaotic (floor 2e-7 at
cycle 300) while the mixed run's density is 2.7e-3 off: that is single
precision's own loss, so there the bar is the measured one, density and
fractions within 1e-2. Both hold crater depth and radius to one cell.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2403_04267_amd import inputs

from .crater import conserved_errors, crater_depth, crater_radius, per_field, rel_l2

pytestmark = pytest.mark.gpu

TOL = 1e-4


def ctx(problems):
    from paper_2403_04267_amd.salec import Salec
    return Salec(problems)


def check_pair(pb, early, late, label, floor_bar):
    pm = pb.replace(precision="mixed")
    g, o, p = ctx(pm), Oracle(pb), Oracle(pb)
    F0 = p.fields(eos=False)
    p.set_fields(F0["rho"], F0["I"], F0["f"], np.nextafter(F0["v"], np.inf), F0["s"])
    g.step(early)
    o.step(early)
    p.step(early)
    e = conserved_errors(g.fields(), o.fields(), pb.grid)
    print(f"[{label} cycle {early}] " + " ".join(f"{k} {v:.2e}" for k, v in e.items()), flush=True)
    bad = {k: v for k, v in e.items() if not v <= TOL}
    assert not bad, bad
    g.step(late - early)
    o.step(late - early)
    p.step(late - early)
    Fg, Fo, Fp = g.fields(), o.fields(), p.fields()
    e = conserved_errors(Fg, Fo, pb.grid)
    sj = pb.scene.surface_j
    eg, ep = per_field(Fg, Fo, pb.grid, sj), per_field(Fp, Fo, pb.grid, sj)
    for name, x in (("mixed", eg), ("FP64 floor", ep)):
        print(f"[{label} cycle {late}, {name}] " + " ".join(f"{k} {v:.2e}" for k, v in x.items()), flush=True)
    if floor_bar:
        for k, v in e.items():
            assert v <= max(TOL, 10.0 * ep["cons." + k]), (k, v, ep["cons." + k])
    else:
        assert e["rho"] < 1e-2 and e["f"] < 1e-2
    dg, do = crater_depth(Fg["f"], pb.grid, sj), crater_depth(Fo["f"], pb.grid, sj)
    rg, ro = crater_radius(Fg["f"], pb.grid, sj), crater_radius(Fo["f"], pb.grid, sj)
    print(f"[{label} cycle {late}] " + " ".join(f"{k} {v:.2e}" for k, v in e.items()) +
          f" depth {dg:.3f}/{do:.3f} radius {rg:.3f}/{ro:.3f}", flush=True)
    assert abs(dg - do) <= pb.grid.dz
    assert abs(rg - ro) <= pb.grid.dr
    dgd, dod = g.diag(), o.diag()
    assert dgd["cycle"] == dod["cycle"] == late
    # dt follows the fastest ejecta, where the runs differ most
    assert abs(dgd["t"] - dod["t"]) <= 1e-2 * dod["t"]
    return g, o


def test_mixed_small_impact_against_oracle():
    """100x100 + 20 PML hydrodynamic impact, 500 cycles."""
    check_pair(inputs.config_small(), 100, 500, "small", floor_bar=True)


def test_mixed_strength_two_materials_against_oracle():
    pb = inputs.impact(61, 13, 6, 15e3, nmat=2, strength=True, cycles=300, name="strength-61")
    check_pair(pb, 100, 300, "strength-61", floor_bar=False)


def test_mixed_mass_budget_is_exact_to_fp64_sums():
    pb = inputs.config_small().replace(precision="mixed")
    g = ctx(pb)
    d0 = g.diag()
    g.step(300)
    d = g.diag()
    total = d["mass"] + d["mass_out"] + d["mass_pml"]
    assert abs(total - d0["mass"]) <= 1e-12 * d0["mass"]


def test_mixed_rest_state_is_bitwise_unchanged():
    mat = inputs.basalt(strength=True)
    g = inputs.Grid(n_r=40, n_z=40, pml_r=8, pml_b=8, nmat=2)
    pb = inputs.Problem(grid=g, mats=[mat, mat], pml=inputs.Pml(), precision="mixed")
    NR, NZ = g.NR, g.NZ
    rho = np.full((NZ, NR), 2860.0)
    I = np.zeros((NZ, NR))
    f = np.zeros((2, NZ, NR))
    f[0] = 0.75
    f[1] = 0.25
    v = np.zeros((2, NZ + 1, NR + 1))
    c = ctx(pb)
    c.set_fields(rho, I, f, v)
    c.step(200)
    F = c.fields()
    assert np.array_equal(F["rho"], rho) and np.array_equal(F["I"], I)
    assert np.array_equal(F["f"], f) and not np.any(F["v"]) and not np.any(F["s"])


def test_mixed_tile_shapes_agree_bitwise():
    from paper_2403_04267_amd.salec import SalecError, num_variants
    pb = inputs.impact(61, 13, 6, 15e3, nmat=2, strength=True, cycles=0, precision="mixed")
    ref = None
    for v in range(num_variants()):
        c = ctx(pb)
        try:
            c.set_schedule(v, 0)
        except SalecError:
            assert v in (11, 14)  # built for three slots and the per-material closure only
            continue
        c.step(80)
        F = c.fields()
        if ref is None:
            ref = F
        for k in F:
            assert np.array_equal(F[k], ref[k]), (v, k)


def test_mixed_ensemble_crater_depths_match_fp64_ensemble():
    spec = [(60, 6, 5, 8e3, 5e6), (90, 9, 6, 14e3, 30e6), (75, 8, 7, 18e3, 12e6)]
    members = [inputs.impact(n, p, R, v, nmat=2, strength=True, cycles=0, Y0=y) for (n, p, R, v, y) in spec]
    a = ctx(members)
    b = ctx([m.replace(precision="mixed") for m in members])
    a.step(400)
    b.step(400)
    for k, pb in enumerate(members):
        Fa, Fb = a.fields(k=k), b.fields(k=k)
        sj = pb.scene.surface_j
        da, db = crater_depth(Fa["f"], pb.grid, sj), crater_depth(Fb["f"], pb.grid, sj)
        print(f"member {k}: depth fp64 {da:.3f} mixed {db:.3f}", flush=True)
        assert abs(da - db) <= pb.grid.dz
        assert rel_l2(Fb["rho"], Fa["rho"]) < 1e-2
