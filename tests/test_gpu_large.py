"""The large mixed-precision impact at full size (4000 x 4000 cells + 100-cell
PML, 16.8 M cells, two materials with strength, R = 200 cells, 12 km/s,
2000 cycles), in the launch configuration the benchmark times.

Against the plain-FP64 GPU run of the same problem (which equals the oracle
bit for bit at every size the oracle can run, and for the first cycles of the
1050^2 workload): the conserved densities within 1e-4 (relative L2) at cycle
200, the crater level on the axis within one cell after 2000 cycles, and the
mass budget. Against the oracle on the same problem 10x coarser (400 x 400 +
10-cell PML of 10 m cells, R = 20 cells) run to the same physical time: the
crater level on the axis within one coarse cell, and the fine fields
averaged over 10 x 10 blocks close to the coarse ones (a resolution
comparison, so the bounds are those of the discretisation, not rounding).
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2403_04267_amd import inputs

from .crater import conserved_errors, crater_depth

pytestmark = pytest.mark.gpu


def ctx(problems):
    from paper_2403_04267_amd.salec import Salec
    return Salec(problems)


def block(x, k=10):
    nz, nr = x.shape
    return x[: nz // k * k, : nr // k * k].reshape(nz // k, k, nr // k, k).mean(axis=(1, 3))


@pytest.fixture(scope="module")
def large_runs():
    pb = inputs.config_large("fp64")
    a, b = ctx(pb), ctx(pb.replace(precision="mixed"))
    a.step(200)
    b.step(200)
    e200 = conserved_errors(b.fields(), a.fields(), pb.grid)
    a.step(1800)
    b.step(1800)
    out = {"pb": pb, "e200": e200, "Fa": a.fields(eos=False), "Fb": b.fields(eos=False),
           "da": a.diag(), "db": b.diag()}
    del a, b
    return out


def test_large_mixed_against_fp64_gpu(large_runs):
    r = large_runs
    pb = r["pb"]
    print("[large mixed cycle 200] " + " ".join(f"{k} {v:.2e}" for k, v in r["e200"].items()), flush=True)
    bad = {k: v for k, v in r["e200"].items() if not v <= 1e-4}
    assert not bad, bad
    sj = pb.scene.surface_j
    da, db = crater_depth(r["Fa"]["f"], pb.grid, sj), crater_depth(r["Fb"]["f"], pb.grid, sj)
    print(f"[large cycle 2000] crater level on the axis fp64 {da:.3f} m, mixed {db:.3f} m", flush=True)
    assert abs(da - db) <= pb.grid.dz
    # mass budget of the mixed run: FP64 sums of FP64 densities and fluxes
    d = r["db"]
    assert int(d["cycle"]) == 2000 and d["err"] == 0
    total = d["mass"] + d["mass_out"] + d["mass_pml"]
    assert abs(total - r["da"]["mass"] - r["da"]["mass_out"] - r["da"]["mass_pml"]) <= 1e-6 * total


def test_large_against_the_oracle_on_a_coarse_copy(large_runs):
    r = large_runs
    pb = r["pb"]
    t_end = r["db"]["t"]
    c = inputs.impact(400, 10, 20, 12e3, nmat=2, strength=True, cycles=0, dx=10.0)
    c.grid.t_stop = t_end
    o = Oracle(c)
    for _ in range(100):
        if o.diag()["t"] >= t_end:
            break
        o.step(10)
    assert abs(o.diag()["t"] - t_end) <= 1e-12 * t_end
    F = o.fields(eos=False)
    dc = crater_depth(F["f"], c.grid, c.scene.surface_j)
    df = crater_depth(r["Fb"]["f"], pb.grid, pb.scene.surface_j)
    phi_f, phi_c = block(r["Fb"]["f"].sum(0)), F["f"].sum(0)
    rho_f, rho_c = block(r["Fb"]["rho"]), F["rho"]
    l1 = np.abs(phi_f - phi_c).sum() / np.abs(phi_c).sum()
    l2 = float(np.sqrt(((rho_f - rho_c) ** 2).sum() / (rho_c ** 2).sum()))
    print(f"[large vs coarse oracle, t = {t_end:.4e} s] crater level fine {df:.2f} m, coarse {dc:.2f} m; "
          f"block phi L1 {l1:.2e}, block rho L2 {l2:.2e}", flush=True)
    assert abs(df - dc) <= c.grid.dz
    assert l1 < 1e-2 and l2 < 5e-2
