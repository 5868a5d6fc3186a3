"""GPU checks of the lithostatic two-layer target (initial pressure p0 of
Sec. 3 in the momentum balance and the PML's psi1), through the C ABI.

FP64: the library's lithostatic column (densities and p0) equals the
oracle's bit for bit, a target at rest stays exactly at rest with the PML
on, and a layered impact under gravity matches the oracle bit for bit.
Mixed mode: the FP32 equation of state differs from the FP64 p0 by rounding,
so the column at rest keeps only a rounding-level residual; the layered
impact meets the mixed-precision bar of the other impacts (conserved
densities within 1e-4 of the FP64 oracle over the first 100 cycles).
"""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2403_04267_amd import inputs

from .crater import conserved_errors
from .test_gpu_parity import compare
from .test_oracle_lithostatic import column

pytestmark = pytest.mark.gpu


def ctx(pb):
    from paper_2403_04267_amd.salec import Salec
    return Salec(pb)


def test_lithostatic_column_matches_oracle_and_stays_at_rest():
    pb = column()
    g, o = ctx(pb), Oracle(pb)
    assert np.array_equal(g.p0(), o.p0())
    Fg0, Fo = g.fields(eos=False), o.fields(eos=False)
    for k in Fo:
        assert np.array_equal(Fg0[k], Fo[k]), k
    g.step(150)
    Fg1 = g.fields(eos=False)
    for k in Fg0:
        assert np.array_equal(Fg0[k], Fg1[k]), k
    aux = g.pml_aux()
    for k in ("psi1_b_r", "psi1_b_z", "psi1_r_r", "psi1_r_z"):
        assert np.all(aux[k] == 0.0), k


def test_set_p0_round_trip_and_effect():
    pb = column()
    g, o = ctx(pb), Oracle(pb)
    p0 = g.p0()
    z = np.zeros_like(p0)
    g.set_p0(z)
    o.set_p0(z)
    assert np.array_equal(g.p0(), z)
    g.step(60)
    o.step(60)
    compare(g, o, "column without p0", tol=0.0)
    assert np.abs(g.fields(eos=False)["v"]).max() > 0.1
    with pytest.raises(Exception):
        g.set_p0(np.full_like(p0, np.nan))


def test_layered_impact_fp64_bitwise():
    pb = inputs.layered_impact(60, 12, 6, 15e3, 10, name="layered")
    g, o = ctx(pb), Oracle(pb)
    done = 0
    for n in (1, 60, 200):
        g.step(n - done)
        o.step(n - done)
        done = n
        compare(g, o, f"layered cycle {n}", tol=0.0)


def test_layered_impact_mixed_against_oracle():
    pb = inputs.layered_impact(60, 12, 6, 15e3, 10, name="layered")
    g, o = ctx(pb.replace(precision="mixed")), Oracle(pb)
    g.step(100)
    o.step(100)
    e = conserved_errors(g.fields(), o.fields(), pb.grid)
    print("[layered mixed cycle 100] " + " ".join(f"{k} {v:.2e}" for k, v in e.items()), flush=True)
    bad = {k: v for k, v in e.items() if not v <= 1e-4}
    assert not bad, bad


def test_mixed_column_residual_is_rounding_level():
    pb = column().replace(precision="mixed")
    g = ctx(pb)
    g.step(150)
    v = np.abs(g.fields(eos=False)["v"]).max()
    print(f"[mixed column] max |v| after 150 cycles {v:.3e} m/s", flush=True)
    assert v < 1e-2


def test_layered_impact_with_stress_damping_layers_fp64_bitwise():
    """The PML extension that also relaxes the deviatoric stress in the layers."""
    pb = inputs.layered_impact(60, 12, 6, 15e3, 10, name="layered-damp")
    pb = pb.replace(pml=inputs.Pml(damp_stress=1))
    g, o = ctx(pb), Oracle(pb)
    done = 0
    for n in (1, 60, 200):
        g.step(n - done)
        o.step(n - done)
        done = n
        compare(g, o, f"layered, stress damping, cycle {n}", tol=0.0)
    m = ctx(pb.replace(precision="mixed"))
    m.step(100)
    o2 = Oracle(pb)
    o2.step(100)
    e = conserved_errors(m.fields(), o2.fields(), pb.grid)
    bad = {k: v for k, v in e.items() if not v <= 1e-4}
    assert not bad, bad
