"""Pins of the oracle's lithostatic target (initial pressure p0, Sec. 3).

The paper writes the momentum balance with div(tau - p + p0), p0 the
pressure before impact with -grad p0 + rho g = 0, and carries p - p0 into
the PML auxiliary psi1. What fixes the oracle here, other than itself:

  * the discrete hydrostatic relation: p0 at the top target row is
    g dz rho / 2 and consecutive rows differ by g dz (rho_j + rho_{j+1}) / 2;
  * p0 is the cold (E = 0) Tillotson pressure of the row's density, so a
    target at rest is an exact discrete equilibrium: nothing may move, with
    strength and with the PML on (psi1 sees p - p0 = 0);
  * the same column without p0 is not in equilibrium (it rebounds), so the
    p0 term is what holds it;
  * layers carry their materials and densities at or above rho0.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle, tillotson
from paper_2403_04267_amd import inputs


def column(n=40, pml=10, crust=12, gravity=9.81, strength=True):
    """A two-layer lithostatic target at rest (no projectile)."""
    pb = inputs.layered_impact(n, pml, 6, 0.0, crust, gravity=gravity, strength=strength)
    return pb.replace(scene=inputs.Scene(surface_j=pb.scene.surface_j, radius=0.0, v_imp=0.0,
                                         gravity=gravity, layer_j=pb.scene.layer_j))


def test_hydrostatic_relation():
    pb = column()
    o = Oracle(pb)
    F = o.fields(eos=False)
    rho, p0 = F["rho"][:, 0], o.p0()
    sj, g, dz = pb.scene.surface_j, pb.scene.gravity, pb.grid.dz
    assert np.all(p0[sj:] == 0.0)
    assert p0[sj - 1] == pytest.approx(0.5 * g * dz * rho[sj - 1], rel=1e-12)
    for j in range(sj - 1):
        dp = p0[j] - p0[j + 1]
        assert dp == pytest.approx(0.5 * g * dz * (rho[j] + rho[j + 1]), rel=1e-11), j
    # every row is horizontally uniform
    assert np.all(F["rho"] == F["rho"][:, :1])


def test_p0_is_the_cold_pressure_of_each_row():
    pb = column()
    o = Oracle(pb)
    rho, p0 = o.fields(eos=False)["rho"][:, 0], o.p0()
    sj, lj = pb.scene.surface_j, pb.scene.layer_j
    for j in range(sj):
        m = pb.mats[1 if j < lj else 0]
        assert rho[j] >= m.rho0
        p, _ = tillotson(m, rho[j], 0.0)
        assert p == p0[j], j  # exactly: the column starts in discrete equilibrium


def test_layers_carry_their_materials():
    pb = column()
    o = Oracle(pb)
    f = o.fields(eos=False)["f"]
    sj, lj = pb.scene.surface_j, pb.scene.layer_j
    assert np.all(f[1, :lj] == 1.0) and np.all(f[0, :lj] == 0.0)
    assert np.all(f[0, lj:sj] == 1.0) and np.all(f[1, lj:sj] == 0.0)
    assert np.all(f[:, sj:] == 0.0)


@pytest.mark.parametrize("pml_on", [1, 0])
def test_lithostatic_target_at_rest_stays_at_rest(pml_on):
    pb = column()
    pb = pb.replace(pml=inputs.Pml(enabled=pml_on))
    o = Oracle(pb)
    F0 = o.fields(eos=False)
    o.step(150)
    F1 = o.fields(eos=False)
    for k in F0:
        assert np.array_equal(F0[k], F1[k]), k
    if pml_on:
        aux = o.pml_aux()
        for k in ("psi1_b_r", "psi1_b_z", "psi1_r_r", "psi1_r_z", "phi2_b_r", "phi2_b_z"):
            assert np.all(aux[k] == 0.0), k


def test_without_p0_the_column_moves():
    o = Oracle(column())
    o.set_p0(np.zeros(o.NZ))
    o.step(100)
    assert np.abs(o.fields(eos=False)["v"]).max() > 1.0


def test_zero_gravity_has_no_initial_pressure():
    o = Oracle(column(gravity=0.0))
    assert np.all(o.p0() == 0.0)
    pb = column(gravity=0.0)
    rho = o.fields(eos=False)["rho"]
    assert np.all(rho[:pb.scene.layer_j] == pb.mats[1].rho0)
    assert np.all(rho[pb.scene.layer_j:pb.scene.surface_j] == pb.mats[0].rho0)
