"""Pin of the oracle's PML damping profile (Sec. 3): d(y) = (3c / 2 delta)
(y / delta)^2 ln(1/R), c the largest acoustic speed, delta the layer
thickness, y the distance from the layer's inner face. Written out here from
its closed form on a uniform grid, with c the largest longitudinal speed at
rest over the materials (sqrt((A + 4G/3) / rho0), G from Poisson's ratio),
for a layered target whose deepest material is the fastest."""
import numpy as np
import pytest

from oracle.oracle import Oracle
from paper_2403_04267_amd import inputs


def c_long(m):
    G = 3.0 * m.A * (1.0 - 2.0 * m.poisson) / (2.0 * (1.0 + m.poisson)) if m.strength else 0.0
    return np.sqrt((m.A + 4.0 * G / 3.0) / m.rho0)


@pytest.mark.parametrize("make", [
    lambda: inputs.three_layer_impact(40, 10, 4, 10e3, 3, 8),
    lambda: inputs.layered_impact(40, 10, 4, 10e3, 6),
])
def test_profile_uses_the_largest_acoustic_speed(make):
    pb = make()
    c = max(c_long(m) for m in pb.mats[:pb.grid.nmat])
    assert c > c_long(pb.mats[0]) * 1.2  # the largest speed is not material 0's
    o = Oracle(pb)
    dcz, dnz, dcr, dnr = o.profiles()
    g = pb.grid
    delta_b, delta_r = g.pml_b * g.dz, g.pml_r * g.dr
    lnR = np.log(1.0 / pb.pml.R)
    yc = delta_b - (np.arange(g.pml_b) + 0.5) * g.dz
    yn = delta_b - np.arange(g.pml_b) * g.dz
    np.testing.assert_allclose(dcz[:g.pml_b], 1.5 * c / delta_b * (yc / delta_b) ** 2 * lnR, rtol=1e-12)
    np.testing.assert_allclose(dnz[:g.pml_b], 1.5 * c / delta_b * (yn / delta_b) ** 2 * lnR, rtol=1e-12)
    assert np.all(dcz[g.pml_b:] == 0.0) and np.all(dnz[g.pml_b:] == 0.0)
    xr = (np.arange(g.pml_r) + 0.5) * g.dr
    np.testing.assert_allclose(dcr[g.n_r:], 1.5 * c / delta_r * (xr / delta_r) ** 2 * lnR, rtol=1e-12)
    assert np.all(dcr[:g.n_r] == 0.0)
    # an explicit speed overrides the default
    o2 = Oracle(pb.replace(pml=inputs.Pml(c_ref=1000.0)))
    assert o2.profiles()[0][0] == pytest.approx(dcz[0] * 1000.0 / c, rel=1e-12)


def _random_problem(damp, strength=True):
    # dt_max well below the Courant limit (~1.5e-3 s): both runs take the same
    # steps, so only the damping can make them differ
    g = inputs.Grid(n_r=40, n_z=40, pml_r=10, pml_b=10, nmat=1, dr=10.0, dz=10.0, dt_max=2e-4)
    pb = inputs.Problem(grid=g, mats=[inputs.basalt(strength=strength)], pml=inputs.Pml(damp_stress=damp))
    o = Oracle(pb)
    rho, I, v = inputs.random_state(g, 11)
    o.set_fields(rho, I, np.ones((1, g.NZ, g.NR)), v)
    return o


def test_stress_damping_acts_only_in_the_layers():
    """The extension that also relaxes the deviatoric stress in the layers
    (not in Sec. 3): outside the layers' numerical domain of dependence the
    state is bit for bit that of Sec. 3's layers; inside them the stress is
    smaller; with no stress at all it changes nothing."""
    n = 6
    a, b = _random_problem(0), _random_problem(1)
    a.step(n)
    b.step(n)
    A, B = a.fields(eos=False), b.fields(eos=False)
    g = a.problem.grid
    reach = 5 * n + 2  # cells per cycle of the cycle's stencil, generously
    j0, i1 = g.pml_b + reach, g.n_r - reach
    assert j0 < g.NZ and i1 > 0
    for k in ("rho", "I", "s"):
        x, y = A[k][..., j0:, :i1], B[k][..., j0:, :i1]
        assert np.array_equal(x, y), k
    assert np.array_equal(A["v"][:, j0 + 1:, :i1], B["v"][:, j0 + 1:, :i1])
    lay = np.zeros((g.NZ, g.NR), dtype=bool)
    lay[:g.pml_b, :] = True
    lay[:, g.n_r:] = True
    sa, sb = np.abs(A["s"][:, lay]).sum(), np.abs(B["s"][:, lay]).sum()
    assert 0.0 < sb < sa, (sa, sb)
    # hydrodynamic material: no stress, nothing to relax
    c, d = _random_problem(0, strength=False), _random_problem(1, strength=False)
    c.step(n)
    d.step(n)
    C_, D_ = c.fields(eos=False), d.fields(eos=False)
    for k in C_:
        assert np.array_equal(C_[k], D_[k]), k
