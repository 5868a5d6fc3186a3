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
