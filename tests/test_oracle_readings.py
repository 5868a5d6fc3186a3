"""Pins of oracle readings that only a whole cycle exercises (-m "not gpu").

Each test starts from a uniform state with an affine or linear velocity
field, forces the step with set_clock, runs one cycle, and checks cells far
from the boundaries against the closed form of that cycle. A uniform isotropic
stress exerts no node force in the interior, and the donor-cell remap of a
uniform field leaves it unchanged, so interior cells see only the
Lagrangian-step rule under test. Each test fails on a named plausible mistake.

  R5   mixed-cell volume change: compression closes the void before the
       material is compressed (material volume ratio J_m = min(1, J / phi));
       expansion stretches the material only above its tension floor, with a
       linear ramp over 1e-4 A, and otherwise opens void.
  R10  donor outflow limiter: a donor never gives more than its Lagrangian
       volume; all its outflows are scaled by V^L / outflow.
  G    shear modulus G = 0.6 rho_mat c^2 (Poisson ratio 0.25) times the
       thermal softening (E_cv - E) / (E_cv - E_iv) clipped to [0, 1], read off
       the elastic stress increment of a simple shear; c^2 from central
       differences of the pressure, not from the oracle's closed form.
"""
import numpy as np
import pytest

from oracle.oracle import Oracle, tillotson
from paper_2403_04267_amd import inputs

N = 14  # cells per side; interior = cells at least 3 away from every wall


def interior(g):
    return slice(3, g.NZ - 3), slice(1, g.NR - 3)


def grid(**kw):
    return inputs.Grid(n_r=N, n_z=N, **kw)


def affine_velocity(g, a):
    """v = a x about the origin (axis, bottom): div v = 3a in r-z."""
    rn = np.arange(g.NR + 1)[None, :] * g.dr * np.ones((g.NZ + 1, 1))
    zn = np.arange(g.NZ + 1)[:, None] * g.dz * np.ones((1, g.NR + 1))
    return np.stack([a * rn, a * zn])


def one_cycle(pb, rho, I, f, v, dt, s=None):
    o = Oracle(pb)
    o.set_fields(rho, I, f, v, s)
    o.set_clock(0.0, dt)
    F0 = o.fields()
    o.step(1)
    return F0, o.fields()


# ---------------------------------------------------------------- R5
@pytest.mark.parametrize("phi", [0.5, 0.8])
def test_r5_compression_closes_void_before_compressing_matter(phi):
    """Uniform compression with J = 0.99 of cells holding matter at rho0 in
    a fraction phi > J: the material is not compressed, so the matter density
    stays rho0 and the matter fraction becomes phi / J. The uniform-strain
    closure (void and matter compressed alike, J_m = J) would give a matter
    density rho0 / J, 1 % high."""
    mat = inputs.basalt()
    g = grid()
    pb = inputs.Problem(grid=g, mats=[mat], pml=inputs.Pml(enabled=0))
    J = 0.99
    dt = 1e-4
    a = (J - 1.0) / (3.0 * dt)
    rho = np.full((g.NZ, g.NR), phi * mat.rho0)
    I = np.zeros_like(rho)
    f = np.full((1, g.NZ, g.NR), phi)
    F0, F1 = one_cycle(pb, rho, I, f, affine_velocity(g, a), dt)
    js, is_ = interior(g)
    assert np.all(F0["p"][js, is_] == 0.0)
    rm = F1["rho"][js, is_] / F1["f"][0][js, is_]
    np.testing.assert_allclose(rm, mat.rho0, rtol=1e-12)
    np.testing.assert_allclose(F1["f"][0][js, is_], phi / J, rtol=1e-12)


def test_r5_void_closes_then_matter_compresses():
    """phi = 0.995 compressed with J = 0.99 < phi: the void closes (f = 1)
    and the matter takes the rest, J_m = J / phi, so its density is
    phi rho0 / J."""
    mat = inputs.basalt()
    g = grid()
    pb = inputs.Problem(grid=g, mats=[mat], pml=inputs.Pml(enabled=0))
    phi, J, dt = 0.995, 0.99, 1e-4
    a = (J - 1.0) / (3.0 * dt)
    rho = np.full((g.NZ, g.NR), phi * mat.rho0)
    f = np.full((1, g.NZ, g.NR), phi)
    _, F1 = one_cycle(pb, rho, np.zeros_like(rho), f, affine_velocity(g, a), dt)
    js, is_ = interior(g)
    np.testing.assert_allclose(F1["f"][0][js, is_], 1.0, rtol=1e-12)
    np.testing.assert_allclose(F1["rho"][js, is_], phi * mat.rho0 / J, rtol=1e-12)
    assert np.all(F1["p"][js, is_] > 0.0)


@pytest.mark.parametrize("where", ["at_floor", "in_ramp", "above_ramp"])
def test_r5_expansion_opens_void_at_the_tension_floor(where):
    """A full cell expanded by J = 1.01. Hydrodynamic basalt has its tension
    floor at p_min = 0. At the floor (rho = rho0, p = 0) the matter does not
    stretch: the void opens, f = 1 / J, matter density rho0. Well above the
    floor plus the 1e-4 A ramp it stretches like the cell: f stays 1. Inside
    the ramp the matter takes the fraction s = (p - p_min) / (1e-4 A) of the
    expansion: J_m = 1 + (J - 1) s, f = J_m / J. A rule that always stretches
    (or never does) fails two of the three cases."""
    mat = inputs.basalt()
    g = grid()
    pb = inputs.Problem(grid=g, mats=[mat], pml=inputs.Pml(enabled=0))
    J, dt = 1.01, 1e-4
    a = (J - 1.0) / (3.0 * dt)
    ps = 1e-4 * mat.A
    if where == "at_floor":
        r = mat.rho0
    elif where == "in_ramp":
        # cold compression with A mu + B mu^2 = ps / 2
        mu = (-mat.A + np.sqrt(mat.A ** 2 + 2.0 * mat.B * ps)) / (2.0 * mat.B)
        r = mat.rho0 * (1.0 + mu)
    else:
        r = 1.01 * mat.rho0
    rho = np.full((g.NZ, g.NR), r)
    f = np.ones((1, g.NZ, g.NR))
    F0, F1 = one_cycle(pb, rho, np.zeros_like(rho), f, affine_velocity(g, a), dt)
    js, is_ = interior(g)
    p0 = F0["p"][js, is_]
    s = np.clip((p0 - mat.p_min) / ps, 0.0, 1.0)
    if where == "at_floor":
        assert np.all(s == 0.0)
    elif where == "in_ramp":
        assert np.all(np.abs(s - 0.5) < 1e-6)
    else:
        assert np.all(s == 1.0)
    Jm = 1.0 + (J - 1.0) * s
    np.testing.assert_allclose(F1["f"][0][js, is_], Jm / J, rtol=1e-12)
    np.testing.assert_allclose(F1["rho"][js, is_] / F1["f"][0][js, is_], r / Jm, rtol=1e-12)


# ---------------------------------------------------------------- R10
def test_r10_donor_limited_to_its_lagrangian_volume():
    """A single full cell of matter in void, everything moving up at a speed
    that sweeps 1.5 cells in the forced step. Unlimited, the cell would give
    1.5 times its mass (leaving -0.5 M behind). Limited, each donor's outflow
    is scaled by V^L / outflow = 2/3: the whole mass moves exactly one cell up,
    the donor is left empty (not negative), its fraction moves with it, and
    mass is conserved. A limiter scaled the wrong way (outflow / V^L) would
    create mass; none would leave negative mass."""
    mat = inputs.basalt()
    g = grid(top_closed=0, dt_max=1.0)
    pb = inputs.Problem(grid=g, mats=[mat], pml=inputs.Pml(enabled=0))
    dt, u = 1e-4, 1.5 * g.dz / 1e-4
    rho = np.zeros((g.NZ, g.NR))
    f = np.zeros((1, g.NZ, g.NR))
    jc, ic = 6, 4
    rho[jc, ic] = mat.rho0
    f[0, jc, ic] = 1.0
    v = np.zeros((2, g.NZ + 1, g.NR + 1))
    v[1, 1:, :] = u  # the bottom row of nodes is no-slip
    V = (np.arange(g.NR) + 0.5)[None, :] * g.dr * g.dr * g.dz * np.ones((g.NZ, 1))
    M0 = np.sum(rho * V)
    _, F1 = one_cycle(pb, rho, np.zeros_like(rho), f, v, dt)
    M1 = F1["rho"] * V
    assert F1["rho"][jc, ic] == 0.0
    assert F1["f"][0][jc, ic] == 0.0
    np.testing.assert_allclose(M1[jc + 1, ic], M0, rtol=1e-14)
    np.testing.assert_allclose(F1["f"][0][jc + 1, ic], 1.0, rtol=1e-14)
    assert np.all(F1["rho"] >= 0.0)
    np.testing.assert_allclose(np.sum(M1), M0, rtol=1e-14)


# ---------------------------------------------------------------- G, softening
def c2_by_differences(mat, r, e):
    """c^2 = dp/drho|_E + (p / rho^2) dp/dE|_rho from central differences of
    the oracle's pressure alone."""
    hr = 1e-6 * r
    he = 1e-6 * max(e, 1e5)
    p = tillotson(mat, r, e)[0]
    dpr = (tillotson(mat, r + hr, e)[0] - tillotson(mat, r - hr, e)[0]) / (2 * hr)
    if e - he < 0.0:  # the law sees max(E, 0): one-sided, second order
        dpe = (-3 * p + 4 * tillotson(mat, r, e + he)[0] - tillotson(mat, r, e + 2 * he)[0]) / (2 * he)
    else:
        dpe = (tillotson(mat, r, e + he)[0] - tillotson(mat, r, e - he)[0]) / (2 * he)
    return dpr + p / r ** 2 * dpe


@pytest.mark.parametrize("state", [(1.1, "cold"), (1.1, "mid"), (0.9, "mid"), (1.1, "hot"),
                                   (1.0, "cold")])
def test_shear_modulus_and_softening_hand_values(state):
    """Simple shear v_z = gamma r of a uniform state (rho, E) with s = 0: one
    step gives s_rz = G gamma dt in the interior (div v = 0, no rotation term
    with s = 0), with G = 0.6 rho c^2 (Poisson ratio 0.25) times the softening
    (E_cv - E) / (E_cv - E_iv) clipped to [0, 1]: 1 at E = 0, 1/2 halfway
    between E_iv and E_cv, 0 above E_cv. Checked in a compressed and an
    expanded state and at rest (where G = 10.8 GPa). A modulus that ignored
    the local bulk modulus (constant 0.6 A), a softening of the wrong sign or
    slope, or a missing factor 2 in 2G e_rz fails."""
    fr, energy = state
    mat = inputs.basalt(strength=True)
    E = {"cold": 0.0, "mid": 0.5 * (mat.Eiv + mat.Ecv), "hot": 1.2 * mat.Ecv}[energy]
    soft = {"cold": 1.0, "mid": 0.5, "hot": 0.0}[energy]
    r = fr * mat.rho0
    g = grid(top_closed=1, dt_max=1.0)
    pb = inputs.Problem(grid=g, mats=[mat], pml=inputs.Pml(enabled=0))
    gamma, dt = 10.0, 1e-6
    rho = np.full((g.NZ, g.NR), r)
    I = np.full_like(rho, E)
    f = np.ones((1, g.NZ, g.NR))
    v = np.zeros((2, g.NZ + 1, g.NR + 1))
    v[1] = gamma * np.arange(g.NR + 1)[None, :] * g.dr
    v[1, 0, :] = 0.0
    _, F1 = one_cycle(pb, rho, I, f, v, dt)
    js, is_ = interior(g)
    G_hand = 0.6 * r * c2_by_differences(mat, r, E) * soft
    srz = F1["s"][2][js, is_]
    if soft == 0.0:
        assert np.all(srz == 0.0)
    else:
        np.testing.assert_allclose(srz, G_hand * gamma * dt, rtol=1e-6)
    if state == (1.0, "cold"):
        np.testing.assert_allclose(srz, 10.8e9 * gamma * dt, rtol=1e-12)
    # no normal deviator from a pure shear
    assert np.max(np.abs(F1["s"][0][js, is_])) <= 1e-12 * max(abs(G_hand) * gamma * dt, 1.0)
