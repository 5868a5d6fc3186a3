"""Pins of damage and acoustic fluidization in the oracle (-m "not gpu").

Table 1 lists the damaged material's cohesion, friction and limit and the
block model's gamma_eta, gamma_T and c_vib; the paper gives no equations,
so the oracle follows these readings:
  strength  Y = (1 - D) Y_i(p) + D Y_d, Y_d = min(Y_d0 + mu_d q, Y_dm) at
            q = max(p - p_vib, 0) (p >= 0), max(0, Y_d0 + mu_d p) in tension,
            never above Y_i; p_vib = rho c v_vib (c: longitudinal speed at rest)
  damage    D += (plastic strain of the radial return, (trial - yield) / 3G)
            / max(eps_fb, B (p - p_bd)), capped at 1, advected with the mass
  block     v_vib decays as exp(-dt / T), T = gamma_T h / c, and is excited
            to c_vib times the largest corner speed; the damaged rock's flow
            stress exceeds Y by 3 eta eps_eq, eta = rho gamma_eta c h (weight D,
            ramped in over 1 mm/s of vibration)
Each test fails on a named plausible mistake.
"""
import math

import numpy as np
import pytest

from oracle.oracle import Oracle, failure_strain, shear_modulus, yield_damaged, yield_strength
from paper_2403_04267_amd import inputs

N = 14


def interior(g):
    return slice(3, g.NZ - 3), slice(1, g.NR - 3)


def rock(**kw):
    m = inputs.basalt(strength=True)
    d = dict(Yd0=0.01e6, mu_d=0.6, Ydm=2.5e9, gamma_eta=0.0, gamma_T=0.0, c_vib=0.0, af_h=0.0)
    d.update(kw)
    return inputs.with_damage(m, **d)


def c_long(m):
    return math.sqrt((m.A + 4.0 / 3.0 * shear_modulus(m)) / m.rho0)


# ---------------------------------------------------------------- strength blend
def test_damaged_yield_blend_hand_values():
    """D = 0 gives the intact curve, D = 1 the damaged Coulomb line capped
    at Y_dm (and at the intact value), D = 1/2 their mean; the vibration
    pressure lowers only the damaged part; tension uses the plain line.
    Fails on a swapped blend, the cap applied to the intact part, or p_vib
    acting on the intact curve."""
    m = rock()
    for p in (0.0, 5e7, 1e9, 2e10):
        Yi = yield_strength(m, p)
        Yd = min(min(m.Yd0 + m.mu_d * p, m.Ydm), Yi)
        assert yield_damaged(m, p, 0.0, 0.0) == Yi
        assert yield_damaged(m, p, 1.0, 0.0) == Yd
        assert yield_damaged(m, p, 0.5, 0.0) == pytest.approx(0.5 * (Yi + Yd), rel=1e-15)
    # 1 GPa with a vibration pressure of 0.4 GPa: the damaged line at 0.6 GPa
    assert yield_damaged(m, 1e9, 1.0, 4e8) == pytest.approx(m.Yd0 + m.mu_d * 6e8, rel=1e-15)
    assert yield_damaged(m, 1e9, 0.0, 4e8) == yield_strength(m, 1e9)
    # vibration beyond the overburden leaves only the cohesion
    assert yield_damaged(m, 1e9, 1.0, 2e9) == m.Yd0
    # tension: max(0, Y_d0 + mu_d p)
    assert yield_damaged(m, -1e4, 1.0, 0.0) == pytest.approx(m.Yd0 - m.mu_d * 1e4, rel=1e-15)
    assert yield_damaged(m, -1e6, 1.0, 0.0) == 0.0
    # without damage the intact curve whatever D is
    assert yield_damaged(inputs.basalt(strength=True), 1e9, 1.0, 0.0) == yield_strength(
        inputs.basalt(strength=True), 1e9)


def test_failure_strain_hand_values():
    """eps_f = max(eps_fb, B (p - p_bd)): 1e-4 below the brittle-ductile
    transition, growing by 1e-11 per Pa above it (1e-2 at 1.3 GPa)."""
    m = rock()
    assert failure_strain(m, 0.0) == 1e-4
    assert failure_strain(m, 3e8) == 1e-4
    assert failure_strain(m, 1.3e9) == pytest.approx(1e-2, rel=1e-12)


# ---------------------------------------------------------------- one step
def shear_cycle(m, D0, vib0, gamma, dt, rho_fac=1.1):
    """One forced cycle of the simple shear v_z = gamma r of a uniform full
    state (rho = rho_fac rho0, I = 0, s = 0) with damage D0, vibration vib0."""
    g = inputs.Grid(n_r=N, n_z=N, top_closed=1, dt_max=1.0)
    pb = inputs.Problem(grid=g, mats=[m], pml=inputs.Pml(enabled=0))
    o = Oracle(pb)
    rho = np.full((g.NZ, g.NR), rho_fac * m.rho0)
    v = np.zeros((2, g.NZ + 1, g.NR + 1))
    v[1] = gamma * np.arange(g.NR + 1)[None, :] * g.dr
    v[1, 0, :] = 0.0
    o.set_fields(rho, np.zeros_like(rho), np.ones((1, g.NZ, g.NR)), v)
    o.set_damage(np.full_like(rho, D0), np.full_like(rho, vib0))
    o.set_clock(0.0, dt)
    F0 = o.fields()
    o.step(1)
    return F0, o.fields(), o.damage(), g


def test_damage_grows_by_the_plastic_strain_over_the_failure_strain():
    """An intact, compressed cell sheared past its yield in one step: the
    trial equivalent stress sqrt(3) G gamma dt exceeds Y, the return leaves
    the plastic strain (trial - Y) / 3G, and D grows by that over eps_f(p).
    Fails on a missing 3 in 3G, on eps_f taken at the wrong pressure, or on
    damage from the elastic part."""
    m = rock()
    gamma, dt = 430.0, 1e-4  # trial stress ~1.2 GPa against Y ~1 GPa
    F0, F1, Dm, g = shear_cycle(m, 0.0, 0.0, gamma, dt)
    js, is_ = interior(g)
    p = F0["p"][js, is_]
    # G and Y of the start state (c^2 = dp/drho + p/rho^2 dp/dE at E = 0)
    r = 1.1 * m.rho0
    mu = r / m.rho0 - 1.0
    c2 = (m.A + 2 * m.B * mu) / m.rho0 + p / r ** 2 * (r * (m.a + m.b))
    G = 0.6 * r * c2
    Y = np.array([yield_strength(m, q) for q in p.ravel()]).reshape(p.shape)
    trial = math.sqrt(3.0) * G * gamma * dt
    dep = (trial - Y) / (3.0 * G)
    eps_f = np.array([failure_strain(m, q) for q in p.ravel()]).reshape(p.shape)
    want = np.minimum(dep / eps_f, 1.0)
    assert np.all(want > 0.01) and np.all(want < 1.0)
    np.testing.assert_allclose(Dm["D"][js, is_], want, rtol=1e-10)
    # the returned stress sits on the (still intact) yield surface
    np.testing.assert_allclose(math.sqrt(3.0) * np.abs(F1["s"][2][js, is_]), Y, rtol=1e-10)


def test_elastic_step_leaves_damage_unchanged():
    m = rock()
    F0, F1, Dm, g = shear_cycle(m, 0.25, 0.0, 1.0, 1e-6)
    js, is_ = interior(g)
    assert np.all(Dm["D"][js, is_] == 0.25)


def test_bingham_viscosity_of_fluidized_damaged_rock():
    """Fully damaged rock vibrating faster than the overburden allows: the
    damaged strength is down to the cohesion Y_d0, and the block model's
    viscosity eta = rho gamma_eta c h adds 3 eta eps_eq = sqrt(3) eta gamma to
    the flow stress of the simple shear (eps_eq = gamma / sqrt(3)). So after
    one step sqrt(3) |s_rz| = Y_d0 + sqrt(3) eta gamma. Fails on a viscosity
    without the density, the block size or the factor 3."""
    h = 5.0  # the cap 3 eta eps_eq must stay below the elastic trial: eta < G dt
    m = rock(gamma_eta=0.08, gamma_T=50.0, c_vib=0.0, af_h=h)
    c = c_long(m)
    gamma, dt = 50.0, 1e-3
    r = 1.01 * m.rho0
    p_est = m.A * 0.01 + m.B * 1e-4
    vib0 = 10.0 * p_est / (r * c)  # vibration pressure 10x the overburden
    F0, F1, Dm, g = shear_cycle(m, 1.0, vib0, gamma, dt, rho_fac=1.01)
    js, is_ = interior(g)
    eta = r * m.gamma_eta * c * h
    want = m.Yd0 + math.sqrt(3.0) * eta * gamma
    np.testing.assert_allclose(math.sqrt(3.0) * np.abs(F1["s"][2][js, is_]), want, rtol=1e-10)


# ---------------------------------------------------------------- vibration
def test_vibration_decays_as_the_closed_form():
    """A damaged target at rest with a vibration speed v0 everywhere: with no
    flow nothing excites it, and v_vib(t) = v0 exp(-t / T), T = gamma_T h / c,
    to the rounding of the per-step factors. Fails on a decay per cycle
    instead of per time, or T without the block size."""
    h = 0.5
    m = rock(gamma_eta=0.0, gamma_T=115.0, c_vib=0.1, af_h=h)
    T = m.gamma_T * h / c_long(m)
    g = inputs.Grid(n_r=N, n_z=N, top_closed=1)
    pb = inputs.Problem(grid=g, mats=[m], pml=inputs.Pml(enabled=0))
    o = Oracle(pb)
    rho = np.full((g.NZ, g.NR), m.rho0)
    o.set_fields(rho, np.zeros_like(rho), np.ones((1, g.NZ, g.NR)), np.zeros((2, g.NZ + 1, g.NR + 1)))
    o.set_damage(np.full_like(rho, 0.5), np.full_like(rho, 3.0))
    for _ in range(4):
        o.step(50)
        t = o.diag()["t"]
        vib = o.damage()["vib"]
        np.testing.assert_allclose(vib, 3.0 * math.exp(-t / T), rtol=1e-12)
    assert t / T > 1.0


def test_vibration_excited_by_the_flow():
    """Uniform upward flow at U through damaged rock: after one cycle the
    interior's vibration speed is c_vib U (from zero)."""
    m = rock(gamma_eta=0.0, gamma_T=115.0, c_vib=0.1, af_h=100.0)
    g = inputs.Grid(n_r=N, n_z=N, top_closed=0, dt_max=1.0)
    pb = inputs.Problem(grid=g, mats=[m], pml=inputs.Pml(enabled=0))
    o = Oracle(pb)
    rho = np.full((g.NZ, g.NR), m.rho0)
    v = np.zeros((2, g.NZ + 1, g.NR + 1))
    U = 30.0
    v[1, 1:, :] = U
    o.set_fields(rho, np.zeros_like(rho), np.ones((1, g.NZ, g.NR)), v)
    o.set_clock(0.0, 1e-5)
    o.step(1)
    js, is_ = interior(g)
    np.testing.assert_allclose(o.damage()["vib"][js, is_], 0.1 * U, rtol=1e-12)


# ---------------------------------------------------------------- impact
def test_damage_in_an_impact_stays_in_the_unit_interval_and_only_grows():
    """An impact into damaging rock in a closed box (no outflow, no layers):
    D stays within [0, 1] everywhere, the mass-weighted damage sum M D never
    decreases (the remap moves it with the mass, only the Lagrangian step
    adds to it), and the crater floor is damaged. Fails on damage advected
    by volume, a return that lowers D, or D leaving [0, 1]."""
    m = rock(gamma_eta=0.008, gamma_T=115.0, c_vib=0.1, af_h=6.0)
    pb = inputs.impact(40, 0, 4, 6e3, nmat=2, strength=True, cycles=0, name="damage")
    pb = pb.replace(mats=[m, m], grid=pb.grid, pml=inputs.Pml(enabled=0))
    pb.grid.top_closed = 1
    o = Oracle(pb)
    g = pb.grid
    V = (np.arange(g.NR) + 0.5)[None, :] * g.dr * g.dr * g.dz * np.ones((g.NZ, 1))
    last = 0.0
    for _ in range(12):
        o.step(10)
        Dm = o.damage()
        D = Dm["D"]
        assert np.all(D >= 0.0) and np.all(D <= 1.0)
        assert np.all(Dm["vib"] >= 0.0)
        md = float(np.sum(o.fields(eos=False)["rho"] * V * D))
        assert md >= last * (1 - 1e-13), (md, last)
        last = md
    sj = pb.scene.surface_j
    assert D[sj - 3, 0] > 0.5
    assert np.max(Dm["vib"]) > 0.0
