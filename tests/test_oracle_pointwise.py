"""Pins of the oracle's point functions against closed forms, finite
differences, textbook special cases and exact kinematics.

Equation of state: four-region Tillotson (the paper's EoS module is inherited
from SALEc, Sec. 2). Strength: intact-rock yield curve with the Table 1
parameters (cohesion, friction, limiting strength). Kinematics and the
constitutive update feed eqs. (1)-(2).
"""
import math

import numpy as np
import pytest

from oracle import oracle as O
from paper_2403_04267_amd import inputs

BAS = inputs.basalt()
BAS_S = inputs.basalt(strength=True)


# ---------------------------------------------------------------- EoS
def test_reference_state_has_zero_pressure():
    p, c2 = O.tillotson(BAS, BAS.rho0, 0.0)
    assert p == 0.0
    # bulk sound speed at the reference state: c^2 = A / rho0
    assert c2 == pytest.approx(BAS.A / BAS.rho0, rel=1e-15)


def test_cold_compression_hand_value():
    # rho = 1.1 rho0, E = 0: p = A mu + B mu^2 = 18e9 * 0.1 + 18e9 * 0.01 = 1.98 GPa
    p, _ = O.tillotson(BAS, 1.1 * BAS.rho0, 0.0)
    assert p == pytest.approx(1.98e9, rel=1e-13)


@pytest.mark.parametrize("E", [1e6, 5e6, 1e7, 2e7, 1e8])
def test_continuous_across_reference_density(E):
    # the compressed and expanded forms meet at rho = rho0 for every E
    pa, _ = O.tillotson(BAS, BAS.rho0 * (1 + 1e-12), E)
    pb, _ = O.tillotson(BAS, BAS.rho0 * (1 - 1e-12), E)
    assert abs(pa - pb) <= 1e-9 * max(abs(pa), 1.0)


@pytest.mark.parametrize("eta", [0.3, 0.6, 0.9, 0.99])
def test_continuous_across_energy_thresholds(eta):
    rho = eta * BAS.rho0
    for Eb in (BAS.Eiv, BAS.Ecv):
        lo, _ = O.tillotson(BAS, rho, Eb * (1 - 1e-12))
        hi, _ = O.tillotson(BAS, rho, Eb * (1 + 1e-12))
        assert abs(lo - hi) <= 1e-8 * max(abs(lo), 1.0)


@pytest.mark.parametrize("rho_f,E", [
    (1.8, 1.25e7),    # compressed (region I)
    (1.1, 0.0),       # compressed, cold
    (0.8, 1e6),       # cold expanded (region II)
    (0.7, 3e7),       # hot expanded (region III)
    (0.5, 1e8),       # hot expanded, strongly
    (0.9, 1e7),       # blend (region IV)
    (0.6, 1.5e7),     # blend (region IV)
])
def test_sound_speed_matches_finite_differences(rho_f, E):
    """c^2 = dp/drho|_E + p / rho^2 dp/dE|_rho, with the derivatives taken by
    central differences of the oracle's own pressure."""
    rho = rho_f * BAS.rho0
    p, c2 = O.tillotson(BAS, rho, E)
    hr, hE = rho * 1e-6, max(E, 1e3) * 1e-6
    dpdr = (O.tillotson(BAS, rho + hr, E)[0] - O.tillotson(BAS, rho - hr, E)[0]) / (2 * hr)
    if E > 0:
        dpdE = (O.tillotson(BAS, rho, E + hE)[0] - O.tillotson(BAS, rho, E - hE)[0]) / (2 * hE)
    else:  # the EoS sees max(E, 0): one-sided second-order difference
        dpdE = (-3 * p + 4 * O.tillotson(BAS, rho, hE)[0] - O.tillotson(BAS, rho, 2 * hE)[0]) / (2 * hE)
    fd = dpdr + p / rho ** 2 * dpdE
    assert c2 == pytest.approx(fd, rel=2e-6)


def test_sound_speed_literature_point():
    # shocked basalt state on the 10 km/s symmetric-impact Hugoniot
    _, c2 = O.tillotson(BAS, 5236.4, 12.5e6)
    assert math.sqrt(c2) == pytest.approx(10069.0, rel=2e-4)


@pytest.mark.parametrize("rho,E", [(0.125, 2.0), (1.0, 2.5), (0.5, 1.2), (3.0, 0.7), (1e-3, 5.0)])
def test_ideal_gas_reduction(rho, E):
    """a = gamma-1, b = A = B = 0 makes every Tillotson region p = (gamma-1) rho E
    and c^2 = gamma (gamma-1) E."""
    g = inputs.ideal_gas(1.4)
    p, c2 = O.tillotson(g, rho, E)
    assert p == pytest.approx(0.4 * rho * E, rel=1e-15)
    assert c2 == pytest.approx(1.4 * 0.4 * E, rel=1e-14)


# ---------------------------------------------------------------- strength
def test_yield_curve_shape():
    m = BAS_S
    assert O.yield_strength(m, 0.0) == m.Y0
    # slope mu at p = 0 from both sides (continuous, smooth)
    h = 1.0
    sp = (O.yield_strength(m, h) - m.Y0) / h
    sn = (m.Y0 - O.yield_strength(m, -h)) / h
    assert sp == pytest.approx(m.mu_f, rel=1e-6)
    assert sn == pytest.approx(m.mu_f, rel=1e-6)
    # limit strength at high pressure
    assert O.yield_strength(m, 1e15) == pytest.approx(m.Ylim, rel=1e-4)
    # zero at the tension cut-off p = -Y0 / mu and below
    assert O.yield_strength(m, -m.Y0 / m.mu_f) == 0.0
    assert O.yield_strength(m, -1e9) == 0.0
    # hydrodynamic material has no strength
    assert O.yield_strength(BAS, 1e9) == 0.0


def test_shear_modulus_from_poisson_ratio():
    # G = 3 K (1 - 2 nu) / (2 (1 + nu)), K = A = 18 GPa, nu = 0.25 -> 10.8 GPa
    assert O.shear_modulus(BAS_S) == pytest.approx(10.8e9, rel=1e-15)
    assert O.shear_modulus(BAS) == 0.0


# ---------------------------------------------------------------- kinematics
@pytest.mark.parametrize("i", [0, 1, 7, 40])
def test_kinematics_exact_for_linear_fields(i):
    """v_r = a r + b z + e, v_z = c r + d z + h is reproduced exactly (up to
    rounding) by the face-mean strain rates, including the hoop rate v_r / r."""
    g = inputs.Grid(n_r=64, n_z=8, dr=0.7, dz=1.3)
    a, b, c, d, e, h = 0.31, -0.17, 0.23, -0.41, 0.0, 5.0
    j = 3
    rs = np.array([i, i + 1, i, i + 1]) * g.dr
    zs = np.array([j, j, j + 1, j + 1]) * g.dz
    vr = a * rs + b * zs + e
    vz = c * rs + d * zs + h
    k = O.cell_kinematics(g, i, vr, vz)
    rc, zc = (i + 0.5) * g.dr, (j + 0.5) * g.dz
    assert k["err"] == pytest.approx(a, rel=1e-12, abs=1e-14)
    assert k["ezz"] == pytest.approx(d, rel=1e-12, abs=1e-14)
    assert k["ett"] == pytest.approx((a * rc + b * zc) / rc, rel=1e-12)
    assert k["erz"] == pytest.approx(0.5 * (b + c), rel=1e-12)
    assert k["om"] == pytest.approx(0.5 * (b - c), rel=1e-12)
    # flux-form divergence equals the trace of the strain rate
    assert k["D"] == pytest.approx(k["err"] + k["ezz"] + k["ett"], rel=1e-12, abs=1e-14)


# ---------------------------------------------------------------- constitutive update
def test_elastic_increment_is_2G_deviatoric_strain():
    rates = np.array([1e-3, -2e-3, 5e-4, 7e-4, 0.0])
    G, dt = 10.8e9, 1e-4
    s = O.stress_update(G, 1e30, dt, rates, [0.0, 0.0, 0.0])
    tr = rates[0] + rates[1] + rates[2]
    assert s[0] == pytest.approx(2 * G * (rates[0] - tr / 3) * dt, rel=1e-14)
    assert s[1] == pytest.approx(2 * G * (rates[1] - tr / 3) * dt, rel=1e-14)
    assert s[2] == pytest.approx(2 * G * rates[3] * dt, rel=1e-14)


def test_radial_return_onto_yield_surface():
    rng = np.random.default_rng(7)
    for _ in range(200):
        rates = rng.normal(size=5) * 1e-2
        s0 = rng.normal(size=3) * 1e8
        Y = abs(rng.normal()) * 5e7
        s = O.stress_update(10.8e9, Y, 1e-3, rates, s0)
        J2 = s[0] ** 2 + s[1] ** 2 + s[0] * s[1] + s[2] ** 2
        assert math.sqrt(3 * J2) <= Y * (1 + 1e-14)


def test_jaumann_rotation_matches_rigid_rotation():
    """A stress carried by a rigid rotation of spin W_rz = omega must rotate
    with the material: s(t) = R s0 R^T, R = [[cos wt, sin wt], [-sin wt, cos wt]]
    (the rotation generated by v_r = omega z, v_z = -omega r). Forward Euler
    converges to it at first order and J2 grows by at most (omega dt)^2 per step."""
    om, T = 1.0, math.pi / 4
    s_rr, s_zz, s_rz = 2e8, -1e8, 0.0
    s0 = np.array([s_rr, s_zz, s_rz])
    errs = []
    for nsteps in (200, 400):
        dt = T / nsteps
        s = s0.copy()
        J2_prev = s[0] ** 2 + s[1] ** 2 + s[0] * s[1] + s[2] ** 2
        for _ in range(nsteps):
            s = O.stress_update(0.0, 1e30, dt, [0, 0, 0, 0, om], s)
            J2 = s[0] ** 2 + s[1] ** 2 + s[0] * s[1] + s[2] ** 2
            assert J2 <= J2_prev * (1 + (om * dt) ** 2 * 4.0 + 1e-15)
            J2_prev = J2
        c, sn = math.cos(om * T), math.sin(om * T)
        R = np.array([[c, sn], [-sn, c]])
        S0 = np.array([[s_rr, s_rz], [s_rz, s_zz]])
        St = R @ S0 @ R.T
        errs.append(max(abs(s[0] - St[0, 0]), abs(s[1] - St[1, 1]), abs(s[2] - St[0, 1])) / 2e8)
    assert errs[0] < 0.02
    assert errs[1] < 0.6 * errs[0]  # first-order convergence


def test_spin_sign_from_rigid_rotation_velocity_field():
    # v_r = omega z, v_z = -omega r gives omega (spin) = +omega and zero strain rate
    g = inputs.Grid(n_r=32, n_z=8)
    om = 0.37
    i, j = 5, 2
    rs = np.array([i, i + 1, i, i + 1]) * g.dr
    zs = np.array([j, j, j + 1, j + 1]) * g.dz
    k = O.cell_kinematics(g, i, om * zs, -om * rs)
    assert k["om"] == pytest.approx(om, rel=1e-14)
    assert abs(k["erz"]) < 1e-15 and abs(k["err"]) < 1e-15 and abs(k["ezz"]) < 1e-15


# ---------------------------------------------------------------- exp
def test_exp_method_accuracy():
    """The EoS exponentials use Cody-Waite reduction + degree-13 Taylor
    polynomial: within 2 ulp of the correctly rounded value over the range the
    EoS uses, exact at 0, flushed to 0 below e^-700, monotone."""
    import numpy as np
    xs = np.concatenate([np.linspace(-700, 709, 20001), np.linspace(-1, 1, 20001), -np.logspace(-12, 2.8, 5000)])
    for x in xs:
        y = O.exp(float(x))
        ref = math.exp(float(x))
        assert abs(y - ref) <= 2.5 * np.spacing(ref), (x, y, ref)
    assert O.exp(0.0) == 1.0
    assert O.exp(-701.0) == 0.0 and O.exp(-1e12) == 0.0
    assert math.isinf(O.exp(710.0))
    ys = [O.exp(float(x)) for x in np.linspace(-5, 5, 10001)]
    assert all(b >= a for a, b in zip(ys, ys[1:]))
