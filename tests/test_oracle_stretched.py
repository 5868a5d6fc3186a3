"""Pins of the oracle on stretched grids (Table 2's extension zones).

What fixes the stretched-grid code other than itself:

  * the layout of Table 2 (512 x 532 cells, 400 m fine zone, growth 1.05 per
    cell capped at 1061 m, a 231 km radial extent);
  * the geometry tables are running sums with centres halfway, and each
    cell's volume is the sum of its two r-weighted half areas times its height;
  * a "stretched" grid whose widths are all equal (and exactly representable)
    reproduces the uniform grid bit for bit: the table path against the
    uniform path, which has pins of its own;
  * the strain rates are exact for linear velocity fields on unequal columns
    and rows;
  * rest, uniform translation and a uniform velocity over any mass field stay
    exactly as they are; mass is conserved exactly and energy nearly so in a
    closed box, and the mass budget closes with outflow and PML;
  * the extension zone keeps an impact's crater: the stretched layout agrees
    with a uniform grid of the same fine zone before anything returns from the
    outer boundary.
"""
import numpy as np
import pytest

from oracle import oracle as O
from oracle.oracle import Oracle
from paper_2403_04267_amd import inputs

from .crater import crater_depth, crater_radius


def full_state(g, rho0):
    rho = np.full((g.NZ, g.NR), rho0)
    I = np.zeros((g.NZ, g.NR))
    f = np.ones((g.nmat, g.NZ, g.NR))
    v = np.zeros((2, g.NZ + 1, g.NR + 1))
    return rho, I, f, v


def small_grid(n=24, ext=8, pml=6, **kw):
    return inputs.paper_layout(n, n, (0, ext, ext, ext), (pml, pml), d=4.0, d_max=9.0, nmat=1, **kw)


def test_table2_layout():
    g = inputs.paper_layout()
    assert (g.NR, g.NZ) == (512, 532)
    cols, rows = np.array(g.dr_col), np.array(g.dz_row)
    assert np.all(cols[:462] == 400.0) and cols.max() == 1061.0
    assert np.all(cols[482:] == 1061.0)          # the radial PML at the largest spacing
    assert np.all(np.diff(cols[461:482]) > 0)    # growth through the extension zone
    assert sum(cols) / 1e3 == pytest.approx(231.0, abs=1.0)  # Table 2's radial extent
    assert np.all(rows[:30] == 1061.0) and np.all(rows[50:512] == 400.0)


def test_table2_vertical_extent_reading():
    """Table 2 prints y in [-181, 48.6] km (229.6 km) beside extension counts
    (0, 20, 20, 20) and a 30-row PML below. With the top zone of 20 rows the
    counts give 244.4 km; without it, 230.5 km (the radial extent, printed
    231 km, is 230.5 km too). Only the layout without the top zone fits the
    printed range; the default keeps the printed counts."""
    with_top = inputs.paper_layout()
    no_top = inputs.paper_layout(ext=(0, 20, 0, 20))
    assert sum(with_top.dz_row) / 1e3 == pytest.approx(244.4, abs=0.05)
    assert sum(no_top.dz_row) / 1e3 == pytest.approx(181.0 + 48.6, abs=1.0)
    assert abs(sum(with_top.dz_row) / 1e3 - 229.6) > 14.0
    assert sum(no_top.dr_col) == sum(with_top.dr_col)


def test_geometry_tables():
    g = small_grid()
    o = Oracle(inputs.Problem(grid=g, mats=[inputs.basalt()], pml=inputs.Pml(enabled=0)))
    rn, rc, zn, zc = o.geometry()
    assert rn[0] == 0.0 and zn[0] == 0.0
    assert np.allclose(np.diff(rn), g.dr_col, rtol=1e-14) and np.allclose(np.diff(zn), g.dz_row, rtol=1e-14)
    assert np.allclose(rc, rn[:-1] + 0.5 * np.array(g.dr_col), rtol=1e-15)
    assert np.allclose(zc, zn[:-1] + 0.5 * np.array(g.dz_row), rtol=1e-15)
    # the cell volume (mass per density) is the r-weighted area times the height
    rho, I, f, v = full_state(g, 1.0)
    o.set_fields(rho, I, f, v)
    V = 0.5 * (rn[1:] ** 2 - rn[:-1] ** 2)[None, :] * np.array(g.dz_row)[:, None]
    assert o.diag()["mass"] == pytest.approx(V.sum(), rel=1e-13)


def test_equal_widths_reproduce_the_uniform_grid_bitwise():
    pb = inputs.impact(30, 8, 4, 9e3, nmat=2, strength=True, cycles=0, dx=4.0)
    g = pb.grid
    st = pb.replace(grid=inputs.Grid(**{**g.__dict__, "dr_col": [4.0] * g.NR, "dz_row": [4.0] * g.NZ}))
    a, b = Oracle(pb), Oracle(st)
    for n in (1, 80):
        a.step(n)
        b.step(n)
        Fa, Fb = a.fields(), b.fields()
        for k in Fa:
            assert np.array_equal(Fa[k], Fb[k]), (n, k)
        Pa, Pb = a.pml_aux(), b.pml_aux()
        for k in Pa:
            assert np.array_equal(Pa[k], Pb[k]), (n, k)


@pytest.mark.parametrize("i,j", [(0, 2), (3, 9), (25, 30), (30, 35)])
def test_kinematics_exact_for_linear_fields_on_stretched_cells(i, j):
    g = small_grid()
    rn = np.concatenate([[0.0], np.cumsum(g.dr_col)])
    zn = np.concatenate([[0.0], np.cumsum(g.dz_row)])
    a, b, c, d, h = 0.31, -0.17, 0.23, -0.41, 5.0
    rs = np.array([rn[i], rn[i + 1], rn[i], rn[i + 1]])
    zs = np.array([zn[j], zn[j], zn[j + 1], zn[j + 1]])
    k = O.cell_kinematics(g, i, a * rs + b * zs, c * rs + d * zs + h, j=j)
    rc, zc = 0.5 * (rn[i] + rn[i + 1]), 0.5 * (zn[j] + zn[j + 1])
    assert k["err"] == pytest.approx(a, rel=1e-12, abs=1e-14)
    assert k["ezz"] == pytest.approx(d, rel=1e-12, abs=1e-14)
    assert k["ett"] == pytest.approx((a * rc + b * zc) / rc, rel=1e-12)
    assert k["erz"] == pytest.approx(0.5 * (b + c), rel=1e-12)
    assert k["om"] == pytest.approx(0.5 * (b - c), rel=1e-12)
    assert k["D"] == pytest.approx(k["err"] + k["ezz"] + k["ett"], rel=1e-12, abs=1e-14)


def test_rest_state_bitwise_with_pml():
    g = small_grid()
    mat = inputs.basalt()
    o = Oracle(inputs.Problem(grid=g, mats=[mat], pml=inputs.Pml()))
    rho, I, f, v = full_state(g, mat.rho0)
    rho[30:] = 0.0
    f[0, 30:] = 0.0
    o.set_fields(rho, I, f, v)
    o.step(40)
    F = o.fields(eos=False)
    assert np.array_equal(F["rho"], rho) and np.array_equal(F["v"], v) and np.array_equal(F["f"], f)


def test_uniform_translation_away_from_the_wall():
    g = inputs.paper_layout(10, 60, (0, 4, 10, 0), (0, 0), d=4.0, d_max=9.0, nmat=1)
    mat = inputs.basalt()
    o = Oracle(inputs.Problem(grid=g, mats=[mat], pml=inputs.Pml(enabled=0)))
    rho, I, f, v = full_state(g, mat.rho0)
    v[1, 1:] = 300.0
    o.set_fields(rho, I, f, v)
    o.step(6)
    F = o.fields(eos=False)
    jmin = 5 * 6 + 2
    assert np.array_equal(F["rho"][jmin:], rho[jmin:])
    assert np.array_equal(F["v"][1, jmin:], v[1, jmin:])
    assert not np.any(F["v"][0, jmin:])


def test_momentum_remap_keeps_uniform_velocity_with_any_mass_field():
    g = small_grid(pml=0)
    mat = inputs.basalt()
    o = Oracle(inputs.Problem(grid=g, mats=[mat], pml=inputs.Pml(enabled=0)))
    rng = np.random.default_rng(5)
    rho, I, f, v = full_state(g, mat.rho0)
    phi = rng.uniform(0.2, 1.0, size=rho.shape)
    f[0] = phi
    rho = 0.9 * mat.rho0 * phi * rng.uniform(0.8, 1.0, size=rho.shape)
    v[1, 1:] = -750.0
    o.set_fields(rho, I, f, v)
    o.step(3)
    F = o.fields(eos=False)
    assert np.all(F["v"][1, 4:] == -750.0)
    assert not np.any(F["v"][0, 4:])


def test_conservation_in_a_closed_box():
    """Mass exactly; total energy as well as on the uniform grid with the same
    cell counts (the same impact converts ~80 % of its kinetic energy to heat
    in a box this small; the stretched zone may add at most 0.5 % drift)."""
    pb = inputs.stretched_impact(30, 8, 0, 4, 8e3, d=4.0)
    pb.grid.top_closed = 1
    pb.pml.enabled = 0
    g = pb.grid
    uni = pb.replace(grid=inputs.Grid(**{**g.__dict__, "dr_col": [4.0] * g.NR, "dz_row": [4.0] * g.NZ}))
    drift = {}
    for name, p in (("stretched", pb), ("uniform", uni)):
        o = Oracle(p)
        d0 = o.diag()
        E0 = d0["ie"] + d0["ke"]
        for _ in range(3):
            o.step(100)
            d = o.diag()
            assert abs(d["mass"] - d0["mass"]) <= 1e-13 * d0["mass"], name
        assert d["ke"] < 0.3 * E0, name  # a real conversion took place
        drift[name] = abs(d["ie"] + d["ke"] - E0) / E0
    assert drift["uniform"] < 0.03
    assert drift["stretched"] <= drift["uniform"] + 0.005, drift


def test_mass_budget_with_outflow_and_pml():
    o = Oracle(inputs.stretched_impact(30, 8, 8, 4, 15e3, d=4.0))
    m0 = o.diag()["mass"]
    o.step(300)
    d = o.diag()
    assert d["mass_out"] > 0.0 and d["mass_pml"] != 0.0
    assert abs(d["mass"] + d["mass_out"] + d["mass_pml"] - m0) <= 1e-13 * m0


def test_extension_zone_keeps_the_crater():
    """Same fine zone and impact, with a stretched extension zone + PML and
    with a uniform grid large enough that nothing returns in time: the crater
    depth and radius agree within one fine cell."""
    n, R, v = 48, 4, 10e3
    st = inputs.stretched_impact(n, 12, 10, R, v, strength=False, nmat=1, d=4.0)
    big_n = 3 * n
    big = inputs.impact(big_n, 0, R, v, nmat=1, strength=False, cycles=0, dx=4.0)
    big.pml.enabled = 0
    a = Oracle(st)
    a.step(150)
    t = a.diag()["t"]  # the same stop time on the uniform grid
    b = Oracle(big.replace(grid=inputs.Grid(**{**big.grid.__dict__, "t_stop": t})))
    while b.diag()["t"] < t * (1 - 1e-12):
        b.step(50)
    sa = st.scene.surface_j - (st.grid.pml_b + 12)  # rows below the surface in the fine zone
    Fa, Fb = a.fields(eos=False), b.fields(eos=False)
    ga = inputs.Grid(n_r=n, n_z=sa + 40, dr=4.0, dz=4.0)
    fa = Fa["f"][:, st.grid.pml_b + 12:st.grid.pml_b + 12 + sa + 40, :n]
    fb = Fb["f"][:, big.scene.surface_j - sa:big.scene.surface_j + 40, :n]
    da, db = crater_depth(fa, ga, sa), crater_depth(fb, ga, sa)
    ra, rb = crater_radius(fa, ga, sa), crater_radius(fb, ga, sa)
    assert da > 2 * 4.0 and abs(da - db) <= 4.0, (da, db)
    assert abs(ra - rb) <= 4.0, (ra, rb)


def test_paper_study_window_is_shared_cell_for_cell():
    """The Table 2 PML comparison relies on the window (fine zone plus its
    first 20 extension cells) being the same cells in all three grids, with
    the same scene and lithostatic column relative to it."""
    from paper_2403_04267_amd.pml_study import PaperSetup, paper_problems
    probs, rows, wc, wr = paper_problems(PaperSetup())
    a, r = probs["pml"], probs["ref"]
    assert np.array_equal(np.array(a.grid.dr_col[:wc]), np.array(r.grid.dr_col[:wc]))
    ra, rr = rows["pml"], rows["ref"]
    assert np.array_equal(np.array(a.grid.dz_row[ra:ra + wr]), np.array(r.grid.dz_row[rr:rr + wr]))
    assert a.scene.surface_j - ra == r.scene.surface_j - rr
    assert a.scene.layer_j - ra == r.scene.layer_j - rr
    assert a.scene.layer2_j - ra == r.scene.layer2_j - rr and a.grid.nmat == r.grid.nmat == 3
    assert probs["bare"].grid == a.grid and not probs["bare"].pml.enabled and a.pml.enabled
    # a wave at 6.5 km/s needs over 50 s to cross the reference's extra zone
    # below the window and come back (the comparisons stop at 40 s)
    depth = sum(r.grid.dz_row[:rr])
    assert 2 * depth / 6.5e3 > 50.0
