"""Problem definitions and seeded synthetic inputs.

This module only *describes* problems: grid sizes, material constants, the
impact scene and seeded parameter draws for ensembles. It holds none of the
method's arithmetic, so both the HIP library binding and the CPU oracle can
be driven from the same description without sharing any computation.

Workloads stand in for the paper's vertical-impact simulations (Sec. 4): a
spherical projectile hitting a half-space in axisymmetric r-z geometry, with
PML layers on the right and bottom edges (Table 2 lists the same layer
placement). The paper's Chicxulub set-up needs material laws it does not give,
so a basalt-like Tillotson half-space is used instead.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np


@dataclass
class Material:
    """Tillotson constants plus optional pressure-dependent strength (Table 1 form)."""
    rho0: float
    A: float
    B: float
    E0: float
    a: float
    b: float
    alpha: float
    beta: float
    Eiv: float
    Ecv: float
    p_min: float = 0.0
    c_floor_frac: float = 0.25
    strength: int = 0
    Y0: float = 0.0
    mu_f: float = 0.0
    Ylim: float = 0.0
    poisson: float = 0.25
    # damage and acoustic fluidization (Table 1's damaged cohesion, friction
    # and limit, and the block model's gamma_eta, gamma_T, c_vib); the damage
    # law's failure strain max(eps_fb, B_dmg (p - p_bd)) and the block size
    # af_h (m) are not in the paper
    damage: int = 0
    Yd0: float = 0.0
    mu_d: float = 0.0
    Ydm: float = 0.0
    eps_fb: float = 1e-4
    B_dmg: float = 1e-11
    p_bd: float = 3e8
    gamma_eta: float = 0.0
    gamma_T: float = 0.0
    c_vib: float = 0.0
    af_h: float = 0.0


@dataclass
class Grid:
    n_r: int
    n_z: int
    pml_r: int = 0
    pml_b: int = 0
    nmat: int = 1
    top_closed: int = 0
    # mixed cells: 0 = one material density and specific energy shared by the
    # materials of a cell, 1 = per-material densities and specific energies
    closure: int = 0
    dr: float = 1.0
    dz: float = 1.0
    cfl: float = 0.5
    dt_grow: float = 1.1
    dt_max: float = 1e30
    dt_floor: float = 0.0
    t_stop: float = 0.0
    q_lin: float = 0.25
    q_quad: float = 1.0
    # stretched grid: per-column widths (NR values) and per-row heights (NZ
    # values) in metres, or None for the uniform dr / dz
    dr_col: Optional[Sequence[float]] = None
    dz_row: Optional[Sequence[float]] = None

    @property
    def NR(self) -> int:
        return self.n_r + self.pml_r

    @property
    def NZ(self) -> int:
        return self.n_z + self.pml_b

    @property
    def ncells(self) -> int:
        return self.NR * self.NZ

    @property
    def nnodes(self) -> int:
        return (self.NR + 1) * (self.NZ + 1)


@dataclass
class Pml:
    enabled: int = 1
    R: float = 0.01
    c_ref: float = 0.0  # <= 0: the largest longitudinal speed at rest over the materials
    # 1: the layers also relax the deviatoric stress toward zero at the rate d
    # (an extension; Sec. 3 damps mass, momentum and energy only)
    damp_stress: int = 0
    # which step applies each auxiliary: 0 = psi in the Lagrangian and phi in
    # the Eulerian step (derived from the equations), 1 = Sec. 3's sentence
    # as printed (psi in the Eulerian, phi in the Lagrangian step)
    placement: int = 0
    # damped quantity: 0 = specific velocity and energy; 1 = rho v and rho I
    # as Sec. 3's control equations print them (the CPU oracle only)
    form: int = 0


@dataclass
class Scene:
    surface_j: int
    radius: float            # 0: no projectile
    v_imp: float
    subsample: int = 8
    gravity: float = 0.0     # m/s^2; > 0: lithostatic target (initial pressure p0)
    layer_j: int = 0         # two or three materials: rows below it are material 1
    layer2_j: int = 0        # three materials: rows below it are material 2 (<= layer_j)


@dataclass
class Problem:
    grid: Grid
    mats: List[Material]
    pml: Pml = field(default_factory=Pml)
    scene: Optional[Scene] = None
    cycles: int = 0
    precision: str = "fp64"  # "fp64" or "mixed"
    name: str = ""

    def replace(self, **kw) -> "Problem":
        return dataclasses.replace(self, **kw)


# --------------------------------------------------------------------------
# materials
# --------------------------------------------------------------------------
def basalt(strength: bool = False, Y0: float = 10e6, mu_f: float = 0.8,
           Ylim: float = 2.5e9) -> Material:
    """Basalt-like Tillotson half-space: rho0 = 2860 kg/m^3, A = B = 18 GPa,
    E0 = 487 MJ/kg; a, b, alpha, beta, Eiv, Ecv from the standard basalt set.
    With strength the tension floor is where the yield curve reaches zero."""
    m = Material(rho0=2860.0, A=18e9, B=18e9, E0=487e6, a=0.5, b=1.5, alpha=5.0,
                 beta=5.0, Eiv=4.72e6, Ecv=18.2e6, p_min=0.0, c_floor_frac=0.25)
    if strength:
        m.strength = 1
        m.Y0, m.mu_f, m.Ylim = Y0, mu_f, Ylim
        m.p_min = -Y0 / mu_f
    return m


def mantle_like(strength: bool = False, Y0: float = 10e6, mu_f: float = 0.8,
                Ylim: float = 3.5e9) -> Material:
    """Dense mantle-rock stand-in (the paper's Table 1 gives strength
    parameters only): rho0 = 3320 kg/m^3 and A = B = 131 GPa (a bulk sound
    speed of about 6.3 km/s), the other Tillotson constants as basalt."""
    m = Material(rho0=3320.0, A=131e9, B=131e9, E0=487e6, a=0.5, b=1.5, alpha=5.0,
                 beta=5.0, Eiv=4.72e6, Ecv=18.2e6, p_min=0.0, c_floor_frac=0.25)
    if strength:
        m.strength = 1
        m.Y0, m.mu_f, m.Ylim = Y0, mu_f, Ylim
        m.p_min = -Y0 / mu_f
    return m


def _with_strength(m: Material, Y0: float, mu_f: float, Ylim: float) -> Material:
    m.strength = 1
    m.Y0, m.mu_f, m.Ylim = Y0, mu_f, Ylim
    m.p_min = -Y0 / mu_f
    return m


def granite(strength: bool = True) -> Material:
    """Granite crust: the published Tillotson granite constants (rho0 = 2680
    kg/m^3, A = B = 18 GPa, E0 = 16 MJ/kg, a = 0.5, b = 1.3, alpha = beta = 5,
    Eiv = 3.5 MJ/kg, Ecv = 18 MJ/kg); with strength, Table 1's intact
    cohesion 10 MPa, friction 2.0 and limit 2.5 GPa."""
    m = Material(rho0=2680.0, A=18e9, B=18e9, E0=16e6, a=0.5, b=1.3, alpha=5.0,
                 beta=5.0, Eiv=3.5e6, Ecv=18e6, p_min=0.0, c_floor_frac=0.25)
    return _with_strength(m, 10e6, 2.0, 2.5e9) if strength else m


def dunite(strength: bool = True) -> Material:
    """Dunite mantle and projectile: the mantle-rock stand-in's Tillotson
    constants with Table 1's intact cohesion 10 MPa, friction 1.2 and limit
    3.5 GPa."""
    m = mantle_like(strength=False)
    return _with_strength(m, 10e6, 1.2, 3.5e9) if strength else m


def calcite(strength: bool = True) -> Material:
    """Calcite sediment stand-in (the paper gives strength parameters only):
    calcite's density 2710 kg/m^3 and A = B = 70 GPa (about calcite's bulk
    modulus), the other Tillotson constants as basalt; with strength, Table
    1's intact cohesion 5 MPa, friction 1.0 and limit 0.5 GPa."""
    m = Material(rho0=2710.0, A=70e9, B=70e9, E0=487e6, a=0.5, b=1.5, alpha=5.0,
                 beta=5.0, Eiv=4.72e6, Ecv=18.2e6, p_min=0.0, c_floor_frac=0.25)
    return _with_strength(m, 5e6, 1.0, 0.5e9) if strength else m


def with_damage(m: Material, Yd0: float, mu_d: float, Ydm: float, gamma_eta: float = 0.0,
                gamma_T: float = 0.0, c_vib: float = 0.0, af_h: float = 0.0) -> Material:
    """The same material with damage and, where gamma_eta, gamma_T or c_vib
    are nonzero, the block model of acoustic fluidization (block size af_h)."""
    m = dataclasses.replace(m)
    m.damage = 1
    m.Yd0, m.mu_d, m.Ydm = Yd0, mu_d, Ydm
    m.gamma_eta, m.gamma_T, m.c_vib, m.af_h = gamma_eta, gamma_T, c_vib, af_h
    return m


# Table 1's damaged-material and block-model constants per rock
TABLE1_DAMAGE = {
    "granite": dict(Yd0=0.01e6, mu_d=0.6, Ydm=2.5e9, gamma_eta=0.008, gamma_T=115.0, c_vib=0.1),
    "dunite": dict(Yd0=0.01e6, mu_d=0.6, Ydm=3.5e9, gamma_eta=0.08, gamma_T=50.0, c_vib=0.1),
    "calcite": dict(Yd0=0.01e6, mu_d=0.4, Ydm=0.5e9, gamma_eta=0.0, gamma_T=0.0, c_vib=0.0),
}


def ideal_gas(gamma: float = 1.4) -> Material:
    """Tillotson with a = gamma - 1 and b = A = B = 0 is exactly an ideal gas."""
    return Material(rho0=1.0, A=0.0, B=0.0, E0=1.0, a=gamma - 1.0, b=0.0, alpha=5.0,
                    beta=5.0, Eiv=1.0, Ecv=2.0, p_min=-1e300, c_floor_frac=0.0)


# --------------------------------------------------------------------------
# impact scenes
# --------------------------------------------------------------------------
def surface_row(n: int, pml_b: int, radius_cells: int) -> int:
    """Target surface row: leave 2R + max(4, ceil(R/2)) void rows above it."""
    h_void = 2 * radius_cells + max(4, math.ceil(radius_cells / 2))
    return pml_b + n - h_void


def impact(n: int, pml: int, radius_cells: int, v_imp: float, nmat: int, strength: bool,
           cycles: int, precision: str = "fp64", Y0: float = 10e6, name: str = "",
           dx: float = 1.0, cfl: float = 0.5) -> Problem:
    g = Grid(n_r=n, n_z=n, pml_r=pml, pml_b=pml, nmat=nmat, dr=dx, dz=dx, cfl=cfl)
    mat = basalt(strength=strength, Y0=Y0)
    mats = [mat] * nmat
    sc = Scene(surface_j=surface_row(n, pml, radius_cells), radius=radius_cells * dx, v_imp=v_imp)
    return Problem(grid=g, mats=mats, pml=Pml(), scene=sc, cycles=cycles, precision=precision,
                   name=name)


def layered_impact(n: int, pml: int, radius_cells: int, v_imp: float, crust_cells: int,
                   dx: float = 400.0, gravity: float = 9.81, strength: bool = True, cycles: int = 0,
                   precision: str = "fp64", name: str = "") -> Problem:
    """Vertical impact of a mantle-rock sphere on a two-layer target under
    gravity, the setting of Sec. 4 reduced to two materials: a basalt crust
    of crust_cells rows over a mantle-rock half-space (material 1, the
    projectile's), lithostatic initial pressure, PML right and below.
    Cells of dx metres (the paper's runs use 400 m)."""
    g = Grid(n_r=n, n_z=n, pml_r=pml, pml_b=pml, nmat=2, dr=dx, dz=dx)
    sj = surface_row(n, pml, radius_cells)
    sc = Scene(surface_j=sj, radius=radius_cells * dx, v_imp=v_imp, gravity=gravity,
               layer_j=max(sj - crust_cells, 0))
    return Problem(grid=g, mats=[basalt(strength=strength), mantle_like(strength=strength)], pml=Pml(),
                   scene=sc, cycles=cycles, precision=precision, name=name)


def three_layer_impact(n: int, pml: int, radius_cells: int, v_imp: float, sed_cells: int, crust_cells: int,
                       dx: float = 400.0, gravity: float = 9.81, strength: bool = True, cycles: int = 0,
                       precision: str = "fp64", name: str = "") -> Problem:
    """The three-layer target of Sec. 4 on an n x n uniform grid: sed_cells
    rows of calcite (material 0) over crust_cells rows of granite (material
    1) over a dunite half-space (material 2, also the projectile's),
    lithostatic under `gravity`, PML right and below. With dx = 400 m the
    paper's layers are 7 and 75 rows (2.8 km and 30 km)."""
    g = Grid(n_r=n, n_z=n, pml_r=pml, pml_b=pml, nmat=3, dr=dx, dz=dx)
    sj = surface_row(n, pml, radius_cells)
    lj = max(sj - sed_cells, 0)
    sc = Scene(surface_j=sj, radius=radius_cells * dx, v_imp=v_imp, gravity=gravity,
               layer_j=lj, layer2_j=max(lj - crust_cells, 0))
    return Problem(grid=g, mats=[calcite(strength), granite(strength), dunite(strength)], pml=Pml(),
                   scene=sc, cycles=cycles, precision=precision, name=name)


def stretched_widths(n_fine: int, n_ext: int, n_pml: int, d: float, factor: float = 1.05,
                     d_max: Optional[float] = None) -> List[float]:
    """Cell widths along one axis, outward (Table 2's zones): n_fine cells of
    d, n_ext extension cells each `factor` times the previous one (capped at
    d_max), then n_pml layer cells of the last width."""
    w = [float(d)] * n_fine
    cur = float(d)
    for _ in range(n_ext):
        cur = cur * factor
        if d_max is not None:
            cur = min(cur, float(d_max))
        w.append(cur)
    w += [w[-1] if w else float(d)] * n_pml
    return w


def paper_layout(n_x: int = 462, n_y: int = 462, ext=(0, 20, 20, 20), pml=(30, 30), d: float = 400.0,
                 factor: float = 1.05, d_max: float = 1061.0, nmat: int = 2) -> Grid:
    """The grid of Table 2: an n_x x n_y zone of d-metre cells, extension
    zones (left, right, top, bottom) whose spacing grows by `factor` per cell
    up to d_max, and PML layers (right, bottom) at the last spacing. The
    axis is the left side, so there is no left extension. Defaults: the
    paper's SALEc-2D+PML column, 512 x 532 cells."""
    n_l, n_r, n_t, n_b = ext
    p_r, p_b = pml
    if n_l:
        raise ValueError("the symmetry axis is the left side: no left extension")
    cols = stretched_widths(n_x, n_r, p_r, d, factor, d_max)
    below = stretched_widths(0, n_b, p_b, d, factor, d_max)[::-1]  # PML rows at the bottom
    above = stretched_widths(0, n_t, 0, d, factor, d_max)
    rows = below + [float(d)] * n_y + above
    return Grid(n_r=n_x + n_r, n_z=n_b + n_y + n_t, pml_r=p_r, pml_b=p_b, nmat=nmat, dr=d, dz=d,
                dr_col=cols, dz_row=rows)


def stretched_impact(n: int, ext: int, pml: int, radius_cells: int, v_imp: float, strength: bool = True,
                     nmat: int = 2, d: float = 400.0, precision: str = "fp64", name: str = "") -> Problem:
    """The impact scene on a Table 2-style grid: an n x n zone of d-metre
    cells with `ext` extension cells right, above and below (growth 1.05 per
    cell, capped at 1061 m) and `pml` layer cells right and below; the target
    surface and the projectile sit in the fine zone."""
    g = paper_layout(n, n, (0, ext, ext, ext), (pml, pml), d=d, nmat=nmat)
    sj = g.pml_b + ext + surface_row(n, 0, radius_cells)
    sc = Scene(surface_j=sj, radius=radius_cells * d, v_imp=v_imp)
    mat = basalt(strength=strength)
    return Problem(grid=g, mats=[mat] * nmat, pml=Pml(), scene=sc, precision=precision, name=name)


def config_paper(precision: str = "fp64") -> Problem:
    """Sec. 4's verification setting on Table 2's grid, with two
    materials: 512 x 532 cells (462 x 462 of 400 m, extension zones right, top
    and bottom growing 1.05 per cell to 1061 m, 30-cell PML right and below),
    a mantle-rock sphere of 7.2 km radius (18 cells) at 12 km/s onto a 33 km
    basalt crust over mantle rock, lithostatic under 9.81 m/s^2; Courant
    factor 0.2, the value Sec. 7 gives for this example."""
    g = paper_layout()
    g.cfl = 0.2
    R = 18
    sj = g.pml_b + 20 + surface_row(462, 0, R)
    sc = Scene(surface_j=sj, radius=R * 400.0, v_imp=12e3, gravity=9.81, layer_j=sj - 82)
    return Problem(grid=g, mats=[basalt(strength=True), mantle_like(strength=True)], pml=Pml(), scene=sc,
                   precision=precision, name="paper-layout")


def config_paper_layers(precision: str = "fp64") -> Problem:
    """Sec. 4's verification setting on Table 2's grid with its three layers:
    512 x 532 cells as in the two-material setting, a dunite sphere of 7.2 km
    radius (18 cells) at 12 km/s onto 2.8 km of calcite (7 rows) over 30 km of
    granite (75 rows) over dunite, with Table 1's intact strength,
    lithostatic under 9.81 m/s^2; Courant factor 0.2 as Sec. 7 gives."""
    g = paper_layout(nmat=3)
    g.cfl = 0.2
    R = 18
    sj = g.pml_b + 20 + surface_row(462, 0, R)
    sc = Scene(surface_j=sj, radius=R * 400.0, v_imp=12e3, gravity=9.81, layer_j=sj - 7,
               layer2_j=sj - 82)
    return Problem(grid=g, mats=[calcite(), granite(), dunite()], pml=Pml(), scene=sc,
                   precision=precision, name="paper-layers")


def config_small() -> Problem:
    """100x100 cells + 20-cell PML, one material, hydrodynamic, R = 10 cells,
    10 km/s, 500 cycles, plain FP64."""
    return impact(100, 20, 10, 10e3, nmat=1, strength=False, cycles=500, name="impact-100-hydro-fp64")


def config_scale() -> Problem:
    """1000x1000 cells + 50-cell PML, two materials with strength
    (Y0 = 10 MPa, friction 0.8, Ylim = 2.5 GPa), R = 50 cells, 15 km/s,
    5000 cycles, plain FP64."""
    return impact(1000, 50, 50, 15e3, nmat=2, strength=True, cycles=5000, name="impact-1000-strength-fp64")


def config_large(precision: str = "mixed") -> Problem:
    """4000x4000 cells + 100-cell PML, two materials with strength, R = 200
    cells, 12 km/s, 2000 cycles."""
    return impact(4000, 100, 200, 12e3, nmat=2, strength=True, cycles=2000, precision=precision,
                  name=f"impact-4000-strength-{precision}")


def ensemble(seed: int, n: int, side_lo: int, side_hi: int, cycles: int = 1000,
             precision: str = "fp64") -> List[Problem]:
    """Seeded ensemble of uneven impacts: side ~ U{side_lo..side_hi},
    R ~ U{5..40} cells, v ~ U(5, 20) km/s, Y0 ~ U(1, 50) MPa, PML = 10 % of
    the side (rounded), two materials with strength."""
    rng = np.random.default_rng(seed)
    side = rng.integers(side_lo, side_hi + 1, size=n)
    rad = rng.integers(5, 41, size=n)
    vel = rng.uniform(5e3, 20e3, size=n)
    y0 = rng.uniform(1e6, 50e6, size=n)
    out = []
    for k in range(n):
        s = int(side[k])
        p = (s + 5) // 10
        out.append(impact(s, p, int(rad[k]), float(vel[k]), nmat=2, strength=True,
                          cycles=cycles, precision=precision, Y0=float(y0[k]),
                          name=f"ens{seed}-{k}"))
    return out


def random_state(grid: Grid, seed: int, rho0: float = 2860.0):
    """Seeded smooth random state (for parity tests away from the impact path):
    full cells with density within +-2 %, small energies and velocities."""
    rng = np.random.default_rng(seed)
    NR, NZ = grid.NR, grid.NZ
    rho = rho0 * (1.0 + 0.02 * rng.uniform(-1, 1, size=(NZ, NR)))
    I = 1e4 * rng.uniform(0, 1, size=(NZ, NR))
    v = 10.0 * rng.uniform(-1, 1, size=(2, NZ + 1, NR + 1))
    return rho, I, v
