"""What the perfectly matched layer buys (Sec. 4 compares a PML run with an
unbounded reference): the same vertical impact on

  pml   an n x n domain with a p-cell PML on the right and bottom,
  bare  the same n x n domain with plain walls (no layer),
  big   a (k n) x (k n) domain with plain walls, far enough that nothing
        reflected from its walls reaches the window before the stop time,

each run on the GPU to the same stop time. The n x n window at the top of the
axis (the pml run's physical region) is compared with the big run: the
energy of the difference field (kinetic plus linear-acoustic pressure energy
about the target at rest) per unit impact energy, relative L2 differences of
density and node momentum, and the crater depth and radius (matter-fraction
0.5 crossings, as in Sec. 4's profile comparison), next to each run's cells
and device time.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass

import numpy as np

from . import inputs


@dataclass
class Setup:
    n: int = 100            # physical cells per side
    p: int = 20             # PML cells (right and bottom) of the pml run
    radius: int = 10        # projectile radius, cells
    v_imp: float = 10e3     # impact speed, m/s
    t_end: float = 0.08     # stop time, s
    big: int = 10           # size factor of the reference domain
    strength: bool = False
    precision: str = "fp64"


def problems(s: Setup):
    """The three problems (pml, bare, big) and each one's window rows."""
    hv = 2 * s.radius + max(4, math.ceil(s.radius / 2))
    mats = [inputs.basalt(strength=s.strength)]

    def make(n, p, pml_on, name):
        g = inputs.Grid(n_r=n, n_z=n, pml_r=p, pml_b=p, t_stop=s.t_end)
        sc = inputs.Scene(surface_j=p + n - hv, radius=float(s.radius), v_imp=s.v_imp)
        return inputs.Problem(grid=g, mats=mats, pml=inputs.Pml(enabled=pml_on), scene=sc,
                              precision=s.precision, name=name)

    out = {"pml": make(s.n, s.p, 1, "pml"), "bare": make(s.n, 0, 0, "bare"),
           "big": make(s.big * s.n, 0, 0, "big")}
    # rows of the n x n window under the top of each domain
    rows = {"pml": s.p, "bare": 0, "big": s.big * s.n - s.n}
    return out, rows


def _window(F, r0, n):
    return {"rho": F["rho"][r0:r0 + n, :n], "p": F["p"][r0:r0 + n, :n], "f": F["f"][:, r0:r0 + n, :n],
            "v": F["v"][:, r0:r0 + n + 1, :n + 1]}


def _phi(w):
    """Matter fraction of a window's cells."""
    return w["f"].sum(axis=0)


def _rel_l2(a, b):
    den = float(np.sqrt(np.sum(b * b)))
    return float(np.sqrt(np.sum((a - b) ** 2))) / den if den > 0 else 0.0


def _node_mass(rho, dr, dz):
    nz, nr = rho.shape
    M = rho * ((np.arange(nr) + 0.5) * dr * dr * dz)[None, :]
    out = np.zeros((nz + 1, nr + 1))
    out[:-1, :-1] += M
    out[:-1, 1:] += M
    out[1:, :-1] += M
    out[1:, 1:] += M
    return 0.25 * out


def _crater(f, surface_row, dr, dz):
    """Depth below the surface along the axis and radius along the top
    target row where the matter fraction crosses 0.5."""
    phi = f.sum(axis=0)
    col, depth = phi[:, 0], 0.0
    for j in range(1, col.size):
        if col[j] < 0.5 <= col[j - 1]:
            z = (j - 0.5) + (0.5 - col[j - 1]) / (col[j] - col[j - 1])  # centres at (j + 1/2) dz
            depth = (surface_row - z) * dz
            break
    row, radius = phi[surface_row - 1, :], 0.0
    if row[0] < 0.5:
        radius = (row.size - 0.5) * dr
        for i in range(1, row.size):
            if row[i] >= 0.5 > row[i - 1]:
                radius = ((i - 0.5) + (0.5 - row[i - 1]) / (row[i] - row[i - 1])) * dr
                break
    return depth, radius


def run(s: Setup = Setup(), device: str = "cuda:0", chunk: int = 200, max_cycles: int = 20000) -> dict:
    """Runs the three problems to s.t_end on the GPU and compares them.
    (The step is clipped so that t lands on t_end; cycles after that have
    dt = 0 and change nothing.)"""
    from .salec import Salec
    probs, rows = problems(s)
    res, win = {}, {}
    ke0 = 0.0
    for key, pb in probs.items():
        ctx = Salec(pb, device)
        if key == "big":
            ke0 = ctx.diag()["ke"]  # impact kinetic energy (per radian)
        ms, cycles = 0.0, 0
        while ctx.diag()["t"] < s.t_end * (1.0 - 1e-12) and cycles < max_cycles:
            ctx.step(chunk)
            ms += ctx.last_step_ms()
            cycles += chunk
        d = ctx.diag()
        F = ctx.fields()
        w = _window(F, rows[key], s.n)
        win[key] = w
        sj = pb.scene.surface_j - rows[key]
        depth, radius = _crater(w["f"], sj, pb.grid.dr, pb.grid.dz)
        res[key] = {"cells": pb.grid.ncells, "cycles": int(d["cycle"]), "t": d["t"], "device_ms": ms,
                    "crater_depth": depth, "crater_radius": radius}
        del ctx
    ref = win["big"]
    g = probs["pml"].grid
    mat = probs["pml"].mats[0]
    rho0, c2 = mat.rho0, mat.A / mat.rho0
    vol = _node_mass(np.ones((s.n, s.n)), g.dr, g.dz)  # dual volumes of the window's nodes
    vc = ((np.arange(s.n) + 0.5) * g.dr * g.dr * g.dz)[None, :]
    mref = _node_mass(ref["rho"], g.dr, g.dz)
    for key in ("pml", "bare"):
        w = win[key]
        m = _node_mass(w["rho"], g.dr, g.dz)
        # energy of the difference field (linear acoustics about the target at
        # rest), per unit impact energy: what the walls sent back. Pressures
        # enter weighted by the matter fraction (phi p, the stress the momentum
        # balance sees): cells holding only traces of matter carry
        # ill-conditioned pressures in every run.
        dv2 = np.sum((w["v"] - ref["v"]) ** 2, axis=0)
        e_k = 0.5 * rho0 * np.sum(vol * dv2)
        e_p = np.sum(vc * (_phi(w) * w["p"] - _phi(ref) * ref["p"]) ** 2) / (2.0 * rho0 * c2)
        res[key]["err_vs_big"] = {
            "rho": _rel_l2(w["rho"], ref["rho"]),
            "momentum": _rel_l2(m[None] * w["v"], mref[None] * ref["v"]),
            "reflected_energy": (e_k + e_p) / ke0,
        }
    res["setup"] = {"n": s.n, "p": s.p, "radius": s.radius, "v_imp": s.v_imp, "t_end": s.t_end,
                    "big": s.big, "strength": s.strength, "precision": s.precision}
    return res


# --------------------------------------------------------------------------
# the same comparison in the paper's own setting (Sec. 4, Table 2)
# --------------------------------------------------------------------------
@dataclass
class PaperSetup:
    t_end: float = 30.0     # s (the paper's second panel: the shock has reached the bottom and turned)
    ext_ref: int = 200      # extension cells right and below in the reference run
    precision: str = "fp64"
    layers: int = 3         # 3: Sec. 4's calcite, granite, dunite; 2: basalt crust over mantle rock
    closure: int = 0        # mixed cells: 0 shared, 1 per-material densities and energies
    far_km: float = 60.0    # the far field: target cells further than this from the impact point
    strength: bool = True   # Table 1's strength (False: hydrodynamic layers)
    damp_stress: int = 0    # 1: the layers also relax the deviatoric stress (an extension)
    damage: int = 0         # 1: Table 1's damage and block-model constants on every layer
    af_h: float = 0.0       # block size of the block model, m (0: the projectile radius)


def paper_problems(s: PaperSetup):
    """Table 2's grid with its 30-cell PML, the same grid with plain walls, and
    a reference whose right and bottom extension zones run ext_ref cells
    (about 200 km further: nothing returns into the window before ~90 s).
    The window is the fine zone with its first 20 extension cells right, above
    and below, which all three grids share cell for cell."""
    base = inputs.config_paper_layers(s.precision) if s.layers == 3 else inputs.config_paper(s.precision)
    base.grid.t_stop = s.t_end
    base.grid.closure = s.closure
    if not s.strength:
        mats = ([inputs.calcite(False), inputs.granite(False), inputs.dunite(False)] if s.layers == 3
                else [inputs.basalt(False), inputs.mantle_like(False)])
        base = base.replace(mats=mats)
    if s.damage:
        if not s.strength:
            raise ValueError("damage needs Table 1's strength")
        h = s.af_h if s.af_h > 0 else base.scene.radius
        keys = ("calcite", "granite", "dunite") if s.layers == 3 else ("granite", "dunite")
        base = base.replace(mats=[inputs.with_damage(m, **inputs.TABLE1_DAMAGE[k], af_h=h)
                                  for m, k in zip(base.mats, keys)])
    base = base.replace(pml=inputs.Pml(damp_stress=s.damp_stress))
    bare = base.replace(pml=inputs.Pml(enabled=0))
    gref = inputs.paper_layout(462, 462, (0, s.ext_ref, 20, s.ext_ref), (0, 0), nmat=base.grid.nmat)
    gref.cfl = base.grid.cfl
    gref.t_stop = s.t_end
    gref.closure = s.closure
    sj = s.ext_ref + (base.scene.surface_j - base.grid.pml_b - 20)
    b0 = base.scene
    sc = dataclasses.replace(b0, surface_j=sj, layer_j=sj - (b0.surface_j - b0.layer_j),
                             layer2_j=sj - (b0.surface_j - b0.layer2_j) if s.layers == 3 else 0)
    ref = base.replace(grid=gref, scene=sc, pml=inputs.Pml(enabled=0))
    rows = {"pml": base.grid.pml_b, "bare": base.grid.pml_b, "ref": s.ext_ref - 20}
    return {"pml": base, "bare": bare, "ref": ref}, rows, 482, 502


def _geometry(g):
    rn = np.concatenate([[0.0], np.cumsum(g.dr_col)])
    dz = np.asarray(g.dz_row, dtype=np.float64)
    Vc = 0.5 * (rn[1:] ** 2 - rn[:-1] ** 2)[None, :] * dz[:, None]
    return Vc


def paper_run(s: PaperSetup = PaperSetup(), device: str = "cuda:0", chunk: int = 500,
              max_cycles: int = 1000000) -> dict:
    """Runs the three problems to s.t_end and compares the target part of the
    window (below the original surface; the ejecta above it are chaotic in
    every run): energy of the difference field against the reference
    (kinetic with the reference's node masses, acoustic (phi p - phi_ref p_ref)^2 / (2 A)
    with the crust's bulk modulus A) per unit impact kinetic energy, and the
    relative L2 of phi (p - p0) (the quantity the paper plots, weighted by the
    matter fraction), next to cells and device time."""
    from .salec import Salec
    probs, rows, wc, wr = paper_problems(s)
    res, win = {}, {}
    ke0 = 0.0
    for key, pb in probs.items():
        ctx = Salec(pb, device)
        if key == "ref":
            ke0 = ctx.diag()["ke"]
        ms, cycles = 0.0, 0
        while ctx.diag()["t"] < s.t_end * (1.0 - 1e-12) and cycles < max_cycles:
            ctx.step(chunk)
            ms += ctx.last_step_ms()
            cycles += chunk
        d = ctx.diag()
        F = ctx.fields()
        p0 = ctx.p0()
        r0 = rows[key]
        sl = slice(r0, r0 + wr)
        win[key] = {"rho": F["rho"][sl, :wc], "p": F["p"][sl, :wc], "c2": F["c2"][sl, :wc],
                    "dp": F["p"][sl, :wc] - p0[sl, None], "f": F["f"][:, sl, :wc],
                    "v": F["v"][:, r0:r0 + wr + 1, :wc + 1]}
        res[key] = {"cells": pb.grid.ncells, "cycles": int(d["cycle"]), "t": d["t"], "device_ms": ms}
        del ctx
    g = probs["pml"].grid
    ns = probs["pml"].scene.surface_j - rows["pml"]  # target rows of the window
    Vc = _geometry(g)[rows["pml"]:rows["pml"] + ns, :wc]
    # bulk modulus of the crust the shock crosses (granite of the three-layer
    # target, basalt of the two-layer one)
    A = probs["pml"].mats[1 if s.layers == 3 else 0].A
    ref = win["ref"]
    mref = 0.25 * np.pad(ref["rho"][:ns] * Vc, 1)
    mref = (mref[:-1, :-1] + mref[:-1, 1:]) + (mref[1:, :-1] + mref[1:, 1:])
    # distance of the window's cells and nodes from the impact point (axis,
    # original surface)
    rn = np.concatenate([[0.0], np.cumsum(g.dr_col)])[:wc + 1]
    zn = np.concatenate([[0.0], np.cumsum(g.dz_row)])
    r0w, sjw = rows["pml"], probs["pml"].scene.surface_j
    zs = zn[sjw]
    zw = zn[r0w:r0w + ns + 1]
    rc, zc = 0.5 * (rn[1:] + rn[:-1]), 0.5 * (zw[1:] + zw[:-1])
    far = np.hypot(rc[None, :], (zs - zc)[:, None]) > s.far_km * 1e3
    farn = np.hypot(rn[None, :], (zs - zw)[:, None]) > s.far_km * 1e3
    for key in ("pml", "bare"):
        w = win[key]
        dv2 = np.sum((w["v"][:, :ns + 1] - ref["v"][:, :ns + 1]) ** 2, axis=0)
        e_k = 0.5 * np.sum(mref * dv2)
        # pressures weighted by the matter fraction (see run())
        pw, pr = _phi(w)[:ns], _phi(ref)[:ns]
        e_p = np.sum(Vc * (pw * w["p"][:ns] - pr * ref["p"][:ns]) ** 2) / (2.0 * A)
        res[key]["err_vs_ref"] = {"reflected_energy": float((e_k + e_p) / ke0),
                                  "dp": _rel_l2(pw * w["dp"][:ns], pr * ref["dp"][:ns])}
        # the same away from the crater, whose flow is chaotic by ~30 s in any
        # two runs: what the boundaries sent back
        fe_k = 0.5 * np.sum(np.where(farn, mref * dv2, 0.0))
        fe_p = np.sum(np.where(far, Vc * (pw * w["p"][:ns] - pr * ref["p"][:ns]) ** 2, 0.0)) / (2.0 * A)
        res[key]["err_vs_ref_far"] = {"reflected_energy": float((fe_k + fe_p) / ke0),
                                      "dp": _rel_l2(np.where(far, pw * w["dp"][:ns], 0.0),
                                                    np.where(far, pr * ref["dp"][:ns], 0.0))}
    res["setup"] = {"t_end": s.t_end, "ext_ref": s.ext_ref, "precision": s.precision, "layers": s.layers,
                    "closure": s.closure, "window_cells": [wr, wc], "far_km": s.far_km,
                    "strength": s.strength, "damp_stress": s.damp_stress, "damage": s.damage,
                    "af_h": s.af_h}
    return res


if __name__ == "__main__":
    import json
    print(json.dumps(run(), indent=1))


# --------------------------------------------------------------------------
# crater profiles in the paper's setting (Sec. 4 compares them over time)
# --------------------------------------------------------------------------
def _level_from_top(x, zc, level=0.5):
    """Per column: the height where x first reaches `level` scanning down
    from the top (linear between cell centres zc); NaN where it never does."""
    nz, nr = x.shape
    out = np.full(nr, np.nan)
    for i in range(nr):
        col = x[:, i]
        hit = np.nonzero(col >= level)[0]
        if hit.size == 0:
            continue
        j = hit[-1]
        if j == nz - 1:
            out[i] = zc[j]
            continue
        a, b = col[j], col[j + 1]
        out[i] = zc[j] + (a - level) / (a - b) * (zc[j + 1] - zc[j])
    return out


def _level_from_bottom(x, zc, level=0.5):
    """Per column: the height where x first reaches `level` scanning up from
    the bottom; NaN where it never does."""
    nz, nr = x.shape
    out = np.full(nr, np.nan)
    for i in range(nr):
        col = x[:, i]
        hit = np.nonzero(col >= level)[0]
        if hit.size == 0:
            continue
        j = hit[0]
        if j == 0:
            out[i] = zc[0]
            continue
        a, b = col[j - 1], col[j]
        out[i] = zc[j - 1] + (level - a) / (b - a) * (zc[j] - zc[j - 1])
    return out


def paper_profiles(times=(10.0, 30.0, 60.0), r_crater_km: float = 60.0, r_inner_km: float = 35.0,
                   r_moho_km: float = 100.0,
                   device: str = "cuda:0", bare_until: float = 30.0, chunk: int = 500,
                   max_cycles: int = 1000000, **setup) -> dict:
    """The crater surface (matter fraction 0.5 from below) and the base of
    the granite crust (granite fraction 0.5 from below: the crust-mantle
    boundary, unaffected by the dunite projectile in the crater floor) of the
    PML run and of the reference with ~200 km longer extension zones, at each
    time, within r_crater_km (and inside the rim, r_inner_km) and r_moho_km of
    the axis; largest, mean and median absolute differences in metres (the
    largest sit at the rim, where an overturned flap makes any level reading
    fragile). Plain walls too up to bare_until (later
    their trapped reflections collapse the time step)."""
    from .salec import Salec
    out = {}
    for t in times:
        s = PaperSetup(t_end=float(t), **setup)
        probs, rows, wc, wr = paper_problems(s)
        keys = ("pml", "ref", "bare") if t <= bare_until else ("pml", "ref")
        prof, reached = {}, {}
        for key in keys:
            pb = probs[key]
            ctx = Salec(pb, device)
            cycles = 0
            while ctx.diag()["t"] < s.t_end * (1.0 - 1e-12) and cycles < max_cycles:
                ctx.step(chunk)
                cycles += chunk
            d = ctx.diag()
            reached[key] = {"t": d["t"], "cycles": int(d["cycle"])}
            F = ctx.fields(eos=False)
            del ctx
            g = pb.grid
            r0 = rows[key]
            zn = np.concatenate([[0.0], np.cumsum(g.dz_row)])
            zs = zn[pb.scene.surface_j]
            zc = 0.5 * (zn[1:] + zn[:-1])[r0:r0 + wr] - zs  # heights relative to the original surface
            f = F["f"][:, r0:r0 + wr, :wc]
            # the target's surface: matter fraction 0.5 scanning up from the
            # bottom, so that ejecta in flight over the cavity do not count
            prof[key] = {"crater": _level_from_bottom(1.0 - f.sum(axis=0), zc),
                         "moho": _level_from_bottom(f[1], zc) if pb.grid.nmat == 3 else None}
        g = probs["pml"].grid
        rn = np.concatenate([[0.0], np.cumsum(g.dr_col)])[:wc + 1]
        rc = 0.5 * (rn[1:] + rn[:-1])
        res = {}
        for key in keys:
            if key == "ref":
                continue
            d = {}
            for name, src, rmax in (("crater", "crater", r_crater_km), ("crater_inner", "crater", r_inner_km),
                                    ("moho", "moho", r_moho_km)):
                a, b = prof[key][src], prof["ref"][src]
                if a is None:
                    continue
                sel = (rc <= rmax * 1e3) & np.isfinite(a) & np.isfinite(b)
                if not sel.any():  # no column where both runs have the level
                    d[name] = None
                    continue
                diff = np.abs(a[sel] - b[sel])
                d[name] = {"max_m": float(diff.max()), "mean_m": float(diff.mean()),
                           "median_m": float(np.median(diff)), "r_at_max_km": float(rc[sel][np.argmax(diff)] / 1e3),
                           "columns": int(sel.sum())}
            res[key] = d
        ref = prof["ref"]
        sel = rc <= r_crater_km * 1e3
        res["ref_crater_depth_m"] = float(-np.nanmin(ref["crater"][sel]))
        if ref["moho"] is not None:
            m = ref["moho"][rc <= r_moho_km * 1e3]
            res["ref_moho_uplift_m"] = float(np.nanmax(m) - np.nanmedian(m[-20:]))
        pm = prof["pml"]
        res["pml_crater_depth_m"] = float(-np.nanmin(pm["crater"][sel]))
        if pm["moho"] is not None:
            m = pm["moho"][rc <= r_moho_km * 1e3]
            res["pml_moho_uplift_m"] = float(np.nanmax(m) - np.nanmedian(m[-20:]))
        res["reached"] = reached
        out[f"{t:g}s"] = res
    return out
