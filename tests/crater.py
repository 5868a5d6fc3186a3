"""Crater depth and radius of an impact state (harness-side metric, applied
identically to every run being compared).

Depth: the matter fraction phi = sum of volume fractions is scanned up the
axis column from the bottom; z* is the first height where phi falls below
0.5, interpolated linearly between cell centres, and depth = z_surface - z*.
Radius: along the top target row (j_s - 1), scanning outward from the axis,
the first r where phi rises back to >= 0.5, interpolated between the cell
centres r_{i+1/2}. Material ejected above the cavity does not affect either.
"""
import numpy as np


def _cross(x0, x1, p0, p1, level=0.5):
    if p1 == p0:
        return x1
    return x0 + (level - p0) * (x1 - x0) / (p1 - p0)


def crater_depth(f, grid, surface_j):
    phi = f.sum(axis=0)
    col = phi[:, 0]
    zc = (np.arange(col.size) + 0.5) * grid.dz
    zs = surface_j * grid.dz
    for j in range(1, col.size):
        if col[j] < 0.5 <= col[j - 1]:
            return zs - _cross(zc[j - 1], zc[j], col[j - 1], col[j])
    return 0.0


def crater_radius(f, grid, surface_j):
    phi = f.sum(axis=0)
    row = phi[surface_j - 1, :]
    rc = (np.arange(row.size) + 0.5) * grid.dr
    if row[0] >= 0.5:
        return 0.0
    for i in range(1, row.size):
        if row[i] >= 0.5 > row[i - 1]:
            return _cross(rc[i - 1], rc[i], row[i - 1], row[i])
    return float(rc[-1])


def rel_l2(a, b):
    den = float(np.sqrt(np.sum(np.asarray(b, dtype=np.float64) ** 2)))
    num = float(np.sqrt(np.sum((np.asarray(a, dtype=np.float64) - b) ** 2)))
    return num / den if den > 0 else num


def node_mass(rho, grid):
    """A quarter of the masses (rho V, per radian) of the cells around each node."""
    NZ, NR = rho.shape
    V = (np.arange(NR) + 0.5) * grid.dr * grid.dr * grid.dz
    M = rho * V[None, :]
    out = np.zeros((NZ + 1, NR + 1))
    out[:-1, :-1] += M
    out[:-1, 1:] += M
    out[1:, :-1] += M
    out[1:, 1:] += M
    return 0.25 * out


def conserved_errors(Fa, Fb, grid):
    """Relative L2 errors of run a against reference run b on the volume
    densities the scheme conserves or uses: rho, rho I, phi p (the pressure
    that enters the stress), f, phi s, and the node momentum m v. Intensive
    p, I and v are ill-conditioned in cells and nodes holding only traces of
    matter, so they are compared through these densities."""
    pa, pb = Fa["f"].sum(0), Fb["f"].sum(0)
    e = {"rho": rel_l2(Fa["rho"], Fb["rho"]),
         "rhoI": rel_l2(Fa["rho"] * Fa["I"], Fb["rho"] * Fb["I"]),
         "phi_p": rel_l2(pa * Fa["p"], pb * Fb["p"]),
         "f": rel_l2(Fa["f"], Fb["f"])}
    if np.any(Fb["s"]):
        e["phi_s"] = rel_l2(pa[None] * Fa["s"], pb[None] * Fb["s"])
    ma, mb = node_mass(Fa["rho"], grid), node_mass(Fb["rho"], grid)
    e["mv_r"] = rel_l2(ma * Fa["v"][0], mb * Fb["v"][0])
    e["mv_z"] = rel_l2(ma * Fa["v"][1], mb * Fb["v"][1])
    return e


MATTER = 1e-3  # cells (nodes) holding matter: the ones the Courant step accounts for


def node_phi(phi):
    """Matter fraction at the nodes: the mean over the (up to four) cells
    around each node."""
    NZ, NR = phi.shape
    o, c = np.zeros((NZ + 1, NR + 1)), np.zeros((NZ + 1, NR + 1))
    for dj in (0, 1):
        for di in (0, 1):
            o[dj:dj + NZ, di:di + NR] += phi
            c[dj:dj + NZ, di:di + NR] += 1
    return o / c


def per_field(Fm, Fa, grid, sj):
    """Run m against reference run a: plain per-field relative L2 of rho, p,
    I, v_r, v_z over all cells (nodes) and over those holding matter, the
    conserved densities, and the crater depth and radius difference in
    cells."""
    phi = Fa["f"].sum(0)
    mc, mn = phi >= MATTER, node_phi(phi) >= MATTER
    e = {}
    for k in ("rho", "p", "I"):
        e[k] = rel_l2(Fm[k], Fa[k])
        e[k + "@matter"] = rel_l2(Fm[k][mc], Fa[k][mc])
    for q, k in ((0, "v_r"), (1, "v_z")):
        e[k] = rel_l2(Fm["v"][q], Fa["v"][q])
        e[k + "@matter"] = rel_l2(Fm["v"][q][mn], Fa["v"][q][mn])
    e.update({"cons." + k: v for k, v in conserved_errors(Fm, Fa, grid).items()})
    e["depth_cells"] = abs(crater_depth(Fm["f"], grid, sj) - crater_depth(Fa["f"], grid, sj)) / grid.dz
    e["radius_cells"] = abs(crater_radius(Fm["f"], grid, sj) - crater_radius(Fa["f"], grid, sj)) / grid.dr
    return e
