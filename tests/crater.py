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
