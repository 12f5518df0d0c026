"""The operator H of one level, its vertical part H_z and column solves.

Test infrastructure (see the package docstring).

Section 2.1 splits H = H_z + dH: H_z holds the diagonal and the couplings
inside a vertical column, dH the horizontal couplings. With the finite-volume
form of the geometry module this reads:
  * H_z is tridiagonal per column with off-diagonals -Tr_{k-1/2}, -Tr_{k+1/2}
    and diagonal Tr_{k-1/2} + Tr_{k+1/2} + mt_k, where
        mt = M + 2 Tlam + Tth_south + Tth_north
    collects every diagonal term (the mass and the horizontal face terms);
  * dH holds only the horizontal off-diagonals -Tlam (to i+-1) and -Tth (to
    J+-1).

H is always evaluated in difference form (sum of T (u_c - u_nb) + M u_c).

Column solves H_z^{-1} s use the Thomas algorithm with its pivots written in
row-sum form (a reading: the paper gives no column solver). With the textbook
pivots p_k = D_k - Tr_k^2 / p_{k-1}, write p_k = Tr_{k+1/2} + g_k; then
    g_0 = mt_0,   g_k = mt_k + Tr_{k-1/2} g_{k-1} / (Tr_{k-1/2} + g_{k-1}),
which is the same number computed without subtracting nearly equal terms
(the vertical couplings exceed mt by up to 1e8 on thin shells).
Forward:  y_k = (s_k + Tr_{k-1/2} y_{k-1}) / p_k
Backward: x_k = y_k + (Tr_{k+1/2} / p_k) x_{k+1}
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .geometry import Level


def apply(level: Level, x: np.ndarray) -> np.ndarray:
    """y = H x in difference form; x has shape (nz, nlat, nlon)."""
    y = level.M * x
    # longitude faces (periodic): both neighbours i-1 and i+1
    y += level.Tlam[:, :, None] * ((x - np.roll(x, 1, axis=2))
                                   + (x - np.roll(x, -1, axis=2)))
    # latitude faces 1..nJ-1: face F lies between rows F-1 and F
    if level.nlat > 1:
        flux = level.Tth[:, 1:-1, None] * (x[:, :-1, :] - x[:, 1:, :])
        y[:, :-1, :] += flux
        y[:, 1:, :] -= flux
    # vertical faces 1..nz-1: face F lies between layers F-1 and F
    if level.nz > 1:
        flux = level.Tr[1:-1, :, None] * (x[:-1] - x[1:])
        y[:-1] += flux
        y[1:] -= flux
    return y


def mtilde(level: Level) -> np.ndarray:
    """Diagonal excess of H_z: M + 2 Tlam + Tth(south face) + Tth(north face)."""
    horiz = 2.0 * level.Tlam + level.Tth[:, :-1] + level.Tth[:, 1:]
    return level.M + horiz[:, :, None]


def column_pivots(level: Level) -> np.ndarray:
    """Thomas pivots p[k, J, i] of every column of H_z (row-sum form)."""
    mt = mtilde(level)
    Tr = level.Tr[:, :, None]
    g = np.empty_like(mt)
    g[0] = mt[0]
    for k in range(1, level.nz):
        g[k] = mt[k] + Tr[k] * g[k - 1] / (Tr[k] + g[k - 1])
    return Tr[1:] + g


def column_solve(level: Level, s: np.ndarray) -> np.ndarray:
    """H_z^{-1} s for every vertical column at once."""
    if level._pivots is None:
        level._pivots = column_pivots(level)
    p = level._pivots
    Tr = level.Tr[:, :, None]
    nz = level.nz
    y = np.empty_like(s)
    y[0] = s[0] / p[0]
    for k in range(1, nz):
        y[k] = (s[k] + Tr[k] * y[k - 1]) / p[k]
    x = np.empty_like(s)
    x[nz - 1] = y[nz - 1]
    for k in range(nz - 2, -1, -1):
        x[k] = y[k] + (Tr[k + 1] / p[k]) * x[k + 1]
    return x


def _index(level: Level):
    nz, nJ, nI = level.shape
    return np.arange(nz * nJ * nI).reshape(nz, nJ, nI)


def assemble(level: Level, part: str = "H") -> sp.csr_matrix:
    """Assemble H (or H_z, or dH) as a sparse matrix by visiting every face.

    The unknown (k, J, i) has global index (k*nlat + J)*nlon + i. Each interior
    face between cells c and n with transmissibility T adds T to both
    diagonals and -T to the two off-diagonals; the mass adds M_c to the
    diagonal. part = "Hz" keeps the vertical faces and puts the horizontal
    face terms on the diagonal only; part = "dH" keeps only the horizontal
    off-diagonals.
    """
    nz, nJ, nI = level.shape
    idx = _index(level)
    rows, cols, vals = [], [], []

    def add(c, n, T, horizontal):
        T = np.broadcast_to(T, c.shape).ravel(); c = c.ravel(); n = n.ravel()
        if part == "H" or (part == "Hz" and not horizontal):
            rows.extend([c, n, c, n]); cols.extend([c, n, n, c])
            vals.extend([T, T, -T, -T])
        elif part == "Hz" and horizontal:
            rows.extend([c, n]); cols.extend([c, n]); vals.extend([T, T])
        elif part == "dH" and horizontal:
            rows.extend([c, n]); cols.extend([n, c]); vals.extend([-T, -T])

    # longitude faces: the east face of every cell, between i and i+1 (mod
    # nI); for nI == 2 these are the two distinct faces joining the same
    # pair; for nI == 1 the face joins a cell to itself and adds nothing
    if nI > 1:
        T = np.broadcast_to(level.Tlam[:, :, None], idx.shape)
        add(idx, np.roll(idx, -1, axis=2), T, True)
    # latitude faces between rows F-1 and F
    for F in range(1, nJ):
        add(idx[:, F - 1, :], idx[:, F, :],
            np.broadcast_to(level.Tth[:, F, None], (nz, nI)), True)
    # vertical faces between layers F-1 and F
    for F in range(1, nz):
        add(idx[F - 1], idx[F],
            np.broadcast_to(level.Tr[F, :, None], (nJ, nI)), False)
    if part in ("H", "Hz"):
        d = idx.ravel()
        rows.append(d); cols.append(d); vals.append(level.M.ravel())
    n = nz * nJ * nI
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows),
                                               np.concatenate(cols))),
                      shape=(n, n))
    return A.tocsr()
