"""Multigrid hierarchy: horizontal-only coarsening with conditional
semi-coarsening in latitude.

Test infrastructure (see the package docstring).

Follows the paper:
  * Section 2.1: the grid is coarsened only horizontally; the vertical is
    never coarsened (the block-Jacobi smoother handles the vertical
    anisotropy).
  * Section 2.2: longitude is coarsened uniformly; latitude coarsening is
    conditional on the horizontal anisotropy, so rows near the poles (where
    cells are much longer in latitude than in longitude) are coarsened in
    longitude only.
  * Section 2.3: a shallow hierarchy whose coarsest level is handled by a
    simple iteration.

Readings where the paper is silent:
  * anisotropy of row J at a level with longitude width dlam:
        a_J = (dth_J / (cos th_J * dlam))^2,
    the ratio of the longitude to the latitude coupling at the cell centre
    (the inverse square of the paper's length ratio dx_lon/dx_lat);
  * pairing: in the southern hemisphere walk from the equator toward the
    pole; rows {J-1, J} merge iff a_J <= threshold and a_{J-1} <= threshold,
    otherwise row J stays alone; the northern hemisphere is the mirror image,
    so the equator is always a coarse face;
  * threshold 2 by default. Local Fourier analysis of damped point-Jacobi in
    the horizontal (the vertical is solved exactly) gives the smoothing
    factor max(|1-2w|, 1 - w a/(a+1)) for rows coarsened in longitude only
    (a >= 1), and max(|1-2w|, 1 - w min(a,1)/(a+1)) for merged rows. Rows
    coarsened in longitude only have a divided by 4, so coarse levels carry
    a in (t/4, t]; the worst merged-row factor over that range is smallest
    for t = 2 (with w = 0.8 it is 1 - 0.8/3 ~ 0.73 per sweep);
  * level count: "auto" keeps coarsening until the coarsest level has
    max a <= threshold; a fixed count (the paper's 4) is also allowed;
    coarsening stops when the number of longitudes is odd, and no level has
    fewer than MIN_NLON = 4 longitudes: with 2 or 3 cells (120-180 degrees)
    around a circle of latitude the cell-centred distances no longer
    approximate the fluxes, and an accurate solve on such a level makes the
    V-cycle converge worse (measured on a 192x96x70 shell: factor 0.36 with
    a 3x6 coarsest level, 0.19 when coarsening stops at 6x10);
  * coarse operators by rediscretisation on the coarse geometry, with the
    mass term aggregated (sum of the children's alpha V).
"""
from __future__ import annotations

import numpy as np

from .geometry import Level, vertical_coords, fine_lat_edges

MIN_NLON = 4


def anisotropy(level: Level) -> np.ndarray:
    """Per-row horizontal anisotropy a_J of a level."""
    return (level.dtheta / (np.cos(level.theta) * level.dlam)) ** 2


def coarsen_rows(a: np.ndarray, threshold: float):
    """Group the rows of one level into coarse rows.

    Returns a list of (first_row, count) in south-to-north order.
    """
    nJ = len(a)
    assert nJ % 2 == 0, "the number of latitude rows must be even"
    half = nJ // 2
    south = []                      # groups found walking equator -> south pole
    J = half - 1
    while J >= 0:
        if J >= 1 and a[J] <= threshold and a[J - 1] <= threshold:
            south.append((J - 1, 2))
            J -= 2
        else:
            south.append((J, 1))
            J -= 1
    south.reverse()                 # now south pole -> equator
    groups = list(south)
    for first, cnt in reversed(south):   # mirror: row j -> nJ-1-j
        last = first + cnt - 1
        groups.append((nJ - 1 - last, cnt))
    return groups


def _aggregate_mass(fine: Level, coarse: Level) -> np.ndarray:
    """M_c = sum of the children's M (two longitudes x the merged rows)."""
    Ms = fine.M[:, :, 0::2] + fine.M[:, :, 1::2]
    Mc = np.empty(coarse.shape)
    for J in range(coarse.nlat):
        f0, cnt = coarse.child_first[J], coarse.child_count[J]
        Mc[:, J, :] = Ms[:, f0:f0 + cnt, :].sum(axis=1)
    return Mc


def build_hierarchy(shell, alpha: np.ndarray, levels: int = 0,
                    threshold: float = 2.0, max_levels: int = 32):
    """Build the list of levels, finest first.

    shell : object with nlon, nlat, nlev, radius, thickness, stretch, K
    alpha : (nlev, nlat, nlon) positive Helmholtz coefficient
    levels: 0 = auto rule, otherwise the maximum number of levels
    """
    re, rc = vertical_coords(shell.nlev, shell.radius, shell.thickness,
                             shell.stretch)
    fine = Level(shell.nlon, fine_lat_edges(shell.nlat), re, rc, shell.K)
    fine.M = np.asarray(alpha, dtype=np.float64) * fine.V[:, :, None]
    out = [fine]
    while len(out) < max_levels:
        cur = out[-1]
        if levels > 0 and len(out) >= levels:
            break
        a = anisotropy(cur)
        if levels == 0 and a.max() <= threshold:
            break
        if cur.nlon % 2 != 0 or cur.nlon // 2 < MIN_NLON:
            break
        groups = coarsen_rows(a, threshold)
        edges = [cur.edges[0]] + [cur.edges[f + c] for f, c in groups]
        coarse = Level(cur.nlon // 2, edges, re, rc, shell.K)
        coarse.child_first = np.array([f for f, _ in groups], dtype=np.int64)
        coarse.child_count = np.array([c for _, c in groups], dtype=np.int64)
        coarse.M = _aggregate_mass(cur, coarse)
        out.append(coarse)
    return out
