"""Pins for the oracle's hierarchy (Sections 2.1-2.3): horizontal-only
coarsening, conditional semi-coarsening in latitude, aggregated mass.

The worked maps below are derived by hand from the rule (walk from the
equator toward each pole; merge two rows iff both have anisotropy
a = (dth/(cos th * dlam))^2 <= threshold; mirror to the north):

8x4 (dlam = dth = pi/4): rows at -67.5, -22.5 deg have a = 1/cos^2 = 6.83,
1.17; the equator row could only pair with the polar one, so level 0 merges
nothing -> 4x4. At dlam = pi/2 the same rows have a = 1.71, 0.29 (both <= 2),
so the auto rule stops at 4x4; a third level would merge both pairs, but it
would have 2 longitudes, below the minimum of 4, so even a fixed count of 3
levels stops at 4x4.

16x8 (dlam = dth = pi/8): from the equator a = 1.04, 1.45, 3.24, 26.3;
rows {2,3} merge, rows 1 and 0 stay -> 8x6. At dlam = pi/4: a({2,3}) = 1.17,
a(1) = 0.81, a(0) = 6.57 -> {1,2} merge, {0} stays -> 4x4, where the rows
(centres -78.75 and -33.75 deg) have a = 1.64 and 0.81 <= 2: stop.
"""
import numpy as np
import pytest

import shellgen
from oracle import build_hierarchy, anisotropy, coarsen_rows


def _shell(nlon, nlat, nz=3, **kw):
    return shellgen.Shell("t", nlon, nlat, nz, **kw)


def _sizes(L):
    return [(l.nlon, l.nlat) for l in L]


def test_worked_map_8x4():
    sh = _shell(8, 4)
    assert _sizes(build_hierarchy(sh, shellgen.alpha(sh))) == [(8, 4), (4, 4)]
    L = build_hierarchy(sh, shellgen.alpha(sh), levels=3)
    assert _sizes(L) == [(8, 4), (4, 4)]
    np.testing.assert_allclose(anisotropy(L[0])[:2], [6.83, 1.17], atol=5e-3)
    np.testing.assert_allclose(anisotropy(L[1])[:2], [1.71, 0.29], atol=5e-3)
    assert list(L[1].child_count) == [1, 1, 1, 1]
    assert coarsen_rows(anisotropy(L[1]), 2.0) == [(0, 2), (2, 2)]


def test_worked_map_16x8():
    sh = _shell(16, 8)
    L = build_hierarchy(sh, shellgen.alpha(sh))
    assert _sizes(L) == [(16, 8), (8, 6), (4, 4)]
    np.testing.assert_allclose(anisotropy(L[0])[:4][::-1], [1.04, 1.446, 3.24, 26.27], rtol=2e-3,
                               atol=0)
    assert list(L[1].child_first) == [0, 1, 2, 4, 6, 7]
    assert list(L[1].child_count) == [1, 1, 2, 2, 1, 1]
    assert list(L[2].child_first) == [0, 1, 3, 5]
    assert list(L[2].child_count) == [1, 2, 2, 1]
    np.testing.assert_allclose(anisotropy(L[2])[:2], [1.64, 0.81], atol=5e-3)


def test_threshold_four_reading():
    """At threshold 4 the polar rows of 8x4 (a = 6.83) still force one
    coarsening, and 16x8 merges the same rows (3.24 > 4 is false, but its
    partner has 26.3)."""
    sh = _shell(8, 4)
    assert _sizes(build_hierarchy(sh, shellgen.alpha(sh), threshold=4.0)) == [(8, 4), (4, 4)]
    sh = _shell(16, 8)
    L = build_hierarchy(sh, shellgen.alpha(sh), threshold=4.0)
    assert list(L[1].child_count) == [1, 1, 2, 2, 1, 1]


@pytest.mark.parametrize("name,sizes,stop", [
    ("shell64x32x16", [(64, 32), (32, 24), (16, 16), (8, 10), (4, 6)], "anisotropy"),
    ("shell384x192x70", [(384, 192), (192, 144), (96, 94), (48, 58), (24, 34),
                         (12, 20), (6, 12)], "width"),
])
def test_workload_hierarchies(name, sizes, stop):
    sh = shellgen.workload(name).with_(nlev=2)
    L = build_hierarchy(sh, shellgen.alpha(sh))
    assert _sizes(L) == sizes
    assert anisotropy(L[-2]).max() > 2.0
    if stop == "anisotropy":
        assert anisotropy(L[-1]).max() <= 2.0
    else:
        # a coarser level would have had fewer than 4 longitudes
        assert anisotropy(L[-1]).max() > 2.0 and L[-1].nlon // 2 < 4


@pytest.mark.parametrize("dims", [(64, 32), (96, 48), (40, 20)])
def test_hierarchy_invariants(dims):
    sh = _shell(*dims, nz=4, stretch=1.2)
    a = shellgen.alpha(sh, 9)
    L = build_hierarchy(sh, a)
    for f, c in zip(L[:-1], L[1:]):
        # every fine row in exactly one coarse row, in order
        covered = np.concatenate([np.arange(s, s + n) for s, n in
                                  zip(c.child_first, c.child_count)])
        np.testing.assert_array_equal(covered, np.arange(f.nlat))
        assert set(c.child_count) <= {1, 2}
        # north/south mirror symmetry and an even row count
        assert c.nlat % 2 == 0
        np.testing.assert_array_equal(c.child_count, c.child_count[::-1])
        np.testing.assert_allclose(c.edges, -c.edges[::-1], atol=1e-15)
        # exact integrals: coarse volumes are sums of children
        Vs = 2 * np.array([f.V[:, s:s + n].sum(axis=1)
                           for s, n in zip(c.child_first, c.child_count)]).T
        np.testing.assert_allclose(c.V, Vs, rtol=1e-13)
        # mass aggregation
        assert c.M.sum() == pytest.approx(f.M.sum(), rel=1e-13)
        # longitude halves each level; vertical untouched
        assert c.nlon * 2 == f.nlon and c.nz == f.nz


def test_coupling_to_mass_ratio_drops_by_four():
    """Section 2.3: each coarsening divides the horizontal condition number
    by about 4. Longitude couplings over mass fall by ~4 in every row; the
    latitude couplings over mass fall by ~4 in merged rows."""
    sh = _shell(128, 64, nz=2)
    sh = sh.with_(alpha_const=1.0)
    L = build_hierarchy(sh, shellgen.alpha(sh))
    for f, c in zip(L[:-1], L[1:]):
        if c.nlat < 12:        # rows spanning tens of degrees: cos th varies
            break
        rf = f.Tlam[0] / (f.M[0, :, 0])
        rc = c.Tlam[0] / (c.M[0, :, 0])
        for J in range(c.nlat):
            s, n = c.child_first[J], c.child_count[J]
            ratio = rf[s:s + n].mean() / rc[J]
            assert 3.99 < ratio < 4.4


def test_rows_merge_only_below_threshold():
    a = np.array([9.0, 1.5, 1.9, 1.0, 1.0, 1.9, 1.5, 9.0])
    assert coarsen_rows(a, 2.0) == [(0, 1), (1, 1), (2, 2), (4, 2), (6, 1), (7, 1)]
    assert coarsen_rows(a, 1.0) == [(0, 1), (1, 1), (2, 1), (3, 1), (4, 1), (5, 1),
                                    (6, 1), (7, 1)]
    assert coarsen_rows(np.ones(4), 2.0) == [(0, 2), (2, 2)]


def test_aggregated_mass_cell_by_cell_by_containment():
    """Coarse mass, cell by cell: each fine cell belongs to the coarse cell
    whose longitude span and latitude edges contain its centre (geometry
    only, none of the hierarchy's child maps or pairings), and the coarse
    cell's M must be the sum of its fine cells' M. alpha varies along every
    direction, so a wrong longitude pairing, row map or layer fails."""
    sh = _shell(16, 8, nz=2)
    nz, nj, ni = sh.shape
    i, j, k = np.arange(ni), np.arange(nj), np.arange(nz)
    alpha = 1.0 + i[None, None, :] + 10.0 * j[None, :, None] + 100.0 * k[:, None, None]
    L = build_hierarchy(sh, alpha, levels=3)
    assert _sizes(L) == [(16, 8), (8, 6), (4, 4)]
    for fine, coarse in zip(L[:-1], L[1:]):
        lon_centre = (np.arange(fine.nlon) + 0.5) * fine.dlam
        I = np.floor(lon_centre / coarse.dlam).astype(int)
        J = np.searchsorted(coarse.edges, fine.theta) - 1
        expect = np.zeros(coarse.M.shape)
        for jj in range(fine.nlat):
            for ii in range(fine.nlon):
                expect[:, J[jj], I[ii]] += fine.M[:, jj, ii]
        np.testing.assert_allclose(coarse.M, expect, rtol=1e-14, atol=0)


def test_aggregated_mass_worked_longitude_average():
    """Worked by hand: with alpha = 1 + i (varying along longitude only),
    coarse column I holds fine columns 2I and 2I+1, whose alpha are 2I+1 and
    2I+2 over equal volumes, so the coarse mass over the coarse volume (the
    volume-weighted mean alpha) is 2I + 1.5 on every row, merged or not;
    one level further it is the mean over columns 4I..4I+3: 4I + 2.5."""
    sh = _shell(16, 8, nz=2)
    alpha = np.broadcast_to(1.0 + np.arange(16.0), sh.shape).copy()
    L = build_hierarchy(sh, alpha, levels=3)
    for l, want in ((1, 2.0 * np.arange(8) + 1.5), (2, 4.0 * np.arange(4) + 2.5)):
        ratio = L[l].M / L[l].V[:, :, None]
        np.testing.assert_allclose(ratio, np.broadcast_to(want, ratio.shape), rtol=1e-13)
