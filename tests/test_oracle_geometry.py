"""Pins for the oracle's shell geometry and finite-volume tables.

Closed forms (shell volume, sphere areas), brute-force quadrature of single
faces and cells, and the consistency of (Hu)/V with the continuous operator
-div(grad u) + alpha u on smooth fields (Section 2: H is a discrete
Laplacian-like operator).
"""
import numpy as np
import pytest
from scipy import integrate

import shellgen
from oracle import vertical_coords, fine_lat_edges, Level, apply, build_hierarchy


def _level(nlon, nlat, nz, R=1.0, D=0.01, q=1.1, K=1.0):
    re, rc = vertical_coords(nz, R, D, q)
    return Level(nlon, fine_lat_edges(nlat), re, rc, K)


def test_vertical_layers_geometric():
    re, rc = vertical_coords(16, 1.0, 0.01, 1.1)
    dz = np.diff(re)
    assert re[0] == 1.0
    assert re[-1] == pytest.approx(1.01, rel=1e-14)
    np.testing.assert_allclose(dz[1:] / dz[:-1], 1.1, rtol=1e-12)
    np.testing.assert_allclose(rc, 0.5 * (re[1:] + re[:-1]))
    re1, _ = vertical_coords(4, 2.0, 1.0, 1.0)
    np.testing.assert_allclose(np.diff(re1), 0.25)


@pytest.mark.parametrize("nlon,nlat,nz,q", [(8, 4, 3, 1.0), (64, 32, 16, 1.1),
                                            (36, 18, 7, 1.05)])
def test_total_volume_is_shell_volume(nlon, nlat, nz, q):
    R, D = 1.0, 0.01
    lev = _level(nlon, nlat, nz, R, D, q)
    total = lev.V.sum() * nlon
    exact = 4.0 * np.pi / 3.0 * ((R + D) ** 3 - R ** 3)
    assert total == pytest.approx(exact, rel=1e-13)
    # per layer: the spherical shell between the two radii
    re = lev.r_edge
    np.testing.assert_allclose(lev.V.sum(axis=1) * nlon,
                               4 * np.pi / 3 * (re[1:] ** 3 - re[:-1] ** 3),
                               rtol=1e-13)


def test_radial_faces_cover_the_sphere():
    lev = _level(24, 12, 6, K=2.5)
    rc, re = lev.r_centre, lev.r_edge
    for F in range(1, lev.nz):
        area = (lev.Tr[F] * (rc[F] - rc[F - 1]) / lev.K).sum() * lev.nlon
        assert area == pytest.approx(4 * np.pi * re[F] ** 2, rel=1e-13)
    assert np.all(lev.Tr[0] == 0) and np.all(lev.Tr[-1] == 0)
    assert np.all(lev.Tth[:, 0] == 0) and np.all(lev.Tth[:, -1] == 0)


def test_face_areas_and_volumes_by_quadrature():
    """Brute force: integrate each face / cell numerically and compare."""
    lev = _level(10, 6, 4, R=1.0, D=0.3, q=1.3, K=1.7)
    re, rc, e, th = lev.r_edge, lev.r_centre, lev.edges, lev.theta
    dl = lev.dlam
    opts = dict(epsabs=0, epsrel=1e-13)
    for k, J in [(0, 0), (1, 2), (3, 5), (2, 3)]:
        # volume: int r^2 cos(theta) dr dtheta dlam
        v, _ = integrate.dblquad(lambda t, r: r * r * np.cos(t), re[k], re[k + 1],
                                 e[J], e[J + 1], **opts)
        assert lev.V[k, J] == pytest.approx(v * dl, rel=1e-12)
        # longitude face: int r dr dtheta, distance r_k cos(th_J) dlam
        a, _ = integrate.dblquad(lambda t, r: r, re[k], re[k + 1], e[J], e[J + 1], **opts)
        assert lev.Tlam[k, J] == pytest.approx(lev.K * a / (rc[k] * np.cos(th[J]) * dl),
                                               rel=1e-12)
        # latitude face at the north edge of row J (if interior)
        F = J + 1
        if F < lev.nlat:
            a, _ = integrate.quad(lambda r: r * np.cos(e[F]), re[k], re[k + 1], **opts)
            assert lev.Tth[k, F] == pytest.approx(
                lev.K * a * dl / (rc[k] * (th[F] - th[F - 1])), rel=1e-12)
        # radial face at the top of layer k (if interior)
        if k + 1 < lev.nz:
            a, _ = integrate.quad(lambda t: re[k + 1] ** 2 * np.cos(t), e[J], e[J + 1], **opts)
            assert lev.Tr[k + 1, J] == pytest.approx(
                lev.K * a * dl / (rc[k + 1] - rc[k]), rel=1e-12)


def _consistency_error(nlon, nlat, nz, ufun, Lfun, R, D, q, alpha, rows, layers):
    re, rc = vertical_coords(nz, R, D, q)
    lev = Level(nlon, fine_lat_edges(nlat), re, rc, 1.0)
    lev.M = alpha * np.broadcast_to(lev.V[:, :, None], lev.shape)
    lam = (np.arange(nlon) + 0.5) * lev.dlam
    r3, t3, l3 = np.meshgrid(rc, lev.theta, lam, indexing="ij")
    u = ufun(r3, t3, l3)
    Hu = apply(lev, u) / (lev.V[:, :, None])
    Lu = Lfun(r3, t3, l3)
    sel = (slice(*layers), rows(lev.theta), slice(None))
    return np.abs(Hu - Lu)[sel].max() / np.abs(Lu[sel]).max()


@pytest.mark.parametrize("case", ["lat", "lonlat", "radial"])
def test_operator_consistent_with_pde(case):
    """(Hu)_c / V_c -> (-lap + alpha) u at the cell centre, at second order.

    u = sin(th):              -lap u = 2 sin(th)/r^2
    u = cos(th) cos(lam):     -lap u = 2 u / r^2   (degree-1 spherical harmonic)
    u = r^2:                  -lap u = -6         (interior layers only)
    """
    alpha = 3.0
    if case == "lat":
        uf = lambda r, t, l: np.sin(t)
        Lf = lambda r, t, l: 2 * np.sin(t) / r ** 2 + alpha * np.sin(t)
        kw = dict(R=1.0, D=0.01, q=1.0, rows=lambda th: np.abs(th) < 1.2, layers=(0, None))
    elif case == "lonlat":
        uf = lambda r, t, l: np.cos(t) * np.cos(l)
        Lf = lambda r, t, l: (2 / r ** 2 + alpha) * np.cos(t) * np.cos(l)
        kw = dict(R=1.0, D=0.01, q=1.0, rows=lambda th: np.abs(th) < 1.2, layers=(0, None))
    else:
        uf = lambda r, t, l: r ** 2
        Lf = lambda r, t, l: -6.0 + alpha * r ** 2
        kw = dict(R=1.0, D=1.0, q=1.0, rows=lambda th: slice(None), layers=(1, -1))
    errs = []
    for n in (1, 2, 4):
        nz = 4 * n if case == "radial" else 2
        errs.append(_consistency_error(16 * n, 8 * n, nz, uf, Lf, alpha=alpha, **kw))
    assert errs[-1] < 2e-2
    if case == "radial":
        # a quadratic in r is reproduced exactly by the radial fluxes
        assert max(errs) < 1e-12, errs
    else:
        assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0, errs


def test_fine_mass_is_alpha_times_volume():
    sh = shellgen.workload("shell64x32x16").with_(alpha_const=None)
    a = shellgen.alpha(sh)
    lev = build_hierarchy(sh, a, levels=1)[0]
    np.testing.assert_array_equal(lev.M, a * lev.V[:, :, None])
