"""Pins for the oracle's operator H, its split H = H_z + dH (Section 2.1) and
the column (vertical-line) solves.

H 1 = M, symmetry and positivity, agreement of the difference-form apply with
a face-by-face assembled matrix, dense tridiagonal solves, exact rational
arithmetic on an ill-conditioned column, and the Eq. (1) special case dH = 0.
"""
from fractions import Fraction

import numpy as np
import pytest

import shellgen
from oracle import (build_hierarchy, apply, assemble, mtilde, column_pivots,
                    column_solve, sweep_from_zero)
from oracle.geometry import Level


def _hier(nlon, nlat, nz, q=1.1, D=0.01, seed=5, levels=0):
    sh = shellgen.Shell("t", nlon, nlat, nz, stretch=q, thickness=D)
    a = shellgen.alpha(sh, seed)
    return sh, build_hierarchy(sh, a, levels=levels)


@pytest.mark.parametrize("dims", [(8, 4, 3), (16, 8, 5), (64, 32, 16)])
def test_constant_vector_gives_mass(dims):
    _, L = _hier(*dims)
    for lev in L:
        one = np.ones(lev.shape)
        np.testing.assert_allclose(apply(lev, one), lev.M, rtol=1e-9,
                                   atol=1e-12 * np.abs(lev.M).max())


@pytest.mark.parametrize("dims", [(8, 4, 3), (16, 8, 5), (2, 2, 3), (12, 6, 1)])
def test_apply_matches_assembled_symmetric_spd(dims):
    _, L = _hier(*dims)
    rng = np.random.default_rng(0)
    for lev in L:
        A = assemble(lev)
        x = rng.standard_normal(lev.shape)
        np.testing.assert_allclose(A @ x.ravel(), apply(lev, x).ravel(),
                                   rtol=1e-12, atol=1e-12 * np.abs(A).max())
        assert abs(A - A.T).max() == 0.0
        if A.shape[0] <= 800:
            ev = np.linalg.eigvalsh(A.toarray())
            assert ev.min() > 0
        # split: H = H_z + dH, and H_z's diagonal excess is mtilde
        Hz, dH = assemble(lev, "Hz"), assemble(lev, "dH")
        assert abs(Hz + dH - A).max() <= 1e-12 * abs(A).max()
        diag = Hz.diagonal().reshape(lev.shape)
        Tr = lev.Tr[:, :, None]
        np.testing.assert_allclose(diag, Tr[:-1] + Tr[1:] + mtilde(lev), rtol=1e-13)


def test_column_solve_matches_dense_tridiagonal():
    _, L = _hier(16, 8, 9, q=1.2, D=0.2)
    rng = np.random.default_rng(1)
    for lev in L:
        s = rng.standard_normal(lev.shape)
        x = column_solve(lev, s)
        Hz = assemble(lev, "Hz").toarray()
        nz, nJ, nI = lev.shape
        for J in range(nJ):
            for i in range(0, nI, max(1, nI // 3)):
                idx = [(k * nJ + J) * nI + i for k in range(nz)]
                T = Hz[np.ix_(idx, idx)]
                # only the column's own couplings: tridiagonal
                assert np.count_nonzero(np.triu(T, 2)) == 0
                xd = np.linalg.solve(T, s[:, J, i])
                np.testing.assert_allclose(x[:, J, i], xd, rtol=1e-11,
                                           atol=1e-13 * np.abs(xd).max())


def _exact_tridiag_solve(Tr, mt, s):
    """Exact rational Gaussian elimination of one column."""
    n = len(mt)
    F = [Fraction(v) for v in s]
    T = [Fraction(v) for v in Tr]
    m = [Fraction(v) for v in mt]
    diag = [T[k] + T[k + 1] + m[k] for k in range(n)]
    sub = [-T[k] for k in range(n)]          # A[k, k-1]
    sup = [-T[k + 1] for k in range(n)]      # A[k, k+1]
    for k in range(1, n):
        f = sub[k] / diag[k - 1]
        diag[k] -= f * sup[k - 1]
        F[k] -= f * F[k - 1]
    x = [Fraction(0)] * n
    x[n - 1] = F[n - 1] / diag[n - 1]
    for k in range(n - 2, -1, -1):
        x[k] = (F[k] - sup[k] * x[k + 1]) / diag[k]
    return np.array([float(v) for v in x])


def test_row_sum_pivots_on_ill_conditioned_column():
    """Vertical couplings 1e9 times the diagonal excess (thin shell): the
    solve and the row-sum pivots keep full FP64 accuracy against exact
    rational arithmetic, while the textbook pivots D_k - T^2/p_{k-1} lose
    digits to cancellation in the last pivot (where no coupling is left to
    hide the mass term)."""
    nz = 7
    rng = np.random.default_rng(2)
    Tr = np.concatenate([[0.0], rng.uniform(1e9, 3e9, nz - 1), [0.0]])
    mt = rng.uniform(0.5, 1.5, nz)
    s = rng.standard_normal(nz)
    lev = Level.__new__(Level)
    lev.nz = nz
    lev.Tr = Tr[:, None]
    lev.M = mt[:, None, None]
    lev.Tlam = np.zeros((nz, 1))
    lev.Tth = np.zeros((nz, 2))
    lev._pivots = None
    x = column_solve(lev, s[:, None, None])[:, 0, 0]
    xe = _exact_tridiag_solve(Tr, mt, s)
    np.testing.assert_allclose(x, xe, rtol=1e-13)
    p = column_pivots(lev)[:, 0, 0]
    T = [Fraction(v) for v in Tr]
    D = [T[k] + T[k + 1] + Fraction(mt[k]) for k in range(nz)]
    pex = [D[0]]
    for k in range(1, nz):
        pex.append(D[k] - T[k] * T[k] / pex[-1])
    pex = np.array([float(v) for v in pex])
    np.testing.assert_allclose(p, pex, rtol=1e-14)
    Df = Tr[:-1] + Tr[1:] + mt
    ptext = [Df[0]]
    for k in range(1, nz):
        ptext.append(Df[k] - Tr[k] ** 2 / ptext[-1])
    assert abs(ptext[-1] - pex[-1]) / pex[-1] > 1e-10


def test_eq1_without_horizontal_coupling_is_exact_solve():
    """With dH = 0 and omega = 1, one sweep of Eq. (1) from zero is H^{-1} f."""
    _, L = _hier(8, 4, 6, q=1.3, D=0.1)
    lev = L[0]
    lev.Tlam = np.zeros_like(lev.Tlam)
    lev.Tth = np.zeros_like(lev.Tth)
    lev._pivots = None
    f = np.random.default_rng(3).standard_normal(lev.shape)
    x = sweep_from_zero(lev, f, 1.0)
    xd = np.linalg.solve(assemble(lev).toarray(), f.ravel())
    np.testing.assert_allclose(x.ravel(), xd, rtol=1e-12, atol=1e-14 * np.abs(xd).max())
