"""Pins for the oracle's V-cycle, outer iteration and adjoint (Sections 2,
2.1, 2.3 and the implicit-function adjoint of L = <w, u>).

The solve is pinned to the plain definition u = H^{-1} b (dense and sparse
direct solves), manufactured solutions, the transfer and V-cycle transposes
by dot-product tests, the adjoint against a direct solve and central finite
differences, and the convergence factor per V-cycle.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import shellgen
from oracle import (build_hierarchy, apply, assemble, Options, solve,
                    solve_adjoint, vcycle, vcycle_T, restrict, inject, prolong,
                    prolong_T, grad_alpha, convergence_factors, prolong_weights)


def _setup(nlon, nlat, nz, q=1.1, D=0.01, seed=4):
    sh = shellgen.Shell("t", nlon, nlat, nz, stretch=q, thickness=D)
    return sh, build_hierarchy(sh, shellgen.alpha(sh, seed))


@pytest.mark.parametrize("dims", [(8, 4, 3), (16, 8, 5), (24, 12, 4)])
def test_solve_matches_dense_direct(dims):
    sh, L = _setup(*dims)
    b = shellgen.rhs(sh)
    u, st = solve(L, b, Options(nu_pre=1, nu_post=1), tol=1e-13)
    ud = np.linalg.solve(assemble(L[0]).toarray(), b.ravel()).reshape(sh.shape)
    assert st["relres"] <= 1e-13
    np.testing.assert_allclose(u, ud, rtol=0, atol=1e-10 * np.abs(ud).max())


def test_solve_matches_sparse_direct_small_shell():
    sh = shellgen.workload("shell64x32x16")
    L = build_hierarchy(sh, shellgen.alpha(sh))
    b = shellgen.rhs(sh)
    opt = Options(nu_pre=sh.nu_pre, nu_post=sh.nu_post)
    u, st = solve(L, b, opt, tol=1e-12)
    ud = spla.splu(assemble(L[0]).tocsc()).solve(b.ravel()).reshape(sh.shape)
    assert np.linalg.norm(u - ud) / np.linalg.norm(ud) < 1e-10
    # the workload's own target: relative residual 1e-5 with V(1,1)
    u5, st5 = solve(L, b, opt, tol=sh.tol)
    assert st5["relres"] <= sh.tol and st5["iters"] <= 12


def test_manufactured_solution():
    sh, L = _setup(32, 16, 6, q=1.15)
    lam = (np.arange(32) + 0.5) * 2 * np.pi / 32
    th = L[0].theta
    rc = L[0].r_centre
    ustar = (np.cos(th)[None, :, None] * np.cos(lam)[None, None, :]
             * ((rc - rc[0]) / 0.01)[:, None, None]
             + np.random.default_rng(7).standard_normal(sh.shape))
    b = apply(L[0], ustar)
    u, st = solve(L, b, Options(), tol=1e-13)
    assert np.linalg.norm(u - ustar) / np.linalg.norm(ustar) < 1e-9


def test_transfers_are_transposes_and_interpolate():
    sh, L = _setup(48, 24, 3)
    rng = np.random.default_rng(8)
    for f, c in zip(L[:-1], L[1:]):
        x, y = rng.standard_normal(f.shape), rng.standard_normal(c.shape)
        assert np.vdot(restrict(f, c, x), y) == pytest.approx(np.vdot(x, inject(f, c, y)),
                                                              rel=1e-13)
        assert np.vdot(prolong(f, c, y), x) == pytest.approx(np.vdot(y, prolong_T(f, c, x)),
                                                             rel=1e-13)
        # P reproduces constants and fields linear in longitude / latitude
        np.testing.assert_allclose(prolong(f, c, np.ones(c.shape)), 1.0, rtol=1e-14)
        lamc = (np.arange(c.nlon) + 0.5) * c.dlam
        lamf = (np.arange(f.nlon) + 0.5) * f.dlam
        vc = np.broadcast_to(np.sin(lamc), c.shape)
        got = prolong(f, c, vc)[0, 0]
        want = 0.75 * np.sin(lamc).repeat(2) + 0.25 * np.sin(
            np.roll(lamc, 1)).repeat(2) * (np.arange(f.nlon) % 2 == 0) + 0.25 * np.sin(
            np.roll(lamc, -1)).repeat(2) * (np.arange(f.nlon) % 2 == 1)
        np.testing.assert_allclose(got, want, rtol=1e-13)
        tc = np.broadcast_to(c.theta[None, :, None], c.shape)
        pt = prolong(f, c, tc)[0, :, 0]
        rows, w = prolong_weights(f, c)
        interior = (w[:, 1] != 0)
        np.testing.assert_allclose(pt[interior], f.theta[interior], rtol=1e-13, atol=1e-15)
        # rows not interpolated in latitude are single children: same centre
        single = c.child_count[rows[:, 0]] == 1
        np.testing.assert_allclose(pt[single], f.theta[single], rtol=1e-13, atol=1e-15)
        # R of a constant field is the child count
        cnt = 2 * c.child_count
        np.testing.assert_allclose(restrict(f, c, np.ones(f.shape))[0, :, 0], cnt)


@pytest.mark.parametrize("nu", [(1, 1), (2, 2), (2, 1), (0, 3)])
def test_vcycle_transpose_dot_product(nu):
    sh, L = _setup(32, 16, 5, q=1.2)
    opt = Options(nu_pre=max(nu[0], 1), nu_post=nu[1], coarse_sweeps=4)
    rng = np.random.default_rng(9)
    x, y = rng.standard_normal(sh.shape), rng.standard_normal(sh.shape)
    lhs = np.vdot(vcycle(L, x, opt), y)
    rhs = np.vdot(x, vcycle_T(L, y, opt))
    assert lhs == pytest.approx(rhs, rel=1e-12)
    # the V-cycle is linear
    a, b = 0.3, -1.7
    np.testing.assert_allclose(vcycle(L, a * x + b * y, opt),
                               a * vcycle(L, x, opt) + b * vcycle(L, y, opt),
                               rtol=1e-9, atol=1e-12 * np.abs(vcycle(L, x, opt)).max())


def test_vcycle_not_symmetric_since_R_is_not_PT():
    sh, L = _setup(32, 16, 5)
    rng = np.random.default_rng(10)
    x, y = rng.standard_normal(sh.shape), rng.standard_normal(sh.shape)
    opt = Options()
    assert abs(np.vdot(vcycle(L, x, opt), y) - np.vdot(x, vcycle(L, y, opt))) > \
        1e-6 * abs(np.vdot(vcycle(L, x, opt), y))


def test_convergence_factor():
    """Section 2: each outer iteration reduces the residual by a large factor.

    Damped block-Jacobi bounds the smoothing factor per sweep from below
    (about 0.6-0.73, see the hierarchy module); V(1,1) on the small shell
    (constant omega, a one-sweep step) measures below 0.45. V(2,2) and V(2,3)
    on a 70-level medium shell (reduced horizontally), with the default
    per-sweep Chebyshev factors, must stay below 0.2 per cycle (measured:
    at most 0.103 and 0.074)."""
    sh = shellgen.workload("shell64x32x16")
    L = build_hierarchy(sh, shellgen.alpha(sh))
    _, st = solve(L, shellgen.rhs(sh), Options(nu_pre=1, nu_post=1), tol=1e-11)
    rho = convergence_factors(st["res_hist"])
    assert rho.max() < 0.45, rho
    sh2 = shellgen.workload("shell384x192x70").with_(nlon=192, nlat=96)
    L2 = build_hierarchy(sh2, shellgen.alpha(sh2))
    _, st2 = solve(L2, shellgen.rhs(sh2), Options(), tol=1e-11, fixed_iters=8)
    rho2 = convergence_factors(st2["res_hist"])
    assert rho2.max() < 0.2, rho2
    _, st3 = solve(L2, shellgen.rhs(sh2), Options(nu_post=3), tol=1e-11, fixed_iters=8)
    rho3 = convergence_factors(st3["res_hist"])
    assert rho3.max() < 0.2, rho3


def test_convergence_insensitive_to_vertical_geometry():
    """Section 2.1: with horizontal-only coarsening the rate is set by the
    horizontal, not the vertical, coupling: shell depth and stretching
    barely change it."""
    out = []
    for D, q in [(0.01, 1.1), (0.001, 1.1), (0.01, 1.0), (0.05, 1.2)]:
        sh = shellgen.Shell("t", 64, 32, 16, thickness=D, stretch=q, alpha_const=1e2)
        L = build_hierarchy(sh, shellgen.alpha(sh))
        _, st = solve(L, shellgen.rhs(sh), Options(nu_pre=1, nu_post=1), fixed_iters=8)
        out.append(convergence_factors(st["res_hist"])[-3:].mean())
    assert max(out) - min(out) < 0.08, out


def test_adjoint_matches_direct_and_finite_differences():
    sh, L = _setup(16, 8, 5, q=1.2, D=0.05)
    a = shellgen.alpha(sh, 4)
    b, w = shellgen.rhs(sh), shellgen.weights(sh)
    u, _ = solve(L, b, Options(), tol=1e-14)
    lam, st = solve_adjoint(L, w, Options(), tol=1e-14)
    A = assemble(L[0]).toarray()
    np.testing.assert_allclose(lam.ravel(), np.linalg.solve(A.T, w.ravel()),
                               rtol=0, atol=1e-11 * np.abs(lam).max())
    g = grad_alpha(L, lam, u)

    def loss(alpha, bb):
        LL = build_hierarchy(sh, alpha)
        uu, _ = solve(LL, bb, Options(), fixed_iters=30)
        return np.vdot(w, uu)

    h = 1e-6
    for m in range(3):
        d = shellgen.fd_direction(sh, m)
        fd_b = (loss(a, b + h * d) - loss(a, b - h * d)) / (2 * h)
        assert fd_b == pytest.approx(np.vdot(lam, d), rel=1e-7)
        fd_a = (loss(a * (1 + h * d), b) - loss(a * (1 - h * d), b)) / (2 * h)
        assert fd_a == pytest.approx(np.vdot(g, a * d), rel=1e-6)


def test_chebyshev_sweep_factors_closed_form():
    """With a smoothing interval [lo, hi] the nu sweeps of one smoothing step
    multiply an eigencomponent lambda of H_z^{-1} H by prod_k (1 - w_k
    lambda), which must be the Chebyshev polynomial of degree nu on [lo, hi],
    scaled to 1 at lambda = 0 (closed form T_nu(z) = cos(nu arccos z) inside
    the interval, cosh(nu arccosh z) outside)."""
    from oracle import sweep_omegas
    lo, hi = 1.0 / 3.0, 2.0
    opt = Options(smooth_lo=lo, smooth_hi=hi)
    # a single sweep keeps omega
    assert sweep_omegas(opt, 1) == [opt.omega]
    for nu in (2, 3, 4):
        w = np.array(sweep_omegas(opt, nu))
        lam = np.linspace(0.0, 2.5, 101)
        got = np.prod(1.0 - np.outer(lam, w), axis=1)
        z = (hi + lo - 2.0 * lam) / (hi - lo)
        t_nu = np.where(np.abs(z) <= 1, np.cos(nu * np.arccos(np.clip(z, -1, 1))),
                        np.sign(z) ** nu * np.cosh(nu * np.arccosh(np.maximum(np.abs(z), 1))))
        z0 = (hi + lo) / (hi - lo)
        want = t_nu / np.cosh(nu * np.arccosh(z0))
        np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-13)
    # largest eigenvalue node first: the smallest factor leads
    assert np.all(np.diff(sweep_omegas(opt, 3)) > 0)
    # no interval: every sweep uses omega
    assert sweep_omegas(Options(omega=0.7, smooth_lo=0.0), 3) == [0.7, 0.7, 0.7]


def _transposed_as_forward(L, g, opt, l=0):
    """The transposed V-cycle in the shape of a forward one: with H and H_z
    symmetric a transposed sweep is a forward sweep on the right-hand side
    xbar (its iterate fbar, its residual xbar), so the reversed chain of
    transposed sweeps is a chain of forward sweeps from zero with the
    factors reversed; the transfers enter transposed (P^T restricts the
    residual, R^T = injection prolongates)."""
    from oracle.multigrid import coarse_solve, sweep, sweep_from_zero, sweep_omegas
    lev = L[l]
    if l == len(L) - 1:
        return coarse_solve(lev, g, opt)
    pre, post = sweep_omegas(opt, opt.nu_pre), sweep_omegas(opt, opt.nu_post)
    x = np.zeros_like(g)
    for i, w in enumerate(reversed(post)):
        x = sweep_from_zero(lev, g, w) if i == 0 else sweep(lev, x, g, w)
    xc = _transposed_as_forward(L, prolong_T(lev, L[l + 1], g - apply(lev, x)), opt, l + 1)
    x = x + inject(lev, L[l + 1], xc)
    for w in reversed(pre):
        x = sweep(lev, x, g, w)
    return x


@pytest.mark.parametrize("nu", [(1, 1), (2, 2), (2, 1), (1, 3), (2, 4), (2, 0)])
@pytest.mark.parametrize("interval", [(1 / 3, 2.0), (0.0, 2.0)], ids=["chebyshev", "constant"])
def test_transposed_cycle_is_a_forward_cycle(nu, interval):
    """The step-by-step transposed V-cycle equals the forward-shaped one
    (swapped smoothing steps with reversed factors, transposed transfers),
    the form the GPU path computes, on a ragged hierarchy."""
    sh, L = _setup(36, 18, 6, q=1.15)
    opt = Options(nu_pre=nu[0], nu_post=nu[1], coarse_sweeps=5, smooth_lo=interval[0],
                  smooth_hi=interval[1])
    g = np.random.default_rng(23).standard_normal(sh.shape)
    ref = vcycle_T(L, g, opt)
    got = _transposed_as_forward(L, g, opt)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("nu", [(2, 2), (2, 1)])
def test_chebyshev_vcycle_transpose_and_convergence(nu):
    sh, L = _setup(32, 16, 5, q=1.2)
    opt = Options(nu_pre=nu[0], nu_post=nu[1], coarse_sweeps=4, smooth_lo=1 / 3, smooth_hi=2.0)
    rng = np.random.default_rng(19)
    x, y = rng.standard_normal(sh.shape), rng.standard_normal(sh.shape)
    assert np.vdot(vcycle(L, x, opt), y) == pytest.approx(np.vdot(x, vcycle_T(L, y, opt)),
                                                          rel=1e-12)
    if nu == (2, 2):
        # the schedule damps the smoothing range better than a constant
        # factor: smaller convergence factors once the first, white-noise
        # dominated iteration is past
        sh2 = shellgen.workload("shell384x192x70").with_(nlon=192, nlat=96)
        L2 = build_hierarchy(sh2, shellgen.alpha(sh2))
        b = shellgen.rhs(sh2)
        _, st_c = solve(L2, b, Options(smooth_lo=0.0), tol=1e-11, fixed_iters=6)
        _, st_t = solve(L2, b, Options(smooth_lo=1 / 3, smooth_hi=2.0), tol=1e-11,
                        fixed_iters=6)
        rho_c = convergence_factors(st_c["res_hist"])[-3:]
        rho_t = convergence_factors(st_t["res_hist"])[-3:]
        assert rho_t.max() < 0.12 and rho_t.max() < 0.8 * rho_c.min(), (rho_c, rho_t)


def test_timestep_inputs_and_warm_start():
    """The time-step sequence (shellgen.timestep): seeded, alpha_t > 0 within
    2 % of alpha, b_t within 0.02 of b; the oracle's solve of step t started
    from the solution of step t-1 needs fewer iterations than from zero."""
    sh = shellgen.workload("shell64x32x16")
    a0, b0 = shellgen.alpha(sh), shellgen.rhs(sh)
    opt = Options(nu_pre=sh.nu_pre, nu_post=sh.nu_post)
    u, _ = solve(build_hierarchy(sh, a0), b0, opt, tol=1e-8)
    for step in (1, 2):
        a, b = shellgen.timestep(sh, step)
        a2, b2 = shellgen.timestep(sh, step)
        assert np.array_equal(a, a2) and np.array_equal(b, b2)
        assert (a > 0).all() and np.abs(a / a0 - 1).max() <= 0.02
        assert np.abs(b - b0).max() <= 0.02
        Lt = build_hierarchy(sh, a)
        uw, sw = solve(Lt, b, opt, tol=1e-8, u0=u)
        _, sc = solve(Lt, b, opt, tol=1e-8)
        assert sw["relres"] <= 1e-8
        assert sw["iters"] < sc["iters"]
        u = uw
