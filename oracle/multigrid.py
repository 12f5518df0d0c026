"""Multigrid V-cycle, its transpose, the outer iteration and the adjoint.

Test infrastructure (see the package docstring).

Paper steps followed:
  * Eq. (1), Section 2.1: the block-Jacobi smoother
        u <- u + omega H_z^{-1} (b - H u).
    The paper prints a minus sign in front of omega; with H and H_z both
    symmetric positive definite that iteration diverges (its error propagator
    is I + omega H_z^{-1} H), so the sign is read as +. With dH = 0 and
    omega = 1 one sweep from zero is then the exact solve.
  * Section 2: a V-cycle smooths, restricts the residual to a coarser grid,
    solves the coarse residual equation recursively, prolongates the
    correction and smooths again. Each outer iteration should reduce the
    residual norm ||b - Hu|| by about an order of magnitude.
  * Section 2.3: the coarsest grid is handled by "a simple iterative method";
    here n_c smoother sweeps (with the factor omega) from zero, n_c = 40 by
    default. Fewer leave enough coarse error to dominate the convergence
    factor once the smoother is good: with the Chebyshev factors below, 20
    sweeps let the factor climb from about 0.1 to 0.26 (1024x768x70 shell)
    and 0.48 (2560x1920x70, whose coarsest level stops at 5 longitudes,
    still anisotropic) after a few iterations, 40 keep it at or below 0.13
    on both, and 80 or 160 do no better.

Readings where the paper is silent:
  * restriction R sums the residuals of the children cells (the residual is
    an integrated, finite-volume quantity, so the sum is exactly the coarse
    cell's integral); prolongation P is cell-centred bilinear interpolation
    (linear in longitude; linear in latitude for merged rows, injection for
    rows coarsened in longitude only). Piecewise-constant P together with
    rediscretised coarse operators converges slowly or not at all on these
    shells, which is why the linear form is used; R is not P^T, so the
    V-cycle is not symmetric and its transpose differs from it;
  * V(nu1, nu2): the first pre-smoothing sweep starts from zero;
  * the damping factor: Eq. (1) leaves it open ("some" factor). By default
    the nu sweeps of a smoothing step use different factors, 1/lambda_k for
    the Chebyshev nodes lambda_k of [1/3, 2] (see sweep_omegas): the
    interval of eigenvalues of H_z^{-1} H on the modes the smoother must
    damp once latitude rows merge only with anisotropy up to 2 (the
    hierarchy module); for V(2,2) the factors are 0.570 and 1.732. A single
    factor for every sweep (omega = 0.8, the best constant among those tried)
    is the alternative (smooth_lo = 0): on the 1024x768x70 shell it needs 12
    outer iterations to 1e-8 against 9;
  * the outer stopping rule is the unweighted 2-norm ||b - Hu||_2 <=
    tol ||b||_2, evaluated after every outer iteration, starting from u = 0
    unless an initial guess is given;
  * adjoint of L = <w, u> with H(alpha) u = b: lambda = H^{-T} w = H^{-1} w,
    dL/db = lambda, dL/dalpha = -lambda * V * u (the derivative of H with
    respect to alpha at a cell is V at that cell's diagonal);
    lambda is computed by the same outer iteration with the transposed
    V-cycle, obtained by reversing the forward V-cycle step by step.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .geometry import Level
from .operator import apply, column_solve


@dataclass
class Options:
    nu_pre: int = 2
    nu_post: int = 2
    omega: float = 0.8
    coarse_sweeps: int = 40
    max_iters: int = 100
    # the interval [lo, hi] of the Chebyshev smoothing factors (see
    # sweep_omegas); lo = 0: every smoothing sweep uses omega
    smooth_lo: float = 1.0 / 3.0
    smooth_hi: float = 2.0


def sweep_omegas(opt: Options, nu: int):
    """Damping factor of each of the nu sweeps of one smoothing step.

    Eq. (1) leaves the factor open. With smooth_lo > 0 the nu sweeps use
    omega_k = 1/lambda_k for the nu Chebyshev nodes lambda_k of
    [smooth_lo, smooth_hi], largest first: the error of the nu sweeps is
    then multiplied by the degree-nu polynomial that is smallest, in the
    maximum norm, on that interval of eigenvalues of H_z^{-1} H, among those
    equal to 1 at 0. Otherwise, and for a step of a single sweep (where the
    degree-1 node 2/(lo + hi) = 0.857 converged worse than omega = 0.8 on the
    V(1,1) workload: factor 0.50 against 0.45), every sweep uses omega.
    """
    if opt.smooth_lo <= 0 or nu < 2:
        return [opt.omega] * nu
    lo, hi = opt.smooth_lo, opt.smooth_hi
    return [1.0 / (0.5 * (hi + lo) + 0.5 * (hi - lo) * np.cos(np.pi * (2 * k + 1) / (2 * nu)))
            for k in range(nu)]


# --- smoother -----------------------------------------------------------
def sweep(level: Level, x: np.ndarray, f: np.ndarray, omega: float):
    """One block-Jacobi sweep x <- x + omega H_z^{-1}(f - H x) (Eq. 1)."""
    return x + omega * column_solve(level, f - apply(level, x))


def sweep_from_zero(level: Level, f: np.ndarray, omega: float):
    """The sweep applied to x = 0: omega H_z^{-1} f."""
    return omega * column_solve(level, f)


def sweep_T(level: Level, xbar: np.ndarray, fbar: np.ndarray, omega: float):
    """Transpose of one sweep, in place on the adjoint variables.

    The sweep maps (x, f) -> x + omega H_z^{-1}(f - H x); with H and H_z
    symmetric its transpose sends xbar to xbar - omega H H_z^{-1} xbar and
    adds omega H_z^{-1} xbar to fbar.
    """
    z = column_solve(level, xbar)
    fbar += omega * z
    xbar -= omega * apply(level, z)


# --- transfers ----------------------------------------------------------
def restrict(fine: Level, coarse: Level, r: np.ndarray) -> np.ndarray:
    """R: sum over the children (two longitudes times the merged rows)."""
    rs = r[:, :, 0::2] + r[:, :, 1::2]
    out = np.empty(coarse.shape)
    for J in range(coarse.nlat):
        f0, cnt = coarse.child_first[J], coarse.child_count[J]
        out[:, J, :] = rs[:, f0:f0 + cnt, :].sum(axis=1)
    return out


def inject(fine: Level, coarse: Level, xc: np.ndarray) -> np.ndarray:
    """R^T: copy the coarse value into every child."""
    row_of = np.repeat(np.arange(coarse.nlat), coarse.child_count)
    return np.repeat(xc[:, row_of, :], 2, axis=2)


def prolong_weights(fine: Level, coarse: Level):
    """Cell-centred linear interpolation weights of P, per direction.

    Longitude: the fine cell 2I+s (s = 0, 1) lies a quarter of a coarse cell
    from the centre of coarse cell I toward I-1 (s = 0) or I+1 (s = 1), so it
    takes 3/4 of cell I and 1/4 of that neighbour (periodic).
    Latitude: a fine row that is the only child of its coarse row J has the
    same centre and takes row J alone; a child of a merged row J is
    interpolated linearly in theta between the centre of J and the centre of
    the neighbouring coarse row on its own side (J-1 south of th_J, J+1 north
    of it); next to a pole, where that neighbour does not exist, it takes J
    alone.
    Returns (rows_th (nlat_f, 2), w_th (nlat_f, 2)) with the second entry's
    weight 0 where unused.
    """
    thc, thf = coarse.theta, fine.theta
    nJc = coarse.nlat
    row_of = np.repeat(np.arange(nJc), coarse.child_count)
    rows = np.zeros((fine.nlat, 2), dtype=np.int64)
    w = np.zeros((fine.nlat, 2))
    for j in range(fine.nlat):
        J = row_of[j]
        rows[j] = (J, J)
        w[j] = (1.0, 0.0)
        if coarse.child_count[J] == 2:
            nb = J - 1 if thf[j] < thc[J] else J + 1
            if 0 <= nb < nJc:
                wj = (thf[j] - thc[nb]) / (thc[J] - thc[nb])
                rows[j] = (J, nb)
                w[j] = (wj, 1.0 - wj)
    return rows, w


def prolong(fine: Level, coarse: Level, xc: np.ndarray) -> np.ndarray:
    """P: bilinear (cell-centred) interpolation of a coarse correction."""
    rows, w = prolong_weights(fine, coarse)
    xt = (w[None, :, 0, None] * xc[:, rows[:, 0], :]
          + w[None, :, 1, None] * xc[:, rows[:, 1], :])      # (nz, nJf, nIc)
    out = np.empty(fine.shape)
    out[:, :, 0::2] = 0.75 * xt + 0.25 * np.roll(xt, 1, axis=2)
    out[:, :, 1::2] = 0.75 * xt + 0.25 * np.roll(xt, -1, axis=2)
    return out


def prolong_T(fine: Level, coarse: Level, x: np.ndarray) -> np.ndarray:
    """P^T applied to a fine vector (the transpose of ``prolong``)."""
    rows, w = prolong_weights(fine, coarse)
    ev, od = x[:, :, 0::2], x[:, :, 1::2]
    # transpose of the longitude step: coarse I collects 3/4 of its two
    # children and 1/4 of the nearer child of each neighbour
    xt = 0.75 * (ev + od) + 0.25 * np.roll(ev, -1, axis=2) \
        + 0.25 * np.roll(od, 1, axis=2)                      # (nz, nJf, nIc)
    out = np.zeros(coarse.shape)
    for j in range(fine.nlat):
        out[:, rows[j, 0], :] += w[j, 0] * xt[:, j, :]
        out[:, rows[j, 1], :] += w[j, 1] * xt[:, j, :]
    return out


# --- V-cycle --------------------------------------------------------------
def coarse_solve(level: Level, f: np.ndarray, opt: Options):
    x = sweep_from_zero(level, f, opt.omega)
    for _ in range(opt.coarse_sweeps - 1):
        x = sweep(level, x, f, opt.omega)
    return x


def coarse_solve_T(level: Level, g: np.ndarray, opt: Options):
    xbar = g.copy()
    fbar = np.zeros_like(g)
    for _ in range(opt.coarse_sweeps - 1):
        sweep_T(level, xbar, fbar, opt.omega)
    fbar += opt.omega * column_solve(level, xbar)
    return fbar


def vcycle(levels, f: np.ndarray, opt: Options, l: int = 0) -> np.ndarray:
    """Approximate H_l^{-1} f by one V(nu_pre, nu_post) cycle from zero."""
    lev = levels[l]
    if l == len(levels) - 1:
        return coarse_solve(lev, f, opt)
    pre, post = sweep_omegas(opt, opt.nu_pre), sweep_omegas(opt, opt.nu_post)
    x = sweep_from_zero(lev, f, pre[0])
    for w in pre[1:]:
        x = sweep(lev, x, f, w)
    fc = restrict(lev, levels[l + 1], f - apply(lev, x))
    xc = vcycle(levels, fc, opt, l + 1)
    x = x + prolong(lev, levels[l + 1], xc)
    for w in post:
        x = sweep(lev, x, f, w)
    return x


def vcycle_T(levels, g: np.ndarray, opt: Options, l: int = 0) -> np.ndarray:
    """Transpose of the linear map f -> vcycle(f), applied to g.

    The forward steps are undone in reverse order: the post-sweeps, the
    prolongation (transpose P^T), the coarse cycle, the residual
    restriction (whose transpose adds R^T fc_bar to fbar and subtracts
    H R^T fc_bar from xbar), the later pre-sweeps and finally the first sweep from zero.
    """
    lev = levels[l]
    if l == len(levels) - 1:
        return coarse_solve_T(lev, g, opt)
    pre, post = sweep_omegas(opt, opt.nu_pre), sweep_omegas(opt, opt.nu_post)
    xbar = g.copy()
    fbar = np.zeros_like(g)
    for w in reversed(post):
        sweep_T(lev, xbar, fbar, w)
    xc_bar = prolong_T(lev, levels[l + 1], xbar)
    fc_bar = vcycle_T(levels, xc_bar, opt, l + 1)
    y = inject(lev, levels[l + 1], fc_bar)
    fbar += y
    xbar -= apply(lev, y)
    for w in reversed(pre[1:]):
        sweep_T(lev, xbar, fbar, w)
    fbar += pre[0] * column_solve(lev, xbar)
    return fbar


# --- outer iteration ---------------------------------------------------------
def _outer(levels, b, opt, tol, u0, cycle, fixed_iters):
    fine = levels[0]
    u = np.zeros(fine.shape) if u0 is None else np.array(u0, dtype=np.float64)
    r = b - apply(fine, u)
    bnorm = np.linalg.norm(b.ravel())
    hist = [np.linalg.norm(r.ravel())]
    it = 0
    while True:
        if fixed_iters is not None:
            if it >= fixed_iters:
                break
        elif hist[-1] <= tol * bnorm or it >= opt.max_iters:
            break
        u = u + cycle(levels, r, opt)
        r = b - apply(fine, u)
        hist.append(np.linalg.norm(r.ravel()))
        it += 1
    return u, {"iters": it, "res_hist": np.array(hist), "bnorm": bnorm,
               "relres": hist[-1] / bnorm if bnorm > 0 else 0.0}


def solve(levels, b, opt: Options | None = None, tol: float = 1e-8, u0=None,
          fixed_iters: int | None = None):
    """Multigrid outer iteration u <- u + V(b - H u) until the relative
    residual drops below tol (or a fixed number of iterations)."""
    return _outer(levels, b, opt or Options(), tol, u0, vcycle, fixed_iters)


def solve_adjoint(levels, w, opt: Options | None = None, tol: float = 1e-8,
                  fixed_iters: int | None = None):
    """lambda = H^{-T} w by the outer iteration with the transposed V-cycle."""
    return _outer(levels, w, opt or Options(), tol, None, vcycle_T, fixed_iters)


def cell_volumes(levels) -> np.ndarray:
    fine = levels[0]
    return np.broadcast_to(fine.V[:, :, None], fine.shape).copy()


def grad_alpha(levels, lam: np.ndarray, u: np.ndarray) -> np.ndarray:
    """dL/dalpha = -lambda * V * u."""
    return -lam * levels[0].V[:, :, None] * u


def convergence_factors(res_hist) -> np.ndarray:
    """rho_m = ||r_m|| / ||r_{m-1}|| for m >= 1."""
    h = np.asarray(res_hist, dtype=np.float64)
    return h[1:] / h[:-1]
