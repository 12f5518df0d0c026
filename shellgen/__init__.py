"""Seeded synthetic inputs for the spherical-shell Helmholtz solve.

This module is shared by the HIP path's tests/benchmarks and by the CPU
oracle. It holds only the workload shapes and the random draws; none of the
method's arithmetic (no geometry, no operator, no multigrid) lives here.

The paper's operational problem is the ENDGame pressure system on a
2560x1920x70 latitude-longitude grid (Section 2.4, Table 1). Its matrices are not
public, so every workload here is a synthetic shell of the same shape class:
unit radius, a thin shell, geometrically stretched vertical levels, a constant
diffusion coefficient K and a positive Helmholtz coefficient field alpha.

Random fields use numpy's PCG64 ``default_rng(seed)`` and have shape
``(nlev, nlat, nlon)``: index order [k][j][i] with longitude fastest.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

__all__ = [
    "Shell", "WORKLOADS", "workload", "rhs", "alpha", "weights",
    "fd_direction", "timestep", "SEED_RHS", "SEED_ALPHA", "SEED_W", "SEED_FD0",
    "SEED_STEP0",
]

SEED_RHS = 1
SEED_ALPHA = 2
SEED_W = 3
SEED_FD0 = 100
SEED_STEP0 = 1000


@dataclass(frozen=True)
class Shell:
    """Shape of one synthetic workload.

    nlon, nlat, nlev : cells in longitude, latitude and the vertical.
    radius           : inner radius of the shell (the planet's surface).
    thickness        : shell depth.
    stretch          : ratio between successive vertical layer depths,
                       counted upward from the surface.
    K                : scalar diffusion coefficient.
    alpha_const      : if not None, alpha is this constant everywhere;
                       otherwise alpha = alpha_scale*(1 + 0.5*U[0,1]).
    alpha_scale      : scale of the random alpha field.
    nu_pre, nu_post  : smoothing sweeps the workload's V-cycle uses.
    smooth           : interval [lo, hi] whose Chebyshev nodes give the
                       damping factors of the workload's smoothing sweeps.
    tol              : relative residual target of the workload's solve.
    """
    name: str
    nlon: int
    nlat: int
    nlev: int
    radius: float = 1.0
    thickness: float = 0.01
    stretch: float = 1.05
    K: float = 1.0
    alpha_const: float | None = None
    alpha_scale: float = 1e2
    nu_pre: int = 2
    nu_post: int = 2
    smooth: tuple[float, float] = (1.0 / 3.0, 2.0)
    tol: float = 1e-8

    @property
    def shape(self) -> tuple[int, int, int]:
        return (self.nlev, self.nlat, self.nlon)

    @property
    def n(self) -> int:
        return self.nlon * self.nlat * self.nlev

    def with_(self, **kw) -> "Shell":
        return replace(self, **kw)


WORKLOADS: dict[str, Shell] = {
    # Small plain-FP64 case: 32,768 unknowns, V(1,1) to 1e-5, constant alpha.
    "shell64x32x16": Shell("shell64x32x16", 64, 32, 16, stretch=1.1,
                           alpha_const=1e2, nu_pre=1, nu_post=1, tol=1e-5),
    # 5.16M unknowns, random alpha; also the adjoint/gradient workload.
    "shell384x192x70": Shell("shell384x192x70", 384, 192, 70, stretch=1.05),
    # N512-class global grid, 55M unknowns; stretch 1.07 puts the equatorial
    # horizontal-to-vertical spacing ratio near 1e3. Its V-cycle shape is not
    # fixed by the workload: V(2,4) with factors from [0.25, 2] reaches 1e-8
    # in 6 iterations (relres 6.8-7.5e-9 over six alpha and b seeds), V(2,3)
    # with [1/3, 2] in 7, V(2,2) in 9.
    "shell1024x768x70": Shell("shell1024x768x70", 1024, 768, 70, stretch=1.07, nu_post=4,
                              smooth=(0.25, 2.0)),
    # The operational 10 km grid shape of Table 1: 344M unknowns. V(2,3) with
    # [1/3, 2] reaches 1e-8 in 7 iterations; V(2,4) with [0.25, 2] also
    # needs 7 here, so the cheaper cycle stays.
    "shell2560x1920x70": Shell("shell2560x1920x70", 2560, 1920, 70, stretch=1.05, nu_post=3),
}


def workload(name: str) -> Shell:
    return WORKLOADS[name]


def rhs(shell: Shell, seed: int = SEED_RHS) -> np.ndarray:
    """Right-hand side b ~ U[-1,1], FP64, shape (nlev, nlat, nlon)."""
    return np.random.default_rng(seed).uniform(-1.0, 1.0, size=shell.shape)


def alpha(shell: Shell, seed: int = SEED_ALPHA) -> np.ndarray:
    """Helmholtz coefficient field: constant, or scale*(1 + 0.5*U[0,1])."""
    if shell.alpha_const is not None:
        return np.full(shell.shape, float(shell.alpha_const))
    u = np.random.default_rng(seed).uniform(0.0, 1.0, size=shell.shape)
    return shell.alpha_scale * (1.0 + 0.5 * u)


def weights(shell: Shell, seed: int = SEED_W) -> np.ndarray:
    """Loss weights w ~ N(0,1) for L = <w, u>."""
    return np.random.default_rng(seed).standard_normal(size=shell.shape)


def fd_direction(shell: Shell, m: int) -> np.ndarray:
    """Finite-difference direction number m ~ N(0,1), seed 100+m."""
    return np.random.default_rng(SEED_FD0 + m).standard_normal(size=shell.shape)


def timestep(shell: Shell, t: int, drift: float = 0.02) -> tuple[np.ndarray, np.ndarray]:
    """Inputs of step t >= 1 of a sequence of solves whose coefficients and
    right-hand side vary slowly, as in the solves of consecutive semi-implicit
    time steps (Section 1):
        alpha_t = alpha * (1 + drift * p_t),  p_t ~ U[-1,1], seed SEED_STEP0 + 2t
        b_t     = b + drift * q_t,            q_t ~ U[-1,1], seed SEED_STEP0 + 2t + 1
    with alpha = alpha(shell) and b = rhs(shell). Every alpha_t stays > 0."""
    p = np.random.default_rng(SEED_STEP0 + 2 * t).uniform(-1.0, 1.0, size=shell.shape)
    q = np.random.default_rng(SEED_STEP0 + 2 * t + 1).uniform(-1.0, 1.0, size=shell.shape)
    return alpha(shell) * (1.0 + drift * p), rhs(shell) + drift * q
