"""GPU tests of the pure single-precision solve (MG_PREC_FP32) and of the
paper's shallow four-level hierarchy (Section 2.3), against the oracle.

Pure FP32. b, u and b - H u are all FP32. The V-cycle is the mixed
solve's, so until FP32 rounding matters the residual history must follow
the mixed solve's. It then stalls at the floor that rounding the iterate
to FP32 sets. That floor is pinned by the oracle, independently of the
solver: ||H (u* - fl32(u*))|| / ||b||, the residual of the exact solution
u* rounded to FP32. Here u* is the oracle's solve to 1e-11. The stall
must sit within a factor of 2 of that prediction (measured: within 2 %),
and it must stay there without diverging.

Shallow hierarchy. With levels=4 the V-cycle must still match the oracle's
four-level V-cycle element by element. It converges much more slowly than
the automatic hierarchy on these shells: their alpha gives horizontal
Courant numbers far above the paper's, so a 4-level coarsest grid is not
yet coarse enough.
"""
import functools

import numpy as np
import pytest

import shellgen
import oracle
from gpu_util import log, t, n, solver_for, rel_inf, opts_of

pytestmark = pytest.mark.gpu

SMALL = shellgen.workload("shell64x32x16")
MEDIUM = shellgen.workload("shell384x192x70")


@functools.lru_cache(maxsize=4)
def levels_of(sh, levels=0):
    return oracle.build_hierarchy(sh, shellgen.alpha(sh), levels=levels)


@functools.lru_cache(maxsize=2)
def exact_solution(sh):
    L = levels_of(sh)
    u, st = oracle.solve(L, shellgen.rhs(sh), opts_of(sh), tol=1e-11)
    return u


def rounding_floor(sh):
    """||H (u* - fl32(u*))|| / ||b||: the residual of the exact solution
    rounded to FP32."""
    L = levels_of(sh)
    u = exact_solution(sh)
    d = u - u.astype(np.float32).astype(np.float64)
    b = shellgen.rhs(sh)
    return np.linalg.norm(oracle.apply(L[0], d).ravel()) / np.linalg.norm(b.ravel())


@pytest.mark.parametrize("sh", [SMALL, MEDIUM], ids=lambda s: s.name)
def test_fp32_solve_follows_mixed_then_stalls_at_rounding_floor(sh):
    a, b = shellgen.alpha(sh), shellgen.rhs(sh)
    L = levels_of(sh)
    bnorm = np.linalg.norm(b.ravel())
    S32 = solver_for(sh, a, precision="fp32", nu_pre=sh.nu_pre, nu_post=sh.nu_post,
                     max_iters=12)
    Smx = solver_for(sh, a, precision="mixed", nu_pre=sh.nu_pre, nu_post=sh.nu_post,
                     max_iters=12)
    u32, st32 = S32.solve(t(b), tol=1e-12)
    _, stmx = Smx.solve(t(b), tol=1e-12)
    h32 = np.array(st32.res_hist[:st32.iters + 1]) / bnorm
    hmx = np.array(stmx.res_hist[:stmx.iters + 1]) / bnorm
    floor = rounding_floor(sh)
    host = np.linalg.norm((b - oracle.apply(L[0], n(u32))).ravel()) / bnorm
    log(f"{sh.name} fp32 history {' '.join(f'{v:.1e}' for v in h32)}")
    log(f"{sh.name} mixed history {' '.join(f'{v:.1e}' for v in hmx)}")
    log(f"{sh.name} predicted FP32 floor {floor:.2e}, stall {h32[-1]:.2e}, "
        f"oracle residual of the FP32 result {host:.2e}")
    assert st32.status == 1          # MG_ERR_NOT_CONVERGED: 1e-12 is below the floor
    assert st32.iters == 12
    # the same cycle: the same contraction while the residual is far above the floor
    for m in range(1, 4):
        if hmx[m] > 30 * floor:
            assert h32[m] == pytest.approx(hmx[m], rel=0.05)
    # the stall is the rounding floor, and it holds without diverging
    assert 0.5 * floor < h32[-1] < 2 * floor
    assert h32[-4:].max() < 2 * h32[-4:].min()
    # what the solver reports is what the returned u achieves in FP64
    assert host == pytest.approx(h32[-1], rel=0.05)


@pytest.mark.parametrize("sh", [SMALL, MEDIUM], ids=lambda s: s.name)
def test_fp32_solve_above_the_floor_matches_mixed(sh):
    a, b = shellgen.alpha(sh), shellgen.rhs(sh)
    L = levels_of(sh)
    bnorm = np.linalg.norm(b.ravel())
    tol = 2e-3
    u32, st32 = solver_for(sh, a, precision="fp32").solve(t(b), tol=tol)
    _, stmx = solver_for(sh, a, precision="mixed").solve(t(b), tol=tol)
    host = np.linalg.norm((b - oracle.apply(L[0], n(u32))).ravel()) / bnorm
    log(f"{sh.name} tol {tol:g}: fp32 iters {st32.iters} relres {st32.relres:.2e} "
        f"(oracle {host:.2e}); mixed iters {stmx.iters}")
    assert st32.status == 0
    assert st32.iters == stmx.iters
    assert host <= tol * 1.01


def test_shallow_hierarchy_vcycle_and_convergence_match_oracle():
    sh = MEDIUM
    a, b = shellgen.alpha(sh), shellgen.rhs(sh)
    L4 = levels_of(sh, 4)
    assert len(L4) == 4
    opt = opts_of(sh)
    S = solver_for(sh, a, precision="fp64", levels=4)
    got = n(S.vcycle(t(b)))
    ref = oracle.vcycle(L4, b, opt)
    log(f"4-level V-cycle fp64: {rel_inf(got, ref):.2e}")
    assert rel_inf(got, ref) < 1e-12
    # five outer iterations: the GPU history against the oracle's
    Sm = solver_for(sh, a, precision="mixed", levels=4, max_iters=5)
    _, st = Sm.solve(t(b), tol=1e-14)
    _, sref = oracle.solve(L4, b, opt, fixed_iters=5)
    h = np.array(st.res_hist[:6])
    href = sref["res_hist"]
    log(f"4-level history gpu {' '.join(f'{v:.3e}' for v in h)}")
    log(f"4-level history ora {' '.join(f'{v:.3e}' for v in href)}")
    np.testing.assert_allclose(h, href, rtol=1e-3)
    # against the automatic hierarchy: much slower contraction on this shell
    _, sauto = oracle.solve(levels_of(sh), b, opt, fixed_iters=5)
    rho4 = oracle.convergence_factors(href)[-1]
    rho = oracle.convergence_factors(sauto["res_hist"])[-1]
    log(f"convergence factor: 4 levels {rho4:.3f}, automatic ({len(levels_of(sh))}) {rho:.3f}")
    assert rho4 > 3 * rho
