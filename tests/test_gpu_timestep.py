"""GPU test of the time-step workload: a sequence of solves with slowly
varying alpha and b (shellgen.timestep), each after mg_update_coeffs and
warm-started from the previous step's solution.

Per step, on the 384x192x70 shell:
  * the oracle builds the hierarchy of alpha_t on the host and recomputes
    ||b_t - H_t u_t|| / ||b_t||, which must be below the tolerance;
  * a handle set up from scratch with alpha_t, started from the same
    initial guess, returns the same iteration count and a bit-identical
    solution: the update path leaves nothing of the old coefficients behind
    (masses, pivots, the coarsest matrix);
  * the warm start needs fewer iterations than a start from zero.
"""
import numpy as np
import pytest

import shellgen
import oracle
from gpu_util import log, t, n, solver_for

pytestmark = pytest.mark.gpu

MEDIUM = shellgen.workload("shell384x192x70")


def test_timestep_sequence_warm_started_after_coefficient_updates():
    sh = MEDIUM
    tol = 1e-8
    S = solver_for(sh, shellgen.alpha(sh))
    u, st = S.solve(t(shellgen.rhs(sh)), tol=tol)
    cold0 = st.iters
    for step in range(1, 4):
        a_np, b_np = shellgen.timestep(sh, step)
        a_t, b_t = t(a_np), t(b_np)
        u_prev = u.clone()
        S.update_alpha(a_t)
        u, st = S.solve(b_t, tol=tol, u0=u_prev)
        # the same step on a fresh handle
        F = solver_for(sh, a_np)
        uf, stf = F.solve(b_t, tol=tol, u0=u_prev)
        _, stc = F.solve(b_t, tol=tol)
        L = oracle.build_hierarchy(sh, a_np)
        host = np.linalg.norm((b_np - oracle.apply(L[0], n(u))).ravel()) / np.linalg.norm(b_np)
        log(f"step {step}: warm iters {st.iters} (fresh handle {stf.iters}, cold {stc.iters}, "
            f"first step cold {cold0}), relres {st.relres:.2e}, oracle {host:.2e}")
        assert st.status == 0
        assert host <= tol * 1.01
        assert st.iters == stf.iters
        assert np.array_equal(n(u), n(uf))
        assert st.iters < stc.iters
        F.close()
    S.close()
