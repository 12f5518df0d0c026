"""The adjoint workload at its full size: shell384x192x70 with L = <w, u>,
u = H(alpha)^{-1} b, w ~ N(0, 1).

  * dL/db and dL/dalpha from torch.autograd through the library's solve and
    hand-written transposed V-cycle (mixed precision, the product path)
    against the oracle's adjoint (lambda = H^{-T} w by its own transposed
    cycle, dL/dalpha = -lambda V u): 1e-8 relative;
  * the same gradients against FP64 central finite differences with step
    h = 1e-6 (relative for alpha, absolute for b) along 32 seeded random
    directions: 1e-6 relative each.

The central difference quotient along alpha, (L(alpha+) - L(alpha-)) / 2h with
alpha+- = alpha (1 +- h d), is evaluated without cancellation: since
H(alpha+) - H(alpha-) = 2h D with D = diag(alpha d V),
    L(alpha+) - L(alpha-) = <w, u+ - u->,  H(alpha+) (u+ - u-) = -2h D u-,
so the quotient is -<w, H(alpha+)^{-1} D u-> exactly, from two forward FP64
solves and no adjoint. Subtracting the two values of L instead loses the
quotient to rounding: L changes in its ninth digit, while an FP64 solve
leaves L accurate to about 1e-15 relative, and the plain quotient is off
by up to ~1e-5 (measured); it is computed too, and checked only to 1e-4.
"""
import numpy as np
import pytest

import shellgen
import oracle
from gpu_util import log, t, n, solver_for, rel2, opts_of

pytestmark = pytest.mark.gpu

SH = shellgen.workload("shell384x192x70")


def test_adjoint_workload_gradients():
    import torch
    from paper_2307_04528_amd import mg_solve
    sh = SH
    a, b, w = shellgen.alpha(sh), shellgen.rhs(sh), shellgen.weights(sh)

    S = solver_for(sh, a, precision="mixed")
    at = t(a).requires_grad_(True)
    bt = t(b).requires_grad_(True)
    u = mg_solve(bt, at, S, 1e-12)
    (t(w) * u).sum().backward()
    ga, gb = n(at.grad), n(bt.grad)
    S.close()

    log("[oracle] forward and adjoint solves of shell384x192x70")
    L = oracle.build_hierarchy(sh, a)
    opt = opts_of(sh)
    u_ref, _ = oracle.solve(L, b, opt, tol=1e-12)
    lam_ref, _ = oracle.solve_adjoint(L, w, opt, tol=1e-12)
    g_ref = oracle.grad_alpha(L, lam_ref, u_ref)
    log(f"  dL/db vs oracle {rel2(gb, lam_ref):.2e}, dL/dalpha vs oracle {rel2(ga, g_ref):.2e}")
    assert rel2(gb, lam_ref) < 1e-8
    assert rel2(ga, g_ref) < 1e-8

    S2 = solver_for(sh, a, precision="fp64", max_iters=60)
    V = n(S2.cell_volumes())

    def solve(alpha, rhs):
        S2.update_alpha(t(alpha))
        uu, _ = S2.solve(t(rhs), tol=1e-14)
        return n(uu)

    h = 1e-6
    worst = [0.0, 0.0, 0.0]
    for m in range(32):
        d = shellgen.fd_direction(sh, m)
        fd_b = (np.vdot(w, solve(a, b + h * d)) - np.vdot(w, solve(a, b - h * d))) / (2 * h)
        ap, am = a * (1 + h * d), a * (1 - h * d)
        um = solve(am, b)
        up = solve(ap, b)
        fd_a_plain = (np.vdot(w, up) - np.vdot(w, um)) / (2 * h)
        diff = solve(ap, -2 * h * (a * d * V) * um)        # u+ - u-
        fd_a = np.vdot(w, diff) / (2 * h)
        an_b, an_a = float(np.vdot(gb, d)), float(np.vdot(ga, a * d))
        e = [abs(fd_b - an_b) / abs(an_b), abs(fd_a - an_a) / abs(an_a),
             abs(fd_a_plain - an_a) / abs(an_a)]
        worst = [max(x, y) for x, y in zip(worst, e)]
        log(f"  direction {m}: b {e[0]:.1e}, alpha {e[1]:.1e} (subtracting L: {e[2]:.1e})")
        assert e[0] < 1e-6 and e[1] < 1e-6 and e[2] < 1e-4
    log(f"  worst over 32 directions: b {worst[0]:.1e}, alpha {worst[1]:.1e} "
        f"(subtracting L: {worst[2]:.1e})")
    S2.close()
