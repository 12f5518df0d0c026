"""mg_solve_noalloc, the solve for callers that cannot allocate, against
mg_solve on the same handle: two calls in a row, the second on a smaller
grid (the library's scratch keeps the first call's contents), each result
bit-identical to mg_solve's, with the same iterations and residual, from a
zeroed u and, with zero_guess set, from a u that is never read."""
import ctypes as C

import numpy as np
import pytest
import torch

import shellgen
from gpu_util import log, t, solver_for

from paper_2307_04528_amd import _lib as L

pytestmark = pytest.mark.gpu


def _noalloc(S, b, tol, fill=0.0):
    u = torch.full_like(b, fill)
    st = L.mg_stats()
    s = L.lib().mg_solve_noalloc(S.handle, b.data_ptr(), u.data_ptr(), float(tol), C.byref(st))
    L.check(s, S.handle, "mg_solve_noalloc")
    torch.cuda.synchronize()
    return u, st


@pytest.mark.parametrize("prec", ["mixed", "fp64"])
def test_noalloc_matches_solve_twice(prec):
    big = shellgen.workload("shell384x192x70")
    small = shellgen.workload("shell64x32x16")
    for sh in (big, small):
        S = solver_for(sh, shellgen.alpha(sh), precision=prec, nu_pre=sh.nu_pre,
                       nu_post=sh.nu_post)
        b = t(shellgen.rhs(sh))
        tol = 1e-9
        u_na, st_na = _noalloc(S, b, tol)
        u_ref, st_ref = S.solve(b, tol=tol)
        torch.cuda.synchronize()
        log(f"noalloc {sh.name} {prec}: iters {st_na.iters}/{st_ref.iters} relres "
            f"{st_na.relres:.3e}/{st_ref.relres:.3e}")
        assert st_na.iters == st_ref.iters
        assert st_na.relres == st_ref.relres
        assert st_na.relres <= tol
        assert torch.equal(u_na, u_ref)
        assert st_na.ms_vcycle == 0 and st_na.kern_launches[1] == 0
        # S.solve left zero_guess set: the no-alloc solve then reads no
        # initial guess either (u starts as NaN here)
        assert S.option("zero_guess") == 1
        u_z, st_z = _noalloc(S, b, tol, fill=float("nan"))
        assert st_z.iters == st_ref.iters and st_z.relres == st_ref.relres
        assert torch.equal(u_z, u_ref)
        S.close()


def test_noalloc_rejects_null_and_bad_tol():
    sh = shellgen.workload("shell64x32x16")
    S = solver_for(sh, shellgen.alpha(sh), nu_pre=1, nu_post=1)
    b = t(shellgen.rhs(sh))
    u = torch.zeros_like(b)
    st = L.mg_stats()
    assert L.lib().mg_solve_noalloc(S.handle, None, u.data_ptr(), 1e-8,
                                    C.byref(st)) == L.MG_ERR_ARG
    assert L.lib().mg_solve_noalloc(S.handle, b.data_ptr(), u.data_ptr(), 0.0,
                                    C.byref(st)) == L.MG_ERR_ARG
