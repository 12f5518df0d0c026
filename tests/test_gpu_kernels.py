"""GPU parity of the individual HIP kernels against the oracle, element by
element, in FP64 and FP32, on every level of several hierarchies (ragged
widths, tiny grids, the small 64x32x16 shell and a reduced 70-layer shell).

Tolerances (relative to the largest output value):
  * FP64: 1e-12 (both sides evaluate the same sums in a different order;
    the column solves use the cancellation-free row-sum pivots).
  * FP32: 2e-5 for one kernel: single rounding of each term (eps32 = 6e-8)
    through at most ~70 dependent Thomas steps, each a convex combination.
"""
import numpy as np
import pytest

import shellgen
import oracle
from gpu_util import log, t, n, solver_for, rel_inf

pytestmark = pytest.mark.gpu

SHELLS = [
    shellgen.Shell("tiny", 4, 2, 1, stretch=1.0),
    shellgen.Shell("small", 8, 4, 3, stretch=1.1),
    shellgen.Shell("ragged", 100, 50, 7, stretch=1.2, thickness=0.05),
    shellgen.workload("shell64x32x16"),
    shellgen.Shell("deep", 96, 48, 70, stretch=1.05),
    shellgen.Shell("nz128", 36, 18, 128, stretch=1.02),
]
IDS = [f"{s.nlon}x{s.nlat}x{s.nlev}" for s in SHELLS]
TOL = {"fp64": 1e-12, "mixed": 2e-5}


@pytest.mark.parametrize("sh", SHELLS, ids=IDS)
def test_apply_fp64(sh):
    a = shellgen.alpha(sh)
    S = solver_for(sh, a)
    L = oracle.build_hierarchy(sh, a)
    x = np.random.default_rng(11).standard_normal(sh.shape)
    y = n(S.apply(t(x)))
    ref = oracle.apply(L[0], x)
    log(f"apply {sh.name}: rel {rel_inf(y, ref):.2e}")
    assert rel_inf(y, ref) < 1e-13
    V = n(S.cell_volumes())
    np.testing.assert_allclose(V, np.broadcast_to(L[0].V[:, :, None], sh.shape), rtol=1e-11)


# staged: every level's sweeps with the staged kernel (a segment's loads
# staged in LDS by eight wavefronts, its columns solved from there), or none
# (a wavefront pair per segment, straight from memory).
@pytest.mark.parametrize("staged", [True, False], ids=["staged", "pairs"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("sh", SHELLS, ids=IDS)
def test_level_kernels(sh, prec, staged):
    a = shellgen.alpha(sh)
    S = solver_for(sh, a, precision=prec, staged_columns=(1 << 30) if staged else 0)
    L = oracle.build_hierarchy(sh, a)
    rng = np.random.default_rng(12)
    tol = TOL[prec]
    om = 0.8
    for l, lev in enumerate(L):
        assert S.level_shape(l) == lev.shape
        f = rng.standard_normal(lev.shape)
        x = rng.standard_normal(lev.shape)
        # sweep from zero and a full sweep (Eq. 1)
        got0 = n(S.level_sweep(l, t(f)))
        ref0 = oracle.sweep_from_zero(lev, f, om)
        got1 = n(S.level_sweep(l, t(f), t(x)))
        ref1 = oracle.sweep(lev, x, f, om)
        log(f"{sh.name} {prec} l={l} sweep0 {rel_inf(got0, ref0):.2e} sweep {rel_inf(got1, ref1):.2e}")
        assert rel_inf(got0, ref0) < tol
        assert rel_inf(got1, ref1) < tol
        if l + 1 < len(L):
            c = L[l + 1]
            got = n(S.level_residual_restrict(l, t(f), t(x)))
            ref = oracle.restrict(lev, c, f - oracle.apply(lev, x))
            gotf = n(S.level_residual_restrict(l, t(f), None))
            reff = oracle.restrict(lev, c, f)
            # the residual cancels: scale by the restricted |f| + |Hx| terms
            scale = np.abs(oracle.restrict(lev, c, np.abs(f) + np.abs(oracle.apply(lev, x)))).max()
            log(f"  restrict {np.abs(got - ref).max() / scale:.2e} R f {rel_inf(gotf, reff):.2e}")
            assert np.abs(got - ref).max() / scale < tol
            assert rel_inf(gotf, reff) < tol
            xc = rng.standard_normal(c.shape)
            got = n(S.level_prolong_add(l, t(xc), t(x)))
            ref = x + oracle.prolong(lev, c, xc)
            log(f"  prolong {rel_inf(got, ref):.2e}")
            assert rel_inf(got, ref) < tol


# Larger levels (from 2^15 columns) restrict with the kernel that walks
# ranges of 10 layers (one wavefront per coarse segment and range): ragged
# coarse widths (550, 520 and 100 columns are not multiples of 64; their
# lanes load their longitude neighbours), widths of whole segments (512 and
# 128: the neighbours come from the neighbour lanes), and layer counts that
# are not a multiple of the range (16 and 37 layers).
LARGE = [shellgen.Shell("wide16", 1100, 480, 16, stretch=1.1),
         shellgen.Shell("wide37", 1040, 512, 37, stretch=1.05),
         shellgen.Shell("full16", 1024, 512, 16, stretch=1.1),
         shellgen.Shell("mid70", 256, 160, 70, stretch=1.05),
         shellgen.Shell("mid37", 200, 176, 37, stretch=1.05)]


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("sh", LARGE, ids=[f"{s.nlon}x{s.nlat}x{s.nlev}" for s in LARGE])
def test_large_level_restriction(sh, prec):
    a = shellgen.alpha(sh)
    S = solver_for(sh, a, precision=prec)
    L = oracle.build_hierarchy(sh, a)
    assert sh.nlon * sh.nlat >= 1 << 15
    rng = np.random.default_rng(13)
    f = rng.standard_normal(sh.shape)
    x = rng.standard_normal(sh.shape)
    got = n(S.level_residual_restrict(0, t(f), t(x)))
    Hx = oracle.apply(L[0], x)
    ref = oracle.restrict(L[0], L[1], f - Hx)
    scale = np.abs(oracle.restrict(L[0], L[1], np.abs(f) + np.abs(Hx))).max()
    err = np.abs(got - ref).max() / scale
    log(f"{sh.name} {prec}: restrict {err:.2e}")
    assert err < TOL[prec]
