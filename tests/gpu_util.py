"""Helpers shared by the GPU parity tests: seeded inputs, oracle results
(computed on the host, cached per process) and tensor conversion."""
from __future__ import annotations

import functools
import sys

import numpy as np

import shellgen
import oracle

DEV = "cuda:0"


def log(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(DEV)


def n(x):
    return x.detach().cpu().numpy()


def solver_for(sh, alpha, **opts):
    """A handle for shell sh, with the workload's smoothing interval unless
    opts give another."""
    from paper_2307_04528_amd import Solver
    opts.setdefault("smooth_interval", sh.smooth)
    log(f"[gpu] setup {sh.nlon}x{sh.nlat}x{sh.nlev} opts={opts}")
    return Solver.from_shell(sh, t(alpha), **opts)


@functools.lru_cache(maxsize=8)
def hierarchy(sh, levels=0):
    return oracle.build_hierarchy(sh, shellgen.alpha(sh), levels=levels)


def opts_of(sh, **kw):
    o = oracle.Options(nu_pre=sh.nu_pre, nu_post=sh.nu_post, smooth_lo=sh.smooth[0],
                       smooth_hi=sh.smooth[1])
    for k, v in kw.items():
        setattr(o, k, v)
    return o


@functools.lru_cache(maxsize=8)
def oracle_solution(sh, tol=1e-12):
    L = hierarchy(sh)
    u, st = oracle.solve(L, shellgen.rhs(sh), opts_of(sh), tol=tol)
    return u, st


def rel_inf(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def rel2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300))
