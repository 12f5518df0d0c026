"""Python binding of the shell multigrid solver (same names as include/mg.h).

PyTorch provides the device memory (CUDA/HIP tensors) and the stream; every
step of the solve runs in the HIP library. Fields are float64 tensors of
shape (nlev, nlat, nlon), contiguous, on the GPU.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib as L


@dataclass
class SolveStats:
    iters: int
    relres: float
    res_hist: list
    ms_total: float
    levels: int
    alg_bytes: float
    kernels: dict
    ms_vcycle: float = 0.0
    ms_residual: float = 0.0
    fell_back_fp64: bool = False

    @staticmethod
    def from_c(st: L.mg_stats) -> "SolveStats":
        kernels = {}
        for c, name in enumerate(L.KERNEL_CLASSES):
            kernels[name] = dict(ms=st.kern_ms[c], launches=int(st.kern_launches[c]),
                                 bytes=st.kern_bytes[c], fine_ms=st.kern_fine_ms[c],
                                 fine_launches=int(st.kern_fine_launches[c]),
                                 fine_bytes=st.kern_fine_bytes[c])
        return SolveStats(int(st.iters), float(st.relres),
                          [float(st.res_hist[m]) for m in range(st.iters + 1)],
                          float(st.ms_total), int(st.levels_used), float(st.alg_bytes),
                          kernels, float(st.ms_vcycle), float(st.ms_residual),
                          bool(st.fell_back_fp64))


def _grid(nlon, nlat, nlev, radius, thickness, stretch, K) -> L.mg_grid:
    return L.mg_grid(int(nlon), int(nlat), int(nlev), float(radius), float(thickness),
                     float(stretch), float(K))


def _options(levels=0, nu_pre=2, nu_post=2, coarse_sweeps=40, max_iters=100, omega=0.8,
             semi_threshold=2.0, precision="mixed", profile=False, stream=None,
             smooth_interval=(1.0 / 3.0, 2.0), staged_columns=65536, stall_factor=0.9,
             stall_iters=3, graphs=True, zero_guess=False, poison=False) -> L.mg_options:
    """smooth_interval: (lo, hi), per-sweep omegas from the Chebyshev nodes of
    [lo, hi] (the default, see mg.h), or None: every smoothing sweep uses
    omega. staged_columns: levels with fewer columns sweep with the staged
    kernel (0: never). stall_factor, stall_iters: the mixed solve's switch
    to FP64 cycles when it stops contracting (see mg.h). graphs: replay the
    V-cycle below the finest level as a captured HIP graph. zero_guess: solves
    start from u = 0 without reading u (Solver.solve sets it per call).
    poison: fill the library's floating-point arrays with NaN when allocated
    (a debugging check)."""
    o = L.mg_options()
    L.lib().mg_options_default(C.byref(o))
    o.levels = int(levels)
    o.nu_pre, o.nu_post = int(nu_pre), int(nu_post)
    o.coarse_sweeps, o.max_iters = int(coarse_sweeps), int(max_iters)
    o.omega, o.semi_threshold = float(omega), float(semi_threshold)
    o.precision = {"mixed": L.MG_PREC_MIXED, "fp64": L.MG_PREC_FP64,
                   "fp32": L.MG_PREC_FP32}[precision]
    o.stream = stream
    o.profile = int(profile)
    if smooth_interval is None:
        o.smooth_lo = o.smooth_hi = 0.0
    else:
        o.smooth_lo, o.smooth_hi = float(smooth_interval[0]), float(smooth_interval[1])
    o.staged_columns = int(staged_columns)
    o.stall_factor, o.stall_iters = float(stall_factor), int(stall_iters)
    o.graphs = int(graphs)
    o.zero_guess = int(bool(zero_guess))
    o.poison = int(bool(poison))
    return o


def mg_plan(nlon, nlat, nlev, radius=1.0, thickness=0.01, stretch=1.05, K=1.0, **opts):
    """Host-only: level sizes and coarsening maps (no GPU needed)."""
    g = _grid(nlon, nlat, nlev, radius, thickness, stretch, K)
    o = _options(**opts)
    nlev_ = C.c_int32()
    nlon_out = (C.c_int32 * L.MG_MAX_LEVELS)()
    nlat_out = (C.c_int32 * L.MG_MAX_LEVELS)()
    cap = 4 * int(nlat) + 64
    cf = (C.c_int32 * cap)()
    cc = (C.c_int32 * cap)()
    L.check(L.lib().mg_plan(C.byref(g), C.byref(o), C.byref(nlev_), nlon_out, nlat_out,
                            cf, cc, cap), what="mg_plan")
    n = nlev_.value
    sizes = [(nlon_out[l], nlat_out[l]) for l in range(n)]
    maps, pos = [], 0
    for l in range(1, n):
        nJ = sizes[l][1]
        maps.append((list(cf[pos:pos + nJ]), list(cc[pos:pos + nJ])))
        pos += nJ
    return {"levels": n, "sizes": sizes, "child_first": [m[0] for m in maps],
            "child_count": [m[1] for m in maps]}


def mg_plan_tables(level, nlon, nlat, nlev, radius=1.0, thickness=0.01, stretch=1.05, K=1.0,
                   **opts):
    """Host-only: FP64 tables (V, Tlam, Tth, Tr) of one level, as numpy arrays."""
    import numpy as np
    plan = mg_plan(nlon, nlat, nlev, radius, thickness, stretch, K, **opts)
    nJ = plan["sizes"][level][1]
    nz = int(nlev)
    V = np.zeros(nz * nJ)
    Tl = np.zeros(nz * nJ)
    Tt = np.zeros(nz * (nJ + 1))
    Tr = np.zeros((nz + 1) * nJ)
    p = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
    g = _grid(nlon, nlat, nlev, radius, thickness, stretch, K)
    o = _options(**opts)
    L.check(L.lib().mg_plan_tables(C.byref(g), C.byref(o), int(level), p(V), p(Tl), p(Tt),
                                   p(Tr)), what="mg_plan_tables")
    return (V.reshape(nz, nJ), Tl.reshape(nz, nJ), Tt.reshape(nz, nJ + 1),
            Tr.reshape(nz + 1, nJ))


class Solver:
    """A multigrid hierarchy for one shell and one alpha field (mg_setup)."""

    def __init__(self, nlon, nlat, nlev, alpha: torch.Tensor, radius=1.0, thickness=0.01,
                 stretch=1.05, K=1.0, **opts):
        self.shape = (int(nlev), int(nlat), int(nlon))
        self.device = alpha.device
        self._check(alpha, "alpha")
        self._opts = dict(opts)
        self._grid = _grid(nlon, nlat, nlev, radius, thickness, stretch, K)
        self._stream = self._current_stream()
        o = _options(stream=self._stream, **self._opts)
        h = C.c_void_p()
        co = L.mg_coeffs(alpha.data_ptr())
        L.check(L.lib().mg_setup(C.byref(self._grid), C.byref(co), C.byref(o), C.byref(h)),
                what="mg_setup")
        self._h = h
        self._set_alpha(alpha)

    @classmethod
    def from_shell(cls, shell, alpha: torch.Tensor, **opts):
        return cls(shell.nlon, shell.nlat, shell.nlev, alpha, radius=shell.radius,
                   thickness=shell.thickness, stretch=shell.stretch, K=shell.K, **opts)

    # -- helpers ---------------------------------------------------------------
    def _current_stream(self):
        return C.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)

    def _sync_options(self):
        s = self._current_stream()
        if s.value != self._stream.value:
            self._stream = s
            self.set_options(**self._opts)

    def _check(self, t: torch.Tensor, name: str, shape=None):
        shape = shape or self.shape
        if not isinstance(t, torch.Tensor):
            raise TypeError(f"{name} must be a torch.Tensor")
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise ValueError(f"{name} must be a contiguous float64 GPU tensor")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")

    def _empty(self, shape=None):
        return torch.empty(shape or self.shape, dtype=torch.float64, device=self.device)

    @property
    def handle(self):
        return self._h

    def close(self):
        if getattr(self, "_h", None):
            L.lib().mg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- API -----------------------------------------------------------------
    def option(self, name: str):
        """The value of one mg_options field in effect for this solver."""
        return getattr(_options(stream=self._stream, **self._opts), name)

    def _zero_guess(self, zero: bool):
        if bool(self._opts.get("zero_guess", False)) != zero:
            self.set_options(zero_guess=zero)

    def set_options(self, **opts):
        self._opts.update(opts)
        o = _options(stream=self._stream, **self._opts)
        L.check(L.lib().mg_set_options(self._h, C.byref(o)), self._h, "mg_set_options")

    def _set_alpha(self, alpha: torch.Tensor):
        # the tensor whose values the handle holds, and its memory and version
        # counter at upload: an in-place change bumps the version (the
        # reference kept here also keeps the memory from being reused)
        self.alpha = alpha
        self._alpha_key = (alpha.data_ptr(), alpha._version)

    def alpha_is_current(self, alpha: torch.Tensor) -> bool:
        """True if alpha is the tensor last uploaded, unchanged since."""
        return (alpha.data_ptr(), alpha._version) == self._alpha_key and \
            alpha.shape == self.alpha.shape

    def update_alpha(self, alpha: torch.Tensor):
        self._check(alpha, "alpha")
        self._sync_options()
        co = L.mg_coeffs(alpha.data_ptr())
        L.check(L.lib().mg_update_coeffs(self._h, C.byref(co)), self._h, "mg_update_coeffs")
        self._set_alpha(alpha)

    def solve(self, rhs: torch.Tensor, tol: float = 1e-8, u0: torch.Tensor | None = None,
              out: torch.Tensor | None = None):
        """Solve H u = rhs; returns (u, SolveStats). u0 is the initial guess
        (zero if None); out, if given, receives the solution."""
        self._check(rhs, "rhs")
        self._sync_options()
        u = out if out is not None else self._empty()
        self._check(u, "out")
        # from zero: the library neither reads u nor forms H u for it
        self._zero_guess(u0 is None)
        if u0 is not None and u0.data_ptr() != u.data_ptr():
            self._check(u0, "u0")
            u.copy_(u0)
        st = L.mg_stats()
        s = L.lib().mg_solve(self._h, rhs.data_ptr(), u.data_ptr(), float(tol), C.byref(st))
        L.check(s, self._h, "mg_solve")
        stats = SolveStats.from_c(st)
        stats.status = s
        return u, stats

    def solve_adjoint(self, w: torch.Tensor, tol: float = 1e-8):
        """lambda = H^{-T} w with the transposed V-cycle; returns (lambda, stats)."""
        self._check(w, "w")
        self._sync_options()
        self._zero_guess(True)
        lam = torch.empty_like(w)
        st = L.mg_stats()
        s = L.lib().mg_solve_adjoint(self._h, w.data_ptr(), lam.data_ptr(), float(tol),
                                     C.byref(st))
        L.check(s, self._h, "mg_solve_adjoint")
        stats = SolveStats.from_c(st)
        stats.status = s
        return lam, stats

    def grad_alpha(self, lam: torch.Tensor, u: torch.Tensor):
        self._check(lam, "lambda")
        self._check(u, "u")
        self._sync_options()
        g = self._empty()
        L.check(L.lib().mg_grad_alpha(self._h, lam.data_ptr(), u.data_ptr(), g.data_ptr()),
                self._h, "mg_grad_alpha")
        return g

    def apply(self, x: torch.Tensor):
        self._check(x, "x")
        self._sync_options()
        y = self._empty()
        L.check(L.lib().mg_apply(self._h, x.data_ptr(), y.data_ptr()), self._h, "mg_apply")
        return y

    def cell_volumes(self):
        self._sync_options()
        V = self._empty()
        L.check(L.lib().mg_cell_volumes(self._h, V.data_ptr()), self._h, "mg_cell_volumes")
        return V

    def vcycle(self, f: torch.Tensor, transposed: bool = False):
        self._check(f, "f")
        self._sync_options()
        x = self._empty()
        L.check(L.lib().mg_vcycle(self._h, f.data_ptr(), x.data_ptr(), 1 if transposed else 0),
                self._h, "mg_vcycle")
        return x

    def level_shape(self, l: int):
        s = (C.c_int32 * 3)()
        L.check(L.lib().mg_level_shape(self._h, int(l), s), self._h, "mg_level_shape")
        return (s[2], s[1], s[0])

    def level_sweep(self, l: int, f: torch.Tensor, x_in: torch.Tensor | None = None):
        shp = self.level_shape(l)
        self._check(f, "f", shp)
        if x_in is not None:
            self._check(x_in, "x_in", shp)
        self._sync_options()
        out = self._empty(shp)
        L.check(L.lib().mg_level_sweep(self._h, int(l), f.data_ptr(),
                                       None if x_in is None else x_in.data_ptr(),
                                       out.data_ptr()), self._h, "mg_level_sweep")
        return out

    def level_residual_restrict(self, l: int, f: torch.Tensor, x: torch.Tensor | None):
        shp = self.level_shape(l)
        self._check(f, "f", shp)
        if x is not None:
            self._check(x, "x", shp)
        self._sync_options()
        fc = self._empty(self.level_shape(l + 1))
        L.check(L.lib().mg_level_residual_restrict(self._h, int(l), f.data_ptr(),
                                                   None if x is None else x.data_ptr(),
                                                   fc.data_ptr()),
                self._h, "mg_level_residual_restrict")
        return fc

    def level_prolong_add(self, l: int, xc: torch.Tensor, x: torch.Tensor):
        self._check(xc, "xc", self.level_shape(l + 1))
        self._check(x, "x", self.level_shape(l))
        self._sync_options()
        out = x.clone()
        L.check(L.lib().mg_level_prolong_add(self._h, int(l), xc.data_ptr(), out.data_ptr()),
                self._h, "mg_level_prolong_add")
        return out
