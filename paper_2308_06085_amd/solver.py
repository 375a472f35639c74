"""Python surface of the gfx950 Helmholtz solver (thin layer over the C ABI).

PyTorch supplies device memory and the stream; every arithmetic step runs in
the HIP kernels of ``libhh.so``.

* :class:`Solver` - one context: set the model k(x), set sources, solve,
  apply the operator / the shifted operator / one V-cycle.
* :class:`HelmholtzSolve` - ``torch.autograd.Function`` mapping squared
  slowness s (k = omega sqrt(s)) and right-hand sides b to the solutions u,
  with a backward pass made of one adjoint solve with the same
  preconditioned solver plus a pointwise product (``hh_adjoint_rhs`` and
  ``hh_grad_slowness2``).
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import torch

from . import _lib
from ._lib import BC, PREC, Config, Stats, check


def _ptr(t: torch.Tensor) -> int:
    return t.data_ptr()


def _require(t: torch.Tensor, dtype, shape, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


@dataclass
class SolveStats:
    iterations: float
    matvecs: int
    relres: float
    relres_true: float
    status: str
    restarts: int
    ms: float = 0.0  # device time of the whole solve call


class Solver:
    """One solver context for an (nz, ny, nx) grid.

    bc: "sommerfeld" | "dirichlet"; prec: "fp64" | "mixed" (complex64 V-cycle
    inside a complex128 Bi-CGSTAB); beta = (beta1, beta2) of the CSLP
    M = -Laplace - (beta1 - beta2 i) k^2 (default (1, -0.5)); omega: Jacobi
    weight (0.8); n_levels: 0 = coarsen while >= 3 nodes per axis remain;
    cycle: "V" | "F", the multigrid cycle that approximates M^-1 (section 3.4.5);
    method: "bicgstab" | "idrs" (IDR(s) with s = idr_s, section 3.1) | "gmres" (full
    GMRES on the left-preconditioned system, restarted after gmres_m steps).
    """

    def __init__(self, shape, h, bc="sommerfeld", prec="fp64", n_levels=0, nrhs_max=1,
                 beta=(1.0, -0.5), omega=0.8, cycle="V", method="bicgstab", idr_s=4, gmres_m=200, device=None):
        self.lib = _lib.load()
        nz, ny, nx = (int(v) for v in shape)
        self.shape = (nz, ny, nx)
        self.h = float(h)
        self.bc = bc
        self.prec = prec
        self.nrhs_max = int(nrhs_max)
        self.device = torch.device("cuda") if device is None else torch.device(device)
        cfg = Config()
        self.lib.hh_default_config(C.byref(cfg), nx, ny, nz, self.h)
        cfg.bc = BC[bc]
        cfg.prec = PREC[prec]
        cfg.n_levels = int(n_levels)
        cfg.nrhs_max = self.nrhs_max
        cfg.beta1, cfg.beta2 = float(beta[0]), float(beta[1])
        cfg.omega = float(omega)
        with torch.cuda.device(self.device):
            self.stream = torch.cuda.current_stream(self.device)
            ctx = C.c_void_p()
            check(self.lib.hh_create(C.byref(cfg), C.c_void_p(self.stream.cuda_stream), C.byref(ctx)))
        self.ctx = ctx
        self.nrhs = 0
        self._k = None
        self.model_version = 0  # counts set_model calls (HelmholtzSolve reuses a model it set)
        if cycle not in ("V", "F"):
            self.close()
            raise ValueError(f"cycle must be 'V' or 'F', not {cycle!r}")
        self.cycle = cycle
        if cycle == "F":
            self.set_option("cycle", 1)
        if method not in ("bicgstab", "idrs", "gmres"):
            self.close()
            raise ValueError(f"method must be 'bicgstab', 'idrs' or 'gmres', not {method!r}")
        self.method = method
        if method == "idrs":
            self.set_option("idr_s", int(idr_s))
            self.set_option("method", 1)
        elif method == "gmres":
            self.set_option("gmres_m", int(gmres_m))
            self.set_option("method", 2)

    # -- lifetime -----------------------------------------------------------
    def close(self):
        if getattr(self, "ctx", None):
            self.lib.hh_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- info ---------------------------------------------------------------
    def level_shapes(self):
        nx, ny, nz, nl = C.c_int(), C.c_int(), C.c_int(), C.c_int()
        check(self.lib.hh_level_shape(self.ctx, 0, C.byref(nx), C.byref(ny), C.byref(nz), C.byref(nl)),
              self.ctx)
        out = []
        for l in range(nl.value):
            check(self.lib.hh_level_shape(self.ctx, l, C.byref(nx), C.byref(ny), C.byref(nz), None),
                  self.ctx)
            out.append((nz.value, ny.value, nx.value))
        return out

    def set_option(self, name: str, value: int):
        check(self.lib.hh_set_option(self.ctx, name.encode(), int(value)), self.ctx)

    def get_option(self, name: str) -> int:
        v = C.c_longlong()
        check(self.lib.hh_get_option(self.ctx, name.encode(), C.byref(v)), self.ctx)
        return v.value

    # -- model and sources --------------------------------------------------
    def set_model(self, k: torch.Tensor):
        """Real wavenumber k(x) >= 0, float64 (nz, ny, nx) on the device."""
        _require(k, torch.float64, self.shape, "k")
        check(self.lib.hh_set_model(self.ctx, _ptr(k)), self.ctx)
        self._k = k
        self.model_version += 1

    def set_model_slowness2(self, s: torch.Tensor, omega: float):
        """The model as squared slowness s = 1/c^2, float64 (nz, ny, nx) on the
        device, at angular frequency omega: the library forms k = omega sqrt(s)."""
        _require(s, torch.float64, self.shape, "s")
        check(self.lib.hh_set_model_slowness2(self.ctx, _ptr(s), float(omega)), self.ctx)
        self._k = None
        self.model_version += 1

    def set_sources(self, b: torch.Tensor):
        """Right-hand sides, complex128 (nrhs, nz, ny, nx) or (nz, ny, nx)."""
        if b.dim() == 3:
            b = b.unsqueeze(0)
        _require(b, torch.complex128, (b.shape[0],) + self.shape, "b")
        check(self.lib.hh_set_sources(self.ctx, _ptr(b), b.shape[0]), self.ctx)
        self.nrhs = b.shape[0]

    def set_point_sources(self, nodes):
        """Dirac sources 1/h^3 at nodes [(iz, iy, ix), ...] (one right-hand side each)."""
        flat = [int(v) for n in nodes for v in n]
        arr = (C.c_int * len(flat))(*flat)
        check(self.lib.hh_set_point_sources(self.ctx, arr, len(nodes)), self.ctx)
        self.nrhs = len(nodes)

    def set_shadow(self, P: torch.Tensor):
        """IDR(s) shadow vectors, complex128 (s, nz, ny, nx) on the device; stored
        rounded to complex64.  Sets idr_s = s."""
        _require(P, torch.complex128, (P.shape[0],) + self.shape, "P")
        check(self.lib.hh_set_shadow(self.ctx, _ptr(P), P.shape[0]), self.ctx)

    # -- solve / apply ------------------------------------------------------
    def solve(self, x0: torch.Tensor | None = None, rtol=1e-6, maxit=1000, raise_on_fail=False,
              out: torch.Tensor | None = None):
        """Returns (x, [SolveStats per right-hand side]); x is (nrhs, nz, ny, nx)."""
        shape = (self.nrhs,) + self.shape
        if out is None:
            out = torch.empty(shape, dtype=torch.complex128, device=self.device)
        _require(out, torch.complex128, shape, "out")
        use_x0 = 0
        if x0 is not None:
            x0 = x0.reshape(shape)
            _require(x0, torch.complex128, shape, "x0")
            if x0.data_ptr() != out.data_ptr():
                out.copy_(x0)
            use_x0 = 1
        st = (Stats * self.nrhs)()
        status = self.lib.hh_solve(self.ctx, _ptr(out), float(rtol), int(maxit), use_x0, st)
        allow = () if raise_on_fail else (4, 5, 6)
        check(status, self.ctx, allow=allow)
        stats = [SolveStats(s.iterations, s.matvecs, s.relres, s.relres_true,
                            _lib.STATUS_NAMES.get(s.status, str(s.status)), s.restarts, s.ms) for s in st]
        return out, stats

    def _apply(self, fn, x):
        if x.dim() == 3:
            x = x.unsqueeze(0)
        _require(x, torch.complex128, (x.shape[0],) + self.shape, "x")
        y = torch.empty_like(x)
        check(fn(self.ctx, _ptr(x), _ptr(y), x.shape[0]), self.ctx)
        return y

    def apply_operator(self, x):
        """y = A x (complex128)."""
        return self._apply(self.lib.hh_apply_operator, x)

    def apply_shifted(self, x):
        """y = M x, the CSLP operator on the finest grid (complex128)."""
        return self._apply(self.lib.hh_apply_shifted, x)

    def apply_vcycle(self, r):
        """z = one multigrid (1,1) cycle applied to r (approximates M^-1 r): the
        V-cycle, or the F-cycle when the solver was made with cycle="F"."""
        return self._apply(self.lib.hh_apply_vcycle, r)

    def adjoint_rhs(self, g):
        return self._apply(self.lib.hh_adjoint_rhs, g)

    def grad_slowness2(self, u, w, s, omega):
        if u.dim() == 3:
            u, w = u.unsqueeze(0), w.unsqueeze(0)
        _require(u, torch.complex128, (u.shape[0],) + self.shape, "u")
        _require(w, torch.complex128, (u.shape[0],) + self.shape, "w")
        _require(s, torch.float64, self.shape, "s")
        grad = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        check(self.lib.hh_grad_slowness2(self.ctx, _ptr(u), _ptr(w), _ptr(s), float(omega), _ptr(grad),
                                         u.shape[0]), self.ctx)
        return grad

    def time_kernel(self, which: int, nrhs: int = 1, reps: int = 20) -> float:
        ms = C.c_float()
        check(self.lib.hh_time_kernel(self.ctx, int(which), int(nrhs), int(reps), C.byref(ms)), self.ctx)
        return ms.value

    def kernel_times(self):
        """In-solve kernel timing of the solves since ``set_option("trace", 1)``:
        (average ms per launch, launches) per kernel id of ``time_kernel``, and
        at index 6 the event-bracket cost (an empty launch per step)."""
        ms = (C.c_double * 7)()
        n = (C.c_longlong * 7)()
        check(self.lib.hh_kernel_times(self.ctx, ms, n), self.ctx)
        return list(ms), list(n)

    def autotune(self, cache_path: str | None = None) -> dict:
        """Pick the launch shapes by timing the first steps of a solve of the
        current sources (``hh_autotune``); with ``cache_path`` a JSON cache file
        is read first and updated after measuring.  Returns the shapes in use."""
        path = None if cache_path is None else str(cache_path).encode()
        check(self.lib.hh_autotune(self.ctx, path), self.ctx)
        return self.launch_shapes()

    def launch_shapes(self) -> dict:
        """The launch shapes in use: flat-kernel lanes, operator-apply z-planes,
        and per multigrid level with fused passes the down / up z-planes and the
        down-pass region."""
        levels = self.get_option("tail_first")
        return {"block": self.get_option("block"), "zb": self.get_option("zb"),
                "zb_down": [self.get_option(f"zb_down:{l}") for l in range(levels)],
                "zb_up": [self.get_option(f"zb_up:{l}") for l in range(levels)],
                "dn_region": [self.get_option(f"dn_region:{l}") for l in range(levels)],
                "autotune_source": self.get_option("autotune_source")}


def apply_operator_noalloc(k: torch.Tensor, x: torch.Tensor, h: float, bc: str = "sommerfeld",
                           out: torch.Tensor | None = None) -> torch.Tensor:
    """y = A x with no solver context and no device allocation in the library
    (``hh_apply_operator_noalloc``): k float64 (nz, ny, nx), x complex128
    (nrhs, nz, ny, nx) or (nz, ny, nx), both on the device; ``out`` (same shape
    as x) is written if given, else allocated here by PyTorch.  Enqueued on the
    current stream."""
    lib = _lib.load()
    if x.dim() == 3:
        x = x.unsqueeze(0)
    nz, ny, nx = (int(v) for v in k.shape)
    _require(k, torch.float64, (nz, ny, nx), "k")
    _require(x, torch.complex128, (x.shape[0], nz, ny, nx), "x")
    y = torch.empty_like(x) if out is None else out
    _require(y, torch.complex128, tuple(x.shape), "out")
    cfg = Config()
    lib.hh_default_config(C.byref(cfg), nx, ny, nz, float(h))
    cfg.bc = BC[bc]
    stream = torch.cuda.current_stream(x.device)
    check(lib.hh_apply_operator_noalloc(C.byref(cfg), _ptr(k), _ptr(x), _ptr(y), x.shape[0],
                                        C.c_void_p(stream.cuda_stream)))
    return y


class HelmholtzSolve(torch.autograd.Function):
    """u = A(s)^-1 b with k = omega sqrt(s), s the squared slowness 1/c^2.

    forward(s, b, omega, solver, rtol): s float64 (nz, ny, nx), b complex128
    (nrhs, nz, ny, nx); returns u (nrhs, nz, ny, nx).
    backward: with grad_u = dL/du (PyTorch's conjugate-Wirtinger convention),
    one adjoint solve A w = D^-1 conj(grad_u) with the same solver, then
    dL/ds_j = -sum_r Re(D_j w_rj a'_j u_rj), a'_j = -omega^2 - i n_j omega / (h sqrt(s_j)).
    The right-hand sides b are treated as data (no gradient).
    """

    @staticmethod
    def forward(ctx, s, b, omega, solver: Solver, rtol=1e-10, maxit=2000):
        if isinstance(b, torch.Tensor) and b.requires_grad:
            raise NotImplementedError("HelmholtzSolve differentiates with respect to s only")
        s = s.detach().contiguous()
        solver.set_model_slowness2(s, float(omega))
        solver.set_sources(b.contiguous())
        u, stats = solver.solve(rtol=rtol, maxit=maxit, raise_on_fail=True)
        ctx.solver, ctx.omega, ctx.rtol, ctx.maxit = solver, float(omega), rtol, maxit
        ctx.model_version = solver.model_version
        ctx.save_for_backward(s, u)
        return u

    @staticmethod
    def backward(ctx, grad_u):
        s, u = ctx.saved_tensors
        solver = ctx.solver
        # the model (hierarchy and coarsest inverse) of the forward solve is
        # still set unless the solver was given another one in between
        if solver.model_version != ctx.model_version:
            solver.set_model_slowness2(s, ctx.omega)
        rhs = solver.adjoint_rhs(grad_u.contiguous())
        solver.set_sources(rhs)
        w, _ = solver.solve(rtol=ctx.rtol, maxit=ctx.maxit, raise_on_fail=True)
        grad_s = solver.grad_slowness2(u, w, s, ctx.omega) if ctx.needs_input_grad[0] else None
        return grad_s, None, None, None, None, None
