"""MI355X-native solver for the implicit-Euler time-periodic nonlinear eddy-current problem.

Python binding of the C ABI in include/ptsolve.h. Every step of the solver runs in
the HIP kernels of libptsolve.so; this module only marshals arguments: it builds
the problem/option structs, allocates device buffers with torch, and passes raw
pointers and torch's current HIP stream. There is no CPU fallback: importing the
package works without a GPU (plan creation is host-only), but every compute call
needs the built library and a GPU.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Dict, List, Optional

from . import _lib as L

__all__ = ["Plan", "BatchPlan", "SolveStats", "PTError", "library", "problem_struct"]


class PTError(RuntimeError):
    def __init__(self, status: int, where: str):
        lib = L.load()
        self.status = status
        msg = lib.pt_last_error().decode()
        name = lib.pt_status_string(status).decode()
        super().__init__(f"{where}: {name} ({status}): {msg}")


def library():
    return L.load()


def _rect(r) -> L.Rect:
    x0, y0, x1, y1 = r.as_tuple() if hasattr(r, "as_tuple") else tuple(r)
    return L.Rect(x0, y0, x1, y1)


def problem_struct(p, theta=None, sigma=None, load=None, region=None) -> L.Problem:
    """Fill the C problem struct from any object with the fields of a problem description
    (n, N, T, sigma_in, sigma_rect, nu_a, nu_b, nu_out, nu_rect, J0, coil_rect, waveform,
    nu_max; region mode: law and regions, each with sigma, a, b, c, d, j). theta / sigma / load
    are optional device tensors (float64, contiguous); region is the device uint8 tensor of the
    triangles' regions, required in region mode. The struct keeps its regions array alive."""
    s = L.Problem()
    s.n, s.N, s.T = int(p.n), int(p.N), float(p.T)
    s.sigma_in, s.sigma_rect = float(p.sigma_in), _rect(p.sigma_rect)
    s.nu_a, s.nu_b, s.nu_out, s.nu_rect = float(p.nu_a), float(p.nu_b), float(p.nu_out), _rect(p.nu_rect)
    s.J0, s.coil_rect = float(p.J0), _rect(p.coil_rect)
    s.waveform = L.PT_WAVE_SIN if p.waveform == "sin" else L.PT_WAVE_COS
    s.nu_max = float(p.nu_max)
    s.d_theta = _ptr(theta, "theta", 2 * p.n * p.n)
    s.d_sigma = _ptr(sigma, "sigma", 2 * p.n * p.n)
    s.d_load = _ptr(load, "load", p.N * (p.n + 1) ** 2)
    regs = getattr(p, "regions", None)
    s.law = {"rational": L.PT_NU_RATIONAL, "expcap": L.PT_NU_EXPCAP}[getattr(p, "law", "rational")]
    if regs is not None:
        import torch
        if region is None or region.dtype != torch.uint8 or not region.is_cuda or not region.is_contiguous() or \
                region.numel() != 2 * p.n * p.n:
            raise ValueError(f"region mode needs a contiguous uint8 device tensor of {2 * p.n * p.n} region ids")
        arr = (L.Region * len(regs))(*[L.Region(r.sigma, r.a, r.b, r.c, r.d, r.j, r.nu_hat) for r in regs])
        s._regions = arr
        s.nregions = len(regs)
        s.d_region = region.data_ptr()
        s.regions = arr
    return s


def _ptr(t, name, numel):
    if t is None:
        return None
    import torch
    if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or t.numel() != numel:
        raise ValueError(f"{name} must be a contiguous float64 device tensor with {numel} entries")
    return t.data_ptr()


def device_reciprocals(x):
    """The kernels' two FP64 reciprocals of a contiguous float64 device tensor x: (the residual
    sweep's, one Newton step, for x >= 1; the V-cycle's, two Newton steps, for x > 0), each a
    tensor like x (pt_device_reciprocals). Synchronises the current stream."""
    import torch
    if x.dtype != torch.float64 or not x.is_cuda or not x.is_contiguous():
        raise ValueError("x must be a contiguous float64 device tensor")
    y = torch.empty(2 * x.numel(), dtype=torch.float64, device=x.device)
    lib = L.load()
    st = lib.pt_device_reciprocals(C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()), x.numel(),
                                   C.c_void_p(torch.cuda.current_stream().cuda_stream))
    if st != 0:
        raise PTError(st, "pt_device_reciprocals")
    torch.cuda.current_stream().synchronize()
    y = y.view(-1, 2)
    return y[:, 0].reshape(x.shape), y[:, 1].reshape(x.shape)


@dataclass
class SolveStats:
    status: int
    outer_iters: int
    rel_residual: float
    f_norm: float
    time_ms: float
    history: List[float]
    kernel_ms: Dict[str, float] = field(default_factory=dict)
    kernel_launches: Dict[str, int] = field(default_factory=dict)
    converged_at: int = -1
    init_iters: int = 0
    rel_initial: float = float("nan")
    krylov_iters: int = 0
    inner_iters_max: int = 0
    inner_iters_sum: int = 0


def _options(lib, tol, max_outer, check_every, precision, inner, inner_iters, vc_omega, use_initial_guess,
             diverge_factor, xcd_remap, timing, graph, grid_slot=0, grid_team=0, adjoint=False,
             init_static=False, init_tol=1e-8, stop_relative_initial=False, krylov_dim=0, forcing=1e-2,
             max_krylov=100, inner_rtol=0.0, breakdown_tol=0.0, cycle="default", grid_restrict=0, grid_up=0,
             grid_matvec=0) -> L.Options:
    o = L.Options()
    lib.pt_options_default(C.byref(o))
    o.tol, o.max_outer, o.check_every = float(tol), int(max_outer), int(check_every)
    o.precision = {"fp64": L.PT_FP64, "fp32": L.PT_FP32_REFINE}[precision]
    o.inner = {"galerkin1": L.PT_INNER_GALERKIN1, "cocg": L.PT_INNER_COCG}[inner]
    o.inner_iters, o.vc_omega = int(inner_iters), float(vc_omega)
    o.use_initial_guess = 1 if use_initial_guess else 0
    o.diverge_factor, o.xcd_remap = float(diverge_factor), 1 if xcd_remap else 0
    # timing: False, True (every kernel class) or a collection of class names to time alone
    if isinstance(timing, (list, tuple, set, frozenset)):
        names = {lib.pt_kernel_class_name(k).decode(): k for k in range(L.PT_KERNEL_CLASSES)}
        unknown = [c for c in timing if c not in names]
        if unknown or not timing:
            raise ValueError(f"timing: unknown or no kernel classes {unknown}")
        o.timing, o.timing_mask = 1, sum(1 << names[c] for c in set(timing))
    else:
        o.timing = 1 if timing else 0
    o.graph = 1 if graph else 0
    o.grid_slot, o.grid_team = int(grid_slot), int(grid_team)
    o.adjoint = 1 if adjoint else 0
    o.init_static = 1 if init_static else 0
    o.init_tol = float(init_tol)
    o.stop_relative_initial = 1 if stop_relative_initial else 0
    o.krylov_dim, o.forcing, o.max_krylov = int(krylov_dim), float(forcing), int(max_krylov)
    o.inner_rtol, o.breakdown_tol = float(inner_rtol), float(breakdown_tol)
    o.vc_cycle = {"default": L.PT_VC_DEFAULT, "v11": L.PT_VC_V11, "v01": L.PT_VC_V01}[cycle]
    o.grid_restrict, o.grid_up, o.grid_matvec = int(grid_restrict), int(grid_up), int(grid_matvec)
    return o


class _StatsBuf:
    """Host buffers behind one pt_stats struct."""

    def __init__(self, history_cap):
        self.hist = (C.c_double * history_cap)()
        self.kms = (C.c_double * L.PT_KERNEL_CLASSES)()
        self.kcnt = (C.c_int64 * L.PT_KERNEL_CLASSES)()
        self.cap = history_cap

    def fill(self, s: L.Stats):
        s.residual_history = C.cast(self.hist, C.POINTER(C.c_double))
        s.history_cap = self.cap
        s.kernel_ms = C.cast(self.kms, C.POINTER(C.c_double))
        s.kernel_launches = C.cast(self.kcnt, C.POINTER(C.c_int64))

    def result(self, lib, st, s: L.Stats) -> SolveStats:
        names = [lib.pt_kernel_class_name(i).decode() for i in range(L.PT_KERNEL_CLASSES)]
        n = L.PT_KERNEL_CLASSES
        return SolveStats(status=st, outer_iters=s.outer_iters, rel_residual=s.rel_residual, f_norm=s.f_norm,
                          time_ms=s.time_ms, history=list(self.hist[: s.history_len]),
                          kernel_ms={names[i]: self.kms[i] for i in range(n) if self.kcnt[i]},
                          kernel_launches={names[i]: int(self.kcnt[i]) for i in range(n) if self.kcnt[i]},
                          converged_at=s.converged_at, init_iters=s.init_iters, rel_initial=s.rel_initial,
                          krylov_iters=s.krylov_iters, inner_iters_max=s.inner_iters_max,
                          inner_iters_sum=s.inner_iters_sum)


class Plan:
    """A solver plan: validated problem + options, workspace and entry points."""

    def __init__(self, problem, *, tol=1e-8, max_outer=1000, check_every=1, precision="fp64",
                 inner="galerkin1", inner_iters=1, vc_omega=0.8, use_initial_guess=False,
                 diverge_factor=1e3, xcd_remap=True, timing=False, graph=False, grid_slot=0, grid_team=0,
                 adjoint=False, init_static=False, init_tol=1e-8, stop_relative_initial=False, krylov_dim=0,
                 forcing=1e-2, max_krylov=100, inner_rtol=0.0, breakdown_tol=0.0, cycle="default", grid_restrict=0,
                 grid_up=0, grid_matvec=0, theta=None, sigma=None, load=None, region=None, device=None):
        import torch
        self.lib = L.load()
        self.problem = problem
        self.n, self.N = int(problem.n), int(problem.N)
        self.S = self.N // 2
        self.nodes = (self.n + 1) ** 2
        self.precision = precision
        self._keep = (theta, sigma, load, region)  # device tables must outlive the plan's calls
        self._ps = problem_struct(problem, theta, sigma, load, region)
        o = _options(self.lib, tol, max_outer, check_every, precision, inner, inner_iters, vc_omega,
                     use_initial_guess, diverge_factor, xcd_remap, timing, graph, grid_slot, grid_team, adjoint,
                     init_static, init_tol, stop_relative_initial, krylov_dim, forcing, max_krylov, inner_rtol,
                     breakdown_tol, cycle, grid_restrict, grid_up, grid_matvec)
        self._opts = o
        h = C.c_void_p()
        st = self.lib.pt_plan_create(C.byref(self._ps), C.byref(o), C.byref(h))
        if st != L.PT_OK:
            raise PTError(st, "pt_plan_create")
        self._h = h
        nb = C.c_size_t()
        self._check(self.lib.pt_plan_workspace_bytes(self._h, C.byref(nb)), "pt_plan_workspace_bytes")
        self.workspace_bytes = int(nb.value)
        self.device = torch.device(device) if device is not None else None
        self._ws = None
        self.cdtype = torch.complex128 if precision == "fp64" else torch.complex64

    # ---------------------------------------------------------------- helpers
    def _check(self, st, where):
        if st != L.PT_OK:
            raise PTError(st, where)

    def workspace(self):
        import torch
        if self._ws is None:
            dev = self.device or torch.device("cuda", torch.cuda.current_device())
            self._ws = torch.empty(self.workspace_bytes + 256, dtype=torch.uint8, device=dev)
        base = self._ws.data_ptr()
        off = (-base) % 256
        return C.c_void_p(base + off), C.c_size_t(self.workspace_bytes)

    @staticmethod
    def _stream():
        import torch
        return C.c_void_p(torch.cuda.current_stream().cuda_stream)

    def _time_field(self, t, name):
        import torch
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or \
                tuple(t.shape) != (self.N, self.n + 1, self.n + 1):
            raise ValueError(f"{name} must be a contiguous float64 device tensor of shape "
                             f"({self.N}, {self.n + 1}, {self.n + 1})")
        return C.c_void_p(t.data_ptr())

    def _freq_field(self, t, name):
        if t.dtype != self.cdtype or not t.is_cuda or not t.is_contiguous() or \
                tuple(t.shape) != (self.nodes, self.S):
            raise ValueError(f"{name} must be a contiguous {self.cdtype} device tensor of shape "
                             f"({self.nodes}, {self.S})")
        return C.c_void_p(t.data_ptr())

    def new_time_field(self):
        import torch
        dev = self.device or torch.device("cuda", torch.cuda.current_device())
        return torch.zeros((self.N, self.n + 1, self.n + 1), dtype=torch.float64, device=dev)

    def new_freq_field(self):
        import torch
        dev = self.device or torch.device("cuda", torch.cuda.current_device())
        return torch.zeros((self.nodes, self.S), dtype=self.cdtype, device=dev)

    # ---------------------------------------------------------------- entry points
    def solve(self, U=None, history_cap: int = 4096, raise_on_error: bool = True):
        if U is None:
            U = self.new_time_field()
        ws, nb = self.workspace()
        buf = _StatsBuf(history_cap)
        s = L.Stats()
        buf.fill(s)
        st = self.lib.pt_solve(self._h, ws, nb, self._time_field(U, "U"), self._stream(), C.byref(s))
        stats = buf.result(self.lib, st, s)
        if raise_on_error and st != L.PT_OK:
            raise PTError(st, "pt_solve")
        return U, stats

    def solve_noalloc(self, U=None, history_cap: int = 4096, raise_on_error: bool = True):
        """pt_solve_noalloc: the solve with the library's static device scratch as its workspace
        (no workspace tensor is allocated or passed)."""
        if U is None:
            U = self.new_time_field()
        buf = _StatsBuf(history_cap)
        s = L.Stats()
        buf.fill(s)
        st = self.lib.pt_solve_noalloc(self._h, self._solution_field(U, "U"), self._stream(), C.byref(s))
        stats = buf.result(self.lib, st, s)
        if raise_on_error and st != L.PT_OK:
            raise PTError(st, "pt_solve_noalloc")
        return U, stats

    def _solution_field(self, t, name):
        return self._time_field(t, name)

    def adjoint_solve(self, U, Lam=None, history_cap: int = 4096, raise_on_error: bool = True):
        """Adjoint state lambda of the eddy-current loss at the state U (pt_adjoint_solve);
        Lam is the output (and the initial guess if the plan uses one)."""
        if Lam is None:
            Lam = self.new_time_field()
        ws, nb = self.workspace()
        buf = _StatsBuf(history_cap)
        s = L.Stats()
        buf.fill(s)
        st = self.lib.pt_adjoint_solve(self._h, ws, nb, self._time_field(U, "U"), self._time_field(Lam, "Lam"),
                                       self._stream(), C.byref(s))
        stats = buf.result(self.lib, st, s)
        if raise_on_error and st != L.PT_OK:
            raise PTError(st, "pt_adjoint_solve")
        return Lam, stats

    def newton_solve(self, U=None, history_cap: int = 512, raise_on_error: bool = True):
        """Newton's method with flexible GMRES steps and Armijo backtracking (pt_newton_solve)."""
        if U is None:
            U = self.new_time_field()
        ws, nb = self.workspace()
        buf = _StatsBuf(history_cap)
        s = L.Stats()
        buf.fill(s)
        st = self.lib.pt_newton_solve(self._h, ws, nb, self._time_field(U, "U"), self._stream(), C.byref(s))
        stats = buf.result(self.lib, st, s)
        if raise_on_error and st != L.PT_OK:
            raise PTError(st, "pt_newton_solve")
        return U, stats

    def jacobian_apply(self, U, V, transpose: bool = False):
        """J(U) V or J(U)^T V (pt_jacobian_apply)."""
        out = self.new_time_field()
        ws, nb = self.workspace()
        self._check(self.lib.pt_jacobian_apply(self._h, ws, nb, self._time_field(U, "U"), self._time_field(V, "V"),
                                               C.c_void_p(out.data_ptr()), 1 if transpose else 0, self._stream()),
                    "pt_jacobian_apply")
        return out

    def loss_gradients(self, U, Lam=None, per_cell: bool = False):
        """(loss, dl/dtheta, dl/dsigma) at the state U with adjoint state Lam (pt_loss_gradients);
        per triangle (2 n^2) or per cell (n^2)."""
        import torch
        dev = U.device
        m = self.n * self.n * (1 if per_cell else 2)
        gt = torch.zeros(m, dtype=torch.float64, device=dev)
        gs = torch.zeros(m, dtype=torch.float64, device=dev)
        ws, nb = self.workspace()
        loss = C.c_double()
        lam = None if Lam is None else self._time_field(Lam, "Lam")
        self._check(self.lib.pt_loss_gradients(self._h, ws, nb, self._time_field(U, "U"), lam,
                                               C.c_void_p(gt.data_ptr()), C.c_void_p(gs.data_ptr()),
                                               1 if per_cell else 0, C.byref(loss), self._stream()),
                    "pt_loss_gradients")
        return loss.value, gt, gs

    def residual(self, U):
        R = self.new_time_field()
        ws, nb = self.workspace()
        rel, fn = C.c_double(), C.c_double()
        self._check(self.lib.pt_residual(self._h, ws, nb, self._time_field(U, "U"), C.c_void_p(R.data_ptr()),
                                         self._stream(), C.byref(rel), C.byref(fn)), "pt_residual")
        return R, rel.value, fn.value

    def residual_spectrum(self, U):
        """Packed real DFT along time of R = F - A(U) (the frequency field the fixed-point step
        feeds to the frequency solve), with ||R||/||F|| and ||F||."""
        Rh = self.new_freq_field()
        ws, nb = self.workspace()
        rel, fn = C.c_double(), C.c_double()
        self._check(self.lib.pt_residual_spectrum(self._h, ws, nb, self._time_field(U, "U"),
                                                  C.c_void_p(Rh.data_ptr()), self._stream(), C.byref(rel),
                                                  C.byref(fn)), "pt_residual_spectrum")
        return Rh, rel.value, fn.value

    def apply_K(self, U, nslices=None):
        nslices = self.N if nslices is None else int(nslices)
        KU = self.new_time_field()
        ws, nb = self.workspace()
        self._check(self.lib.pt_apply_K(self._h, ws, nb, self._time_field(U, "U"), C.c_void_p(KU.data_ptr()),
                                        nslices, self._stream()), "pt_apply_K")
        return KU

    def rfft(self, X):
        Y = self.new_freq_field()
        ws, nb = self.workspace()
        self._check(self.lib.pt_time_rfft(self._h, ws, nb, self._time_field(X, "X"), C.c_void_p(Y.data_ptr()),
                                          self._stream()), "pt_time_rfft")
        return Y

    def irfft(self, Y):
        X = self.new_time_field()
        ws, nb = self.workspace()
        self._check(self.lib.pt_time_irfft(self._h, ws, nb, self._freq_field(Y, "Y"), C.c_void_p(X.data_ptr()),
                                           self._stream()), "pt_time_irfft")
        return X

    def shifted_apply(self, Xh):
        Yh = self.new_freq_field()
        ws, nb = self.workspace()
        self._check(self.lib.pt_shifted_apply(self._h, ws, nb, self._freq_field(Xh, "X"),
                                              C.c_void_p(Yh.data_ptr()), self._stream()), "pt_shifted_apply")
        return Yh

    def precond_apply(self, Rh):
        Xh = self.new_freq_field()
        ws, nb = self.workspace()
        self._check(self.lib.pt_precond_apply(self._h, ws, nb, self._freq_field(Rh, "R"),
                                              C.c_void_p(Xh.data_ptr()), self._stream()), "pt_precond_apply")
        return Xh

    def periodic_solve(self, R, inner_iters: int = 0):
        X = self.new_time_field()
        ws, nb = self.workspace()
        self._check(self.lib.pt_periodic_solve(self._h, ws, nb, self._time_field(R, "R"), C.c_void_p(X.data_ptr()),
                                               int(inner_iters), self._stream()), "pt_periodic_solve")
        return X

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.pt_plan_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan(Plan):
    """count instances of one grid and period (shared conductivity and nu_max) solved
    together: pt_plan_create_batch / pt_solve_batch. count must be a power of two."""

    def __init__(self, problems, *, tol=1e-8, max_outer=1000, check_every=1, precision="fp64",
                 inner="galerkin1", inner_iters=1, vc_omega=0.8, use_initial_guess=False,
                 diverge_factor=1e3, xcd_remap=True, timing=False, graph=False, grid_slot=0, grid_team=0,
                 adjoint=False, init_static=False, init_tol=1e-8, stop_relative_initial=False, krylov_dim=0,
                 forcing=1e-2, max_krylov=100, inner_rtol=0.0, breakdown_tol=0.0, cycle="default", grid_restrict=0,
                 grid_up=0, grid_matvec=0, device=None):
        import torch
        problems = list(problems)
        self.lib = L.load()
        self.problems = problems
        self.problem = problems[0]
        self.count = len(problems)
        self.n, self.N = int(self.problem.n), int(self.problem.N)
        self.S = self.N // 2
        self.nodes = (self.n + 1) ** 2
        self.precision = precision
        self._keep = ()
        self._pa = (L.Problem * self.count)(*[problem_struct(p) for p in problems])
        o = _options(self.lib, tol, max_outer, check_every, precision, inner, inner_iters, vc_omega,
                     use_initial_guess, diverge_factor, xcd_remap, timing, graph, grid_slot, grid_team, adjoint,
                     init_static, init_tol, stop_relative_initial, krylov_dim, forcing, max_krylov, inner_rtol,
                     breakdown_tol, cycle, grid_restrict, grid_up, grid_matvec)
        self._opts = o
        h = C.c_void_p()
        st = self.lib.pt_plan_create_batch(self._pa, self.count, C.byref(o), C.byref(h))
        if st != L.PT_OK:
            raise PTError(st, "pt_plan_create_batch")
        self._h = h
        nb = C.c_size_t()
        self._check(self.lib.pt_plan_workspace_bytes(self._h, C.byref(nb)), "pt_plan_workspace_bytes")
        self.workspace_bytes = int(nb.value)
        self.device = torch.device(device) if device is not None else None
        self._ws = None
        self.cdtype = torch.complex128 if precision == "fp64" else torch.complex64

    def new_time_field(self):
        import torch
        dev = self.device or torch.device("cuda", torch.cuda.current_device())
        return torch.zeros((self.count, self.N, self.n + 1, self.n + 1), dtype=torch.float64, device=dev)

    def _batch_field(self, t, name):
        import torch
        if t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous() or \
                tuple(t.shape) != (self.count, self.N, self.n + 1, self.n + 1):
            raise ValueError(f"{name} must be a contiguous float64 device tensor of shape "
                             f"({self.count}, {self.N}, {self.n + 1}, {self.n + 1})")
        return C.c_void_p(t.data_ptr())

    def solve(self, U=None, history_cap: int = 4096, raise_on_error: bool = True):
        """Returns U [count, N, n+1, n+1] and one SolveStats per instance."""
        if U is None:
            U = self.new_time_field()
        ws, nb = self.workspace()
        bufs = [_StatsBuf(history_cap) for _ in range(self.count)]
        sa = (L.Stats * self.count)()
        for b, buf in zip(bufs, sa):
            b.fill(buf)
        st = self.lib.pt_solve_batch(self._h, ws, nb, self._batch_field(U, "U"), self._stream(), sa)
        stats = [b.result(self.lib, st, s) for b, s in zip(bufs, sa)]
        if raise_on_error and st != L.PT_OK:
            raise PTError(st, "pt_solve_batch")
        return U, stats

    def _solution_field(self, t, name):
        return self._batch_field(t, name)

    def solve_noalloc(self, U=None, history_cap: int = 4096, raise_on_error: bool = True):
        """pt_solve_noalloc for the batch: U [count, N, n+1, n+1] and one SolveStats per instance."""
        if U is None:
            U = self.new_time_field()
        bufs = [_StatsBuf(history_cap) for _ in range(self.count)]
        sa = (L.Stats * self.count)()
        for b, buf in zip(bufs, sa):
            b.fill(buf)
        st = self.lib.pt_solve_noalloc(self._h, self._batch_field(U, "U"), self._stream(), sa)
        stats = [b.result(self.lib, st, s) for b, s in zip(bufs, sa)]
        if raise_on_error and st != L.PT_OK:
            raise PTError(st, "pt_solve_noalloc")
        return U, stats

    def _single(self, *a, **k):
        raise TypeError("component entry points take a single-problem plan")

    residual = residual_spectrum = apply_K = rfft = irfft = shifted_apply = precond_apply = periodic_solve = _single
    adjoint_solve = loss_gradients = newton_solve = jacobian_apply = _single
