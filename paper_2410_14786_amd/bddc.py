"""Python binding of libbddc.so (ctypes): argument marshalling only.

Every numerical step runs in the HIP library; torch supplies device memory and
the stream.  Importing this module without a built library raises ImportError:
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from typing import Dict, Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbddc.so")

CORNERS, EDGES, FACES, ALL_PRIMAL = 1, 2, 4, 8
X0_GIVEN = 1
SETUP_KEEP_ON_ERROR, SETUP_FULL_SPACE, SETUP_RHO_SCALING, SETUP_COARSE_CG = 1, 2, 4, 8

OK, EINVAL, ENOTSPD, ENOMEM, EHIP, ENOCONV, EBREAKDOWN, ENOTIMPL = 0, -1, -2, -3, -4, -5, -6, -7


class Mesh(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nel", ctypes.c_int64 * 3)]


class Partition(ctypes.Structure):
    _fields_ = [("nsub", ctypes.c_int32 * 3), ("cuts", ctypes.POINTER(ctypes.c_int64) * 3)]


class Coefficients(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_void_p), ("on_device", ctypes.c_int32)]


class Options(ctypes.Structure):
    _fields_ = [("local_bits", ctypes.c_int32), ("use_graph", ctypes.c_int32), ("nb_override", ctypes.c_int32),
                ("stream", ctypes.c_void_p), ("flags", ctypes.c_int32)]


class PcgInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("relres_true", ctypes.c_double), ("relres_rec", ctypes.c_double),
                ("cond_est", ctypes.c_double), ("t_setup_ms", ctypes.c_double), ("t_solve_ms", ctypes.c_double)]


EXPORTS = ["bddc_setup", "bddc_apply", "bddc_pcg_solve", "bddc_spmv", "bddc_elem_grad", "bddc_query",
           "bddc_plan_stats", "bddc_set_timing", "bddc_kernel_time", "bddc_destroy", "bddc_strerror",
           "bddc_last_error", "bddc_debug_read", "bddc_set_tuning", "bddc_autotune", "bddc_setup_stats",
           "bddc_apply_noalloc", "bddc_set_limit", "bddc_sync"]

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run __graft_entry__.build() (hipcc, gfx950)")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.bddc_setup.argtypes = [ctypes.POINTER(Mesh), ctypes.POINTER(Partition), ctypes.POINTER(Coefficients),
                               ctypes.c_uint32, ctypes.POINTER(Options), ctypes.POINTER(vp)]
    lib.bddc_apply.argtypes = [vp, vp, vp]
    lib.bddc_apply_noalloc.argtypes = [vp, vp, vp]
    lib.bddc_set_limit.argtypes = [vp, ctypes.c_char_p, i32]
    lib.bddc_sync.argtypes = [vp]
    lib.bddc_pcg_solve.argtypes = [vp, vp, vp, dbl, i32, i32, ctypes.POINTER(PcgInfo)]
    lib.bddc_spmv.argtypes = [vp, vp, vp]
    lib.bddc_elem_grad.argtypes = [vp, vp, vp, vp]
    lib.bddc_query.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(i32), ctypes.POINTER(i32),
                               ctypes.POINTER(i64)]
    lib.bddc_plan_stats.argtypes = [ctypes.POINTER(Mesh), ctypes.POINTER(Partition), ctypes.c_uint32,
                                    ctypes.POINTER(i64)]
    lib.bddc_set_timing.argtypes = [vp, i32]
    lib.bddc_kernel_time.argtypes = [vp, ctypes.c_char_p, ctypes.POINTER(i64), ctypes.POINTER(dbl)]
    lib.bddc_debug_read.argtypes = [vp, ctypes.c_char_p, i32, ctypes.POINTER(dbl), i64]
    lib.bddc_debug_read.restype = ctypes.c_int64
    lib.bddc_set_tuning.argtypes = [vp, i32]
    lib.bddc_set_tuning.restype = ctypes.c_int
    lib.bddc_autotune.argtypes = [vp, ctypes.POINTER(i32), i32, i32, ctypes.POINTER(i32), ctypes.POINTER(dbl)]
    lib.bddc_autotune.restype = ctypes.c_int
    lib.bddc_setup_stats.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
    lib.bddc_setup_stats.restype = ctypes.c_int
    lib.bddc_destroy.argtypes = [vp]
    lib.bddc_destroy.restype = None
    lib.bddc_strerror.argtypes = [ctypes.c_int]
    lib.bddc_strerror.restype = ctypes.c_char_p
    lib.bddc_last_error.argtypes = []
    lib.bddc_last_error.restype = ctypes.c_char_p
    for name in ["bddc_setup", "bddc_apply", "bddc_apply_noalloc", "bddc_set_limit", "bddc_sync", "bddc_pcg_solve", "bddc_spmv", "bddc_elem_grad", "bddc_query",
                 "bddc_plan_stats", "bddc_set_timing", "bddc_kernel_time"]:
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class BDDCError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def _check(code: int, what: str):
    if code != OK:
        lib = load_library()
        raise BDDCError(code, f"{what}: {lib.bddc_strerror(code).decode()}: {lib.bddc_last_error().decode()}")


def _mesh_partition(dim: int, nel: Sequence[int], cuts: Sequence[Sequence[int]]):
    m = Mesh()
    m.dim = dim
    for a in range(3):
        m.nel[a] = int(nel[a]) if a < min(dim, len(nel)) else 1
    p = Partition()
    keep = []
    for a in range(3):
        c = np.ascontiguousarray(cuts[a] if a < min(dim, len(cuts)) else [0, 1], dtype=np.int64)
        keep.append(c)
        p.nsub[a] = len(c) - 1
        p.cuts[a] = c.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    return m, p, keep


def plan_stats(dim: int, nel: Sequence[int], cuts: Sequence[Sequence[int]], constraints: int) -> Dict[str, int]:
    """Host-only planning sizes (no GPU needed)."""
    lib = load_library()
    m, p, keep = _mesh_partition(dim, nel, cuts)
    out = (ctypes.c_int64 * 8)()
    _check(lib.bddc_plan_stats(ctypes.byref(m), ctypes.byref(p), constraints, out), "bddc_plan_stats")
    names = ["n_free", "n_sub", "n_coarse", "corners", "edges", "faces", "sum_ni", "max_nci"]
    return {k: int(v) for k, v in zip(names, out)}


def _dev_ptr(t, name: str) -> int:
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float64 CUDA tensor")
    return t.data_ptr()


class Solver:
    """A BDDC preconditioner and PCG solver on one GPU (owns a bddc_ctx)."""

    def __init__(self, dim: int, nel: Sequence[int], cuts: Sequence[Sequence[int]], theta, constraints: int,
                 local_bits: int = 64, use_graph: bool = False, stream=None, keep_on_error: bool = False,
                 full_space: bool = False, rho_scaling: bool = False, coarse_cg: bool = False):
        import torch
        self.lib = load_library()
        self.dim = dim
        self.nel = tuple(int(n) for n in nel[:dim])
        m, p, keep = _mesh_partition(dim, nel, cuts)
        co = Coefficients()
        if isinstance(theta, torch.Tensor) and theta.is_cuda:
            th = theta.to(torch.float64).contiguous()
            co.theta = th.data_ptr()
            co.on_device = 1
        else:
            th = np.ascontiguousarray(theta.cpu().numpy() if isinstance(theta, torch.Tensor) else theta,
                                      dtype=np.float64)
            co.theta = th.ctypes.data
            co.on_device = 0
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        opt = Options()
        opt.local_bits = local_bits
        opt.use_graph = int(use_graph)
        opt.nb_override = 0
        opt.stream = stream.cuda_stream
        opt.flags = ((SETUP_KEEP_ON_ERROR if keep_on_error else 0) | (SETUP_FULL_SPACE if full_space else 0)
                     | (SETUP_RHO_SCALING if rho_scaling else 0) | (SETUP_COARSE_CG if coarse_cg else 0))
        ctx = ctypes.c_void_p()
        code = self.lib.bddc_setup(ctypes.byref(m), ctypes.byref(p), ctypes.byref(co), constraints,
                                   ctypes.byref(opt), ctypes.byref(ctx))
        self.setup_status = code
        if not (keep_on_error and ctx.value):
            _check(code, "bddc_setup")
        self.ctx = ctx
        n, ns, nc, nb = ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
        _check(self.lib.bddc_query(self.ctx, ctypes.byref(n), ctypes.byref(ns), ctypes.byref(nc), ctypes.byref(nb)),
               "bddc_query")
        self.n_free, self.n_sub, self.n_coarse, self.dev_bytes = n.value, ns.value, nc.value, nb.value
        self.n_el = int(np.prod(self.nel))
        self.wg_per_cu = 4
        box = sorted({tuple(int(c[i + 1] - c[i]) for i in range(len(c) - 1)) for c in
                      (np.asarray(cc) for cc in cuts[:dim])})
        self.tune_key = (f"dim{dim}|nel{'x'.join(map(str, self.nel))}|boxes{box}|bits{local_bits}|"
                         f"{'full' if full_space else 'iface'}|graph{int(use_graph)}|rho{int(rho_scaling)}|"
                         f"ccg{int(coarse_cg)}")

    def close(self):
        if getattr(self, "ctx", None) is not None and self.ctx.value:
            self.lib.bddc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self, n):
        import torch
        return torch.empty(n, dtype=torch.float64, device="cuda")

    def apply(self, r, out=None):
        z = self._new(self.n_free) if out is None else out
        _check(self.lib.bddc_apply(self.ctx, _dev_ptr(r, "r"), _dev_ptr(z, "z")), "bddc_apply")
        return z

    def apply_noalloc(self, r, out):
        """z = M^{-1} r through bddc_apply_noalloc (fixed device workspace; the
        caller provides z)."""
        _check(self.lib.bddc_apply_noalloc(self.ctx, _dev_ptr(r, "r"), _dev_ptr(out, "z")), "bddc_apply_noalloc")
        return out

    def set_limit(self, what: str, value: int):
        """Device-side limits for failure-path tests: "wait_polls", "coarse_cg_maxit"."""
        _check(self.lib.bddc_set_limit(self.ctx, what.encode(), int(value)), "bddc_set_limit")

    def sync(self):
        """Wait for the ctx stream; raise BDDCError if a device-side wait gave up or the
        coarse CG did not converge since the last report."""
        _check(self.lib.bddc_sync(self.ctx), "bddc_sync")

    def spmv(self, x, out=None):
        y = self._new(self.n_free) if out is None else out
        _check(self.lib.bddc_spmv(self.ctx, _dev_ptr(x, "x"), _dev_ptr(y, "y")), "bddc_spmv")
        return y

    def elem_grad(self, lam, u, out=None):
        g = self._new(self.n_el) if out is None else out
        _check(self.lib.bddc_elem_grad(self.ctx, _dev_ptr(lam, "lam"), _dev_ptr(u, "u"), _dev_ptr(g, "g")),
               "bddc_elem_grad")
        return g

    def solve(self, b, rtol: float, maxit: int = 2000, x0=None, out=None, raise_on_noconv: bool = True):
        x = out if out is not None else self._new(self.n_free)
        flags = 0
        if x0 is not None:
            x.copy_(x0)
            flags = X0_GIVEN
        info = PcgInfo()
        code = self.lib.bddc_pcg_solve(self.ctx, _dev_ptr(b, "b"), _dev_ptr(x, "x"), float(rtol), int(maxit), flags,
                                       ctypes.byref(info))
        if code != OK and not (code == ENOCONV and not raise_on_noconv):
            _check(code, "bddc_pcg_solve")
        return x, {"iters": info.iters, "relres_true": info.relres_true, "relres_rec": info.relres_rec,
                   "cond_est": info.cond_est, "t_setup_ms": info.t_setup_ms, "t_solve_ms": info.t_solve_ms,
                   "status": code}

    def debug_read(self, what: str, sub: int) -> np.ndarray:
        """One subdomain's setup data (test access): sizes, factor, border, schur,
        aci, gmap, dscale, envelope."""
        cap = 64 * 1024 * 1024
        sizes = np.zeros(6)
        n = self.lib.bddc_debug_read(self.ctx, b"sizes", sub, sizes.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 6)
        if n < 0:
            _check(int(n), "bddc_debug_read")
        T = int(sizes[4])
        need = {"sizes": 6, "factor": (T * 64) ** 2, "border": 64 * T * 64, "schur": 4096, "aci": 4096,
                "gmap": int(sizes[5]), "dscale": int(sizes[5]), "envelope": 2 * T}[what]
        buf = np.zeros(min(need, cap))
        n = self.lib.bddc_debug_read(self.ctx, what.encode(), sub, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                     len(buf))
        if n < 0:
            _check(int(n), "bddc_debug_read")
        return buf[:n]

    def setup_stats(self):
        """Floating-point operations of the batched local factorisation (inside the
        factors' envelope) and its GPU time at setup in ms."""
        fl, ms = ctypes.c_double(), ctypes.c_double()
        _check(self.lib.bddc_setup_stats(self.ctx, ctypes.byref(fl), ctypes.byref(ms)), "bddc_setup_stats")
        return fl.value, ms.value

    def set_tuning(self, wg_per_cu: int):
        _check(self.lib.bddc_set_tuning(self.ctx, int(wg_per_cu)), "bddc_set_tuning")
        self.wg_per_cu = int(wg_per_cu)

    def autotune(self, candidates=(1, 2, 3, 4, 6, 8), iters: int = 8, cache: Optional[str] = None):
        """Pick the persistent-kernel launch shape by timing short PCG runs; the
        choice is cached in a JSON file keyed by GPU architecture and problem
        shape (cache=None: ~/.cache/bddc/autotune.json, "" disables caching)."""
        import json
        import torch
        if cache is None:
            cache = os.path.join(os.path.expanduser("~"), ".cache", "bddc", "autotune.json")
        arch = torch.cuda.get_device_properties(0).gcnArchName if torch.cuda.is_available() else "cpu"
        key = f"{arch}|{self.tune_key}"
        table = {}
        if cache:
            try:
                with open(cache) as f:
                    table = json.load(f)
            except (OSError, ValueError):
                table = {}
            if key in table:
                self.set_tuning(table[key]["wg_per_cu"])
                return table[key]
        cand = (ctypes.c_int32 * len(candidates))(*candidates)
        ms = (ctypes.c_double * len(candidates))()
        best = ctypes.c_int32()
        _check(self.lib.bddc_autotune(self.ctx, cand, len(candidates), int(iters), ctypes.byref(best), ms),
               "bddc_autotune")
        self.wg_per_cu = best.value
        rec = {"wg_per_cu": best.value, "candidates": list(candidates), "ms": [round(v, 4) for v in ms],
               "iters": iters}
        if cache:
            table[key] = rec
            os.makedirs(os.path.dirname(cache), exist_ok=True)
            with open(cache, "w") as f:
                json.dump(table, f, indent=1)
        return rec

    def set_timing(self, on: bool):
        _check(self.lib.bddc_set_timing(self.ctx, int(on)), "bddc_set_timing")

    def kernel_time(self, family: str):
        n, ms = ctypes.c_int64(), ctypes.c_double()
        _check(self.lib.bddc_kernel_time(self.ctx, family.encode(), ctypes.byref(n), ctypes.byref(ms)),
               "bddc_kernel_time")
        return n.value, ms.value


def solver_for(w, local_bits: Optional[int] = None, use_graph: bool = False, full_space: bool = False,
               rho_scaling: bool = False, coarse_cg: bool = False) -> Solver:
    """Solver for a workloads.Workload."""
    return Solver(w.dim, w.nel, w.cuts, w.theta, w.constraints,
                  local_bits=w.local_bits if local_bits is None else local_bits, use_graph=use_graph,
                  full_space=full_space, rho_scaling=rho_scaling, coarse_cg=coarse_cg)


def _autograd_function():
    import torch

    class BDDCSolve(torch.autograd.Function):
        """u = A(theta)^{-1} b by BDDC-PCG; the backward pass runs the adjoint
        BDDC-PCG solve A lam = dJ/du on the same preconditioner (A is symmetric)
        and the per-element kernel dJ/dtheta_e = -lam_e^T K_ref u_e."""

        @staticmethod
        def forward(ctx, theta, b, dim, nel, cuts, constraints, rtol, local_bits):
            solver = Solver(dim, nel, cuts, theta.detach(), constraints, local_bits=local_bits)
            u, info = solver.solve(b.detach().contiguous(), rtol)
            ctx.solver = solver
            ctx.rtol = rtol
            ctx.info = info
            ctx.save_for_backward(u)
            return u

        @staticmethod
        def backward(ctx, grad_u):
            (u,) = ctx.saved_tensors
            solver = ctx.solver
            lam, _ = solver.solve(grad_u.contiguous(), ctx.rtol)
            g = solver.elem_grad(lam, u)
            return g, lam, None, None, None, None, None, None

    return BDDCSolve


def bddc_solve(theta, b, dim, nel, cuts, constraints, rtol=1e-10, local_bits=64):
    """Differentiable solve u = A(theta)^{-1} b (gradients for theta and b)."""
    return _autograd_function().apply(theta, b, dim, tuple(nel), [list(map(int, c)) for c in cuts],
                                      constraints, rtol, local_bits)
