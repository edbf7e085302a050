"""MI355X (gfx950) solver for the reduced camera system of bundle adjustment.

Python binding of libba.so (include/ba.h): block-Jacobi PCG (Algorithm 1) and
Multidirectional CG (Algorithm 2) of Weber, Demmel, Cremers (GCPR 2021) on the
implicit Schur complement S = U - W V^-1 W^T.  PyTorch provides device memory
and the stream; every arithmetic step runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import _lib
from ._lib import (BA_ERR_BREAKDOWN, BA_ERR_HIP, BA_ERR_INVALID_ARG, BA_ERR_NOMEM, BA_ERR_NONFINITE,
                   BA_ERR_NOT_SPD, BA_ERR_UNSUPPORTED, BA_ERR_WORKSPACE, BA_MAXITER, BA_OK, PREC)

__all__ = ["System", "Batch", "BatchStats", "BAError", "Stats", "pinv_sym", "partition", "PREC", "lib",
           "mlp_forward", "mlp_loss_grad", "adam_step", "MLP_PARAMS", "Scene", "LMStats"]

MLP_PARAMS = 15432


def lib() -> C.CDLL:
    return _lib.load()


class BAError(RuntimeError):
    def __init__(self, status: int, where: str):
        L = lib()
        msg = L.ba_last_error().decode()
        super().__init__(f"{where}: {L.ba_status_string(status).decode()} ({status}): {msg}")
        self.status = status


def _check(st: int, where: str) -> int:
    if st < 0:
        raise BAError(st, where)
    return st


def _torch():
    import torch
    return torch


def _dev_ptr(t, dtype, numel=None, name="tensor"):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name} must have {numel} elements, has {t.numel()}")
    return C.c_void_p(t.data_ptr())


def _stream_handle(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


@dataclass
class Stats:
    iterations: int
    multi_steps: int
    history_cols: int
    refinement_steps: int
    status: int
    rel_res_recursive: float
    rel_res_true: float
    t_solve_ms: float
    trace_res: np.ndarray = field(default_factory=lambda: np.zeros(0))
    trace_t: np.ndarray = field(default_factory=lambda: np.zeros(0))
    trace_k: np.ndarray = field(default_factory=lambda: np.zeros(0, dtype=np.int32))


def _opts(eps, max_iter, precision, max_history_cols=0, inner_eps=0.0, max_outer=20, max_inner=1000,
          precond=0, history_mfma=False, history_fp32=None):
    o = _lib.SolveOpts()
    lib().ba_default_solve_opts(C.byref(o))
    o.eps = float(eps)
    o.max_iter = int(max_iter)
    o.precision = PREC[precision] if isinstance(precision, str) else int(precision)
    o.max_history_cols = int(max_history_cols)
    o.inner_eps = float(inner_eps)
    o.max_outer = int(max_outer)
    o.max_inner = int(max_inner)
    o.precond = int(precond)
    o.history_mfma = 1 if history_mfma else 0
    if history_fp32 is not None:   # None keeps the library default (on)
        o.history_fp32 = 1 if history_fp32 else 0
    return o


class _Trace:
    def __init__(self, cap):
        self.cap = cap
        self.res = np.full(cap, np.nan)
        self.t = np.full(cap, np.nan)
        self.k = np.zeros(cap, dtype=np.int32)

    def attach(self, st):
        st.trace_cap = self.cap
        st.trace_res = self.res.ctypes.data_as(C.POINTER(C.c_double))
        st.trace_t = self.t.ctypes.data_as(C.POINTER(C.c_double))
        st.trace_k = self.k.ctypes.data_as(C.POINTER(C.c_int32))


def _stats(st, tr: Optional[_Trace]) -> Stats:
    s = Stats(st.iterations, st.multi_steps, st.history_cols, st.refinement_steps, st.status,
              st.rel_res_recursive, st.rel_res_true, st.t_solve_ms)
    if tr is not None:
        n = min(st.iterations, tr.cap)
        s.trace_res, s.trace_t, s.trace_k = tr.res[:n].copy(), tr.t[:n].copy(), tr.k[:n].copy()
    return s


class System:
    """A built reduced camera system (ba_build_system) living on one device."""

    def __init__(self, n_cams, n_lms, obs_cam, obs_lm, J_p, J_l, r, lam, stream=None,
                 max_slots=0, max_tiles=0, store_fp32=False, store_bf16=False, explicit_schur=False,
                 max_tiles_multi=0, workspace=None, ws_groups=0, ws_max_iter=0, size_only=False):
        """workspace: a device uint8 tensor for ba_build_system_ws (kept alive by the object);
        size_only: only run ba_build_workspace_bytes and keep its result in self.ws_bytes."""
        torch = _torch()
        m = int(obs_cam.numel())
        # pose dimension (Sec. 3.1): 9, or 6 for extrinsics only, from the size of J_p
        dp = int(J_p.numel()) // max(2 * m, 1)
        d = _lib.ProblemDesc()
        d.n_cams, d.n_lms, d.n_obs, d.d_p = int(n_cams), int(n_lms), m, dp
        d.obs_cam = _dev_ptr(obs_cam, torch.int32, m, "obs_cam")
        d.obs_lm = _dev_ptr(obs_lm, torch.int32, m, "obs_lm")
        d.J_p = _dev_ptr(J_p, torch.float64, m * 2 * dp, "J_p")
        d.J_l = _dev_ptr(J_l, torch.float64, m * 6, "J_l")
        d.r = _dev_ptr(r, torch.float64, m * 2, "r")
        d.lam = float(lam)
        o = _lib.BuildOpts()
        o.store_fp32, o.store_bf16 = int(store_fp32), int(store_bf16)
        o.max_slots, o.max_tiles, o.max_tiles_multi = int(max_slots), int(max_tiles), int(max_tiles_multi)
        o.explicit_schur = int(explicit_schur)
        o.ws_groups, o.ws_max_iter = int(ws_groups), int(ws_max_iter)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = obs_cam.device
        self.n_cams, self.n_lms, self.n_obs = int(n_cams), int(n_lms), m
        self.d_p = dp
        self.n = dp * self.n_cams
        h = C.c_void_p()
        self._ws = workspace
        if size_only:
            nb = C.c_size_t()
            _check(lib().ba_build_workspace_bytes(C.byref(d), C.byref(o), C.byref(nb)), "ba_build_workspace_bytes")
            self.ws_bytes = int(nb.value)
            self.h = None
            return
        if workspace is not None:
            if not isinstance(workspace, torch.Tensor) or not workspace.is_cuda or workspace.dtype != torch.uint8:
                raise TypeError("workspace must be a device uint8 tensor")
            _check(lib().ba_build_system_ws(C.byref(d), C.byref(o), C.c_void_p(workspace.data_ptr()),
                                            C.c_size_t(workspace.numel()), _stream_handle(self._stream), C.byref(h)),
                   "ba_build_system_ws")
        else:
            _check(lib().ba_build_system(C.byref(d), C.byref(o), _stream_handle(self._stream), C.byref(h)),
                   "ba_build_system")
        self.h = h

    def workspace_used(self):
        """Bytes of the caller's workspace used so far (ba_system_workspace_used)."""
        nb = C.c_size_t()
        _check(lib().ba_system_workspace_used(self.h, C.byref(nb)), "ba_system_workspace_used")
        return int(nb.value)

    @classmethod
    def from_problem(cls, p, device="cuda", **kw):
        """Upload a synthetic problem (host arrays) and build its system."""
        torch = _torch()
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        return cls(p.n_cams, p.n_lms, t(p.obs_cam, torch.int32), t(p.obs_lm, torch.int32),
                   t(p.J_p, torch.float64), t(p.J_l, torch.float64), t(p.r, torch.float64), p.lam, **kw)

    @classmethod
    def _view(cls, h, n_cams, n_lms, n_obs, device, stream):
        """A System object over a system owned elsewhere (the block-diagonal system of a batch)."""
        obj = cls.__new__(cls)
        obj.h = C.c_void_p(h)
        obj._owned = False
        obj._stream = stream
        obj.device = device
        obj.n_cams, obj.n_lms, obj.n_obs = int(n_cams), int(n_lms), int(n_obs)
        obj.d_p = 9
        obj.n = 9 * obj.n_cams
        return obj

    def close(self):
        if getattr(self, "h", None):
            if getattr(self, "_owned", True):
                lib().ba_free_system(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _new(self, *shape):
        torch = _torch()
        return torch.empty(*shape, dtype=torch.float64, device=self.device)

    def info(self):
        a, b, c, d, e, f = C.c_int32(), C.c_int32(), C.c_int64(), C.c_int64(), C.c_int32(), C.c_int64()
        _check(lib().ba_system_info(self.h, C.byref(a), C.byref(b), C.byref(c), C.byref(d), C.byref(e),
                                    C.byref(f)), "ba_system_info")
        return {"n_cams": a.value, "n_lms": b.value, "n_obs": c.value, "n_tiles": d.value,
                "n_chunks": e.value, "matvec_bytes_fp64": f.value}

    def explicit_schur_info(self):
        """(nonzero 9x9 blocks, bytes of their values, assembly ms) of the explicit S."""
        nb, by, ms = C.c_int64(), C.c_int64(), C.c_double()
        _check(lib().ba_explicit_schur_info(self.h, C.byref(nb), C.byref(by), C.byref(ms)), "ba_explicit_schur_info")
        return {"nnz_blocks": nb.value, "bytes": by.value, "assembly_ms": ms.value}

    def profile(self, on: bool = True, every: int = 1):
        """Event timing of the S product kernel: every `every`-th launch while on."""
        _check(lib().ba_profile_enable(self.h, int(every) if on else 0), "ba_profile_enable")

    def profile_read(self, reset: bool = True):
        ms, n = C.c_double(), C.c_int64()
        _check(lib().ba_profile_read(self.h, C.byref(ms), C.byref(n), int(reset)), "ba_profile_read")
        return ms.value, n.value

    def matvec(self, v, precision="fp64", out=None):
        torch = _torch()
        y = out if out is not None else self._new(self.n)
        _check(lib().ba_schur_matvec(self.h, _dev_ptr(v, torch.float64, self.n, "v"),
                                     _dev_ptr(y, torch.float64, self.n, "y"),
                                     PREC[precision] if isinstance(precision, str) else int(precision)),
               "ba_schur_matvec")
        return y

    def matvec_timed(self, v, reps=50, precision="fp64", out=None):
        """Average ms per S product over `reps` back-to-back launches (ba_schur_matvec_timed)."""
        torch = _torch()
        y = out if out is not None else self._new(self.n)
        ms = C.c_double()
        _check(lib().ba_schur_matvec_timed(self.h, _dev_ptr(v, torch.float64, self.n, "v"),
                                           _dev_ptr(y, torch.float64, self.n, "y"),
                                           PREC[precision] if isinstance(precision, str) else int(precision), int(reps),
                                           C.byref(ms)), "ba_schur_matvec_timed")
        return ms.value

    def matvec_noalloc(self, v, out, precision="fp64"):
        """y = S v through the allocation-free entry point (ba_schur_matvec_noalloc); out is required."""
        torch = _torch()
        _check(lib().ba_schur_matvec_noalloc(self.h, _dev_ptr(v, torch.float64, self.n, "v"),
                                             _dev_ptr(out, torch.float64, self.n, "y"),
                                             PREC[precision] if isinstance(precision, str) else int(precision)),
               "ba_schur_matvec_noalloc")
        return out

    def matmat_grouped(self, N, z, precision="fp64"):
        torch = _torch()
        Y = self._new(int(N), self.n)
        _check(lib().ba_schur_matmat_grouped(self.h, int(N), _dev_ptr(z, torch.float64, self.n, "z"),
                                             _dev_ptr(Y, torch.float64, N * self.n, "Y"),
                                             PREC[precision] if isinstance(precision, str) else int(precision)),
               "ba_schur_matmat_grouped")
        return Y

    def precond(self, r):
        torch = _torch()
        z = self._new(self.n)
        _check(lib().ba_precond_apply(self.h, _dev_ptr(r, torch.float64, self.n, "r"),
                                      _dev_ptr(z, torch.float64, self.n, "z")), "ba_precond_apply")
        return z

    def rhs(self):
        torch = _torch()
        b = self._new(self.n)
        _check(lib().ba_get_rhs(self.h, _dev_ptr(b, torch.float64, self.n, "bt")), "ba_get_rhs")
        return b

    def precond_blocks(self):
        torch = _torch()
        D = self._new(self.n_cams, self.d_p, self.d_p)
        _check(lib().ba_get_precond_blocks(self.h, _dev_ptr(D, torch.float64, self.n_cams * self.d_p * self.d_p, "D")),
               "ba_get_precond_blocks")
        return D

    def update(self, J_p, J_l, r, lam):
        """New values for the same observations (ba_update_system): relinearisation or a new lambda."""
        torch = _torch()
        m = self.n_obs
        _check(lib().ba_update_system(self.h, _dev_ptr(J_p, torch.float64, m * 2 * self.d_p, "J_p"),
                                      _dev_ptr(J_l, torch.float64, m * 6, "J_l"),
                                      _dev_ptr(r, torch.float64, m * 2, "r"), float(lam)), "ba_update_system")

    def prepare_mcg(self, N, precision="fp64"):
        """Lay out MCG's partition, multidirectional-product plan and precision copy (ba_prepare_mcg)."""
        _check(lib().ba_prepare_mcg(self.h, int(N), PREC[precision] if isinstance(precision, str) else int(precision)),
               "ba_prepare_mcg")

    def set_lambda(self, lam):
        """A new damping lambda for the same linearisation (ba_set_lambda), J is not read again."""
        _check(lib().ba_set_lambda(self.h, float(lam)), "ba_set_lambda")

    def back_substitute(self, dxp):
        torch = _torch()
        out = self._new(self.n_lms * 3)
        _check(lib().ba_back_substitute(self.h, _dev_ptr(dxp, torch.float64, self.n, "dxp"),
                                        _dev_ptr(out, torch.float64, self.n_lms * 3, "dxl")),
               "ba_back_substitute")
        return out

    # -- learned low-rank preconditioner -------------------------------------
    def lowrank_features(self):
        torch = _torch()
        F = torch.empty(self.n_cams, 47, dtype=torch.float32, device=self.device)
        _check(lib().ba_lowrank_features(self.h, _dev_ptr(F, torch.float32, self.n_cams * 47, "F")),
               "ba_lowrank_features")
        return F

    def set_lowrank_from_mlp(self, out):
        torch = _torch()
        _check(lib().ba_set_lowrank_from_mlp(self.h, _dev_ptr(out, torch.float32, self.n_cams * 72, "out")),
               "ba_set_lowrank_from_mlp")

    def set_lowrank(self, U):
        torch = _torch()
        p = None if U is None else _dev_ptr(U, torch.float64, self.n * 8, "U")
        _check(lib().ba_set_lowrank_precond(self.h, p), "ba_set_lowrank_precond")

    def get_lowrank(self):
        torch = _torch()
        U = self._new(self.n, 8)
        _check(lib().ba_get_lowrank(self.h, _dev_ptr(U, torch.float64, self.n * 8, "U")), "ba_get_lowrank")
        return U

    def block_scale(self, x, transpose=False):
        torch = _torch()
        y = torch.empty_like(x)
        _check(lib().ba_block_scale(self.h, _dev_ptr(x, torch.float64, self.n, "x"),
                                    _dev_ptr(y, torch.float64, self.n, "y"), int(transpose)), "ba_block_scale")
        return y

    def pcg(self, eps=1e-6, max_iter=1000, x0=None, precision="fp64", trace=False, out=None,
            inner_eps=0.0, max_outer=20, max_inner=1000, precond="block_jacobi"):
        """Algorithm 1.  precision "fp32"/"bf16": FP64 iterative refinement around inner
        solves with reduced-precision S products (inner_eps, max_outer, max_inner)."""
        torch = _torch()
        x = out if out is not None else self._new(self.n)
        o = _opts(eps, max_iter, precision, inner_eps=inner_eps, max_outer=max_outer, max_inner=max_inner,
                  precond=_PRECOND[precond])
        st = _lib.SolveStats()
        tr = _Trace(max(int(max_iter), 1)) if trace else None
        if tr:
            tr.attach(st)
        x0p = _dev_ptr(x0, torch.float64, self.n, "x0") if x0 is not None else None
        _check(lib().ba_pcg_solve(self.h, x0p, _dev_ptr(x, torch.float64, self.n, "x"), C.byref(o),
                                  C.byref(st)), "ba_pcg_solve")
        return x, _stats(st, tr)

    def mcg(self, N, tau, eps=1e-6, max_iter=1000, x0=None, precision="fp64", trace=False,
            max_history_cols=0, out=None, inner_eps=0.0, max_outer=20, max_inner=1000, precond="block_jacobi",
            history_mfma=False, history_fp32=None):
        """Algorithm 2 with N subsets and threshold tau (mixed precision as in pcg)."""
        torch = _torch()
        x = out if out is not None else self._new(self.n)
        o = _opts(eps, max_iter, precision, max_history_cols=max_history_cols, inner_eps=inner_eps,
                  max_outer=max_outer, max_inner=max_inner, precond=_PRECOND[precond], history_mfma=history_mfma,
                  history_fp32=history_fp32)
        st = _lib.SolveStats()
        tr = _Trace(max(int(max_iter), 1)) if trace else None
        if tr:
            tr.attach(st)
        x0p = _dev_ptr(x0, torch.float64, self.n, "x0") if x0 is not None else None
        _check(lib().ba_mcg_solve(self.h, int(N), float(tau), x0p, _dev_ptr(x, torch.float64, self.n, "x"),
                                  C.byref(o), C.byref(st)), "ba_mcg_solve")
        return x, _stats(st, tr)


_PRECOND = {"block_jacobi": 0, "lowrank": 1, 0: 0, 1: 1}


def mlp_forward(params, F, bf16=True, stream=None):
    """MLP outputs (rows x 72, FP32) of the learned preconditioner for features F (rows x 47)."""
    torch = _torch()
    rows = int(F.shape[0])
    out = torch.empty(rows, 72, dtype=torch.float32, device=F.device)
    _check(lib().ba_mlp_forward(_dev_ptr(params, torch.float32, MLP_PARAMS, "params"),
                                _dev_ptr(F, torch.float32, rows * 47, "F"), rows,
                                _dev_ptr(out, torch.float32, rows * 72, "out"), int(bf16), _stream_handle(stream)),
           "ba_mlp_forward")
    return out


def mlp_loss_grad(params, F, W, Sw, stream=None):
    """Probe loss and its gradient with respect to the FP32 parameters (one system)."""
    torch = _torch()
    rows = int(F.shape[0])
    n, P = int(W.shape[0]), int(W.shape[1])
    grad = torch.empty(MLP_PARAMS, dtype=torch.float32, device=F.device)
    loss = C.c_double()
    _check(lib().ba_mlp_loss_grad(_dev_ptr(params, torch.float32, MLP_PARAMS, "params"),
                                  _dev_ptr(F, torch.float32, rows * 47, "F"), rows,
                                  _dev_ptr(W, torch.float64, n * P, "W"), _dev_ptr(Sw, torch.float64, n * P, "Sw"), P,
                                  _dev_ptr(grad, torch.float32, MLP_PARAMS, "grad"), C.byref(loss),
                                  _stream_handle(stream)), "ba_mlp_loss_grad")
    return loss.value, grad


def adam_step(params, grad, m, v, t, lr=1e-3, stream=None):
    torch = _torch()
    _check(lib().ba_adam_step(_dev_ptr(params, torch.float32, MLP_PARAMS, "params"),
                              _dev_ptr(grad, torch.float32, MLP_PARAMS, "grad"),
                              _dev_ptr(m, torch.float32, MLP_PARAMS, "m"), _dev_ptr(v, torch.float32, MLP_PARAMS, "v"),
                              int(t), float(lr), _stream_handle(stream)), "ba_adam_step")


def stream_read_gbs(nbytes: int, reps: int = 10, stream=None) -> float:
    """HBM read rate (GB/s) of a pure stream in the S-product kernel's access pattern."""
    g = C.c_double()
    _check(lib().ba_stream_read_gbs(int(nbytes), int(reps), C.byref(g), _stream_handle(stream)), "ba_stream_read_gbs")
    return g.value


def pinv_sym(A, stream=None):
    """Device pseudo-inverse of a symmetric k x k FP64 matrix; returns (A^+, rank)."""
    torch = _torch()
    k = int(A.shape[0])
    Ap = torch.empty_like(A)
    rank = C.c_int32()
    _check(lib().ba_pinv_sym(k, _dev_ptr(A, torch.float64, k * k, "A"), _dev_ptr(Ap, torch.float64, k * k, "Ap"),
                             C.byref(rank), _stream_handle(stream)), "ba_pinv_sym")
    return Ap, int(rank.value)


def partition(n_cams: int, N: int) -> np.ndarray:
    g = np.empty(int(n_cams), dtype=np.int32)
    _check(lib().ba_partition(int(n_cams), int(N), g.ctypes.data_as(C.POINTER(C.c_int32))), "ba_partition")
    return g


@dataclass
class BatchStats:
    iterations: int
    multi_steps: int
    history_cols: int
    refinement_steps: int
    status: int
    rel_res_recursive: float
    rel_res_true: float
    done_ms: float


class Batch:
    """Independent problems solved together (ba_batch_*): one block-diagonal system,
    Algorithm 2 per problem with all solver state on the device."""

    def __init__(self, problems, device="cuda", stream=None, max_slots=0, max_tiles=0, store_fp32=False,
                 store_bf16=False):
        torch = _torch()
        lams = {float(p.lam) for p in problems}
        if len(lams) != 1:
            raise ValueError("the problems of a batch share one lambda")
        cams = np.array([p.n_cams for p in problems], dtype=np.int32)
        lms = np.array([p.n_lms for p in problems], dtype=np.int64)
        c0 = np.concatenate([[0], np.cumsum(cams)[:-1]])
        l0 = np.concatenate([[0], np.cumsum(lms)[:-1]])
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        obs_cam = t(np.concatenate([p.obs_cam.astype(np.int64) + c for p, c in zip(problems, c0)]), torch.int32)
        obs_lm = t(np.concatenate([p.obs_lm.astype(np.int64) + l for p, l in zip(problems, l0)]), torch.int32)
        J_p = t(np.concatenate([p.J_p for p in problems]), torch.float64)
        J_l = t(np.concatenate([p.J_l for p in problems]), torch.float64)
        r = t(np.concatenate([p.r for p in problems]), torch.float64)
        m = int(obs_cam.numel())
        d = _lib.ProblemDesc()
        d.n_cams, d.n_lms, d.n_obs, d.d_p = int(cams.sum()), int(lms.sum()), m, 9
        d.obs_cam = _dev_ptr(obs_cam, torch.int32, m, "obs_cam")
        d.obs_lm = _dev_ptr(obs_lm, torch.int32, m, "obs_lm")
        d.J_p = _dev_ptr(J_p, torch.float64, m * 18, "J_p")
        d.J_l = _dev_ptr(J_l, torch.float64, m * 6, "J_l")
        d.r = _dev_ptr(r, torch.float64, m * 2, "r")
        d.lam = lams.pop()
        o = _lib.BuildOpts()
        o.store_fp32, o.store_bf16 = int(store_fp32), int(store_bf16)
        o.max_slots, o.max_tiles = int(max_slots), int(max_tiles)
        self._stream = stream if stream is not None else torch.cuda.current_stream()
        self.device = obs_cam.device
        h = C.c_void_p()
        cp = np.ascontiguousarray(cams)
        _check(lib().ba_batch_build(C.byref(d), len(problems), cp.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(o),
                                    _stream_handle(self._stream), C.byref(h)), "ba_batch_build")
        self.h = h
        self.B = len(problems)
        self.cams = cams
        self.row0 = (9 * c0).astype(np.int64)
        self.n = 9 * int(cams.sum())
        self.system = System._view(lib().ba_batch_system(h), d.n_cams, d.n_lms, m, self.device, self._stream)

    def close(self):
        if getattr(self, "h", None):
            lib().ba_batch_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def split(self, v):
        """Per-problem views of a batch vector."""
        return [v[int(a):int(a) + 9 * int(c)] for a, c in zip(self.row0, self.cams)]

    def mcg(self, N, tau, eps=1e-6, max_iter=1000, precision="fp64", graph_window=8, inner_eps=0.0,
            max_outer=20, max_inner=1000, max_history_cols=0, out=None):
        """Algorithm 2 for every problem; returns (x, [BatchStats], elapsed ms, worst status)."""
        torch = _torch()
        x = out if out is not None else torch.empty(self.n, dtype=torch.float64, device=self.device)
        o = _opts(eps, max_iter, precision, max_history_cols=max_history_cols, inner_eps=inner_eps,
                  max_outer=max_outer, max_inner=max_inner)
        st = (_lib.BatchStats * self.B)()
        ms = C.c_double()
        rc = _check(lib().ba_batch_mcg_solve(self.h, int(N), float(tau), _dev_ptr(x, torch.float64, self.n, "x"),
                                             C.byref(o), int(graph_window), st, C.byref(ms)), "ba_batch_mcg_solve")
        stats = [BatchStats(s.iterations, s.multi_steps, s.history_cols, s.refinement_steps, s.status,
                            s.rel_res_recursive, s.rel_res_true, s.done_ms) for s in st]
        return x, stats, ms.value, rc



# ------------------------------------------------------------------ LM outer loop

@dataclass
class LMStats:
    iterations: int
    accepted: int
    status: int
    solver_iterations: int
    cost0: float
    cost: float
    t_total_ms: float
    t_solve_ms: float
    t_linearize_ms: float
    trace_lambda: np.ndarray
    trace_cost: np.ndarray
    trace_accepted: np.ndarray
    trace_solver_iterations: np.ndarray
    trace_solve_ms: np.ndarray


class Scene:
    """Observations of a bundle-adjustment scene on one device (ba_scene_desc): the
    nine-parameter camera model, its residuals and Jacobians, and the LM loop of
    Sec. 4.1.  Cameras are [n_cams, 15] (R row-major, t, f, k1, k2), landmarks [n_lms, 3]."""

    def __init__(self, n_cams, n_lms, obs_cam, obs_lm, u_obs, stream=None):
        torch = _torch()
        self.n_cams, self.n_lms, self.n_obs = int(n_cams), int(n_lms), int(obs_cam.numel())
        m = self.n_obs
        self._keep = (obs_cam, obs_lm, u_obs)
        d = _lib.SceneDesc()
        d.n_cams, d.n_lms, d.n_obs = self.n_cams, self.n_lms, m
        d.obs_cam = _dev_ptr(obs_cam, torch.int32, m, "obs_cam")
        d.obs_lm = _dev_ptr(obs_lm, torch.int32, m, "obs_lm")
        d.u_obs = _dev_ptr(u_obs, torch.float64, m * 2, "u_obs")
        self.desc = d
        self.device = obs_cam.device
        self._stream = stream if stream is not None else torch.cuda.current_stream()

    @classmethod
    def from_problem(cls, p, device="cuda", **kw):
        """The scene of a synthetic problem that carries its state (cams, points, u_obs);
        returns (scene, cams [n_cams, 15], X [n_lms, 3]) on the device."""
        torch = _torch()
        t = lambda a, dt: torch.from_numpy(np.ascontiguousarray(a)).to(device=device, dtype=dt)
        R = np.asarray(p.cams["R"]).reshape(p.n_cams, 9)
        cams = np.concatenate([R, p.cams["t"], p.cams["f"][:, None], p.cams["k1"][:, None], p.cams["k2"][:, None]], 1)
        sc = cls(p.n_cams, p.n_lms, t(p.obs_cam, torch.int32), t(p.obs_lm, torch.int32), t(p.u_obs, torch.float64), **kw)
        return sc, t(cams, torch.float64), t(p.points, torch.float64)

    def _state(self, cams, X):
        torch = _torch()
        return (_dev_ptr(cams, torch.float64, self.n_cams * 15, "cams"),
                _dev_ptr(X, torch.float64, self.n_lms * 3, "X"))

    def project(self, cams, X, jacobians=True):
        """(r [m, 2], J_p [m, 2, 9], J_l [m, 2, 3], F) at the state; J_* None without jacobians."""
        torch = _torch()
        m = self.n_obs
        r = torch.empty(m, 2, dtype=torch.float64, device=self.device)
        Jp = torch.empty(m, 2, 9, dtype=torch.float64, device=self.device) if jacobians else None
        Jl = torch.empty(m, 2, 3, dtype=torch.float64, device=self.device) if jacobians else None
        F = C.c_double()
        pc, px = self._state(cams, X)
        _check(lib().ba_project(C.byref(self.desc), pc, px, C.c_void_p(Jp.data_ptr()) if jacobians else None,
                                C.c_void_p(Jl.data_ptr()) if jacobians else None, C.c_void_p(r.data_ptr()),
                                C.byref(F), _stream_handle(self._stream)), "ba_project")
        return r, Jp, Jl, F.value

    def apply_step(self, cams, X, dxp, dxl):
        """The state moved by (dxp, dxl) (ba_apply_step)."""
        torch = _torch()
        co, Xo = torch.empty_like(cams), torch.empty_like(X)
        pc, px = self._state(cams, X)
        _check(lib().ba_apply_step(self.n_cams, self.n_lms, pc, px,
                                   _dev_ptr(dxp, torch.float64, 9 * self.n_cams, "dxp"),
                                   _dev_ptr(dxl, torch.float64, 3 * self.n_lms, "dxl"),
                                   C.c_void_p(co.data_ptr()), C.c_void_p(Xo.data_ptr()),
                                   _stream_handle(self._stream)), "ba_apply_step")
        return co, Xo

    def lm(self, cams, X, solver="pcg", N=1, tau=3.3, max_iter=25, lambda0=1e-4, ftol=1e-6, lambda_factor=10.0,
           eps=1e-6, solver_max_iter=1000, precision="fp64", max_slots=0, max_tiles=0, explicit_schur=False):
        """ba_lm_solve on copies of (cams, X); returns (cams, X, LMStats)."""
        cams, X = cams.clone(), X.clone()
        o = _lib.LMOpts()
        lib().ba_default_lm_opts(C.byref(o))
        o.max_iter, o.solver, o.n_groups, o.tau = int(max_iter), {"pcg": 0, "mcg": 1}[solver], int(N), float(tau)
        o.lambda0, o.ftol, o.lambda_factor = float(lambda0), float(ftol), float(lambda_factor)
        o.solve = _opts(eps, solver_max_iter, precision)
        o.build.max_slots, o.build.max_tiles = int(max_slots), int(max_tiles)
        o.build.store_fp32 = int(precision == "fp32")
        o.build.store_bf16 = int(precision == "bf16")
        o.build.explicit_schur = int(explicit_schur)
        cap = max(int(max_iter), 1)
        tl, tc, ts = np.full(cap, np.nan), np.full(cap, np.nan), np.full(cap, np.nan)
        ta, ti = np.zeros(cap, np.int32), np.zeros(cap, np.int32)
        st = _lib.LMStats()
        st.trace_cap = cap
        dp = lambda a: a.ctypes.data_as(C.POINTER(C.c_double))
        ip = lambda a: a.ctypes.data_as(C.POINTER(C.c_int32))
        st.trace_lambda, st.trace_cost, st.trace_solve_ms = dp(tl), dp(tc), dp(ts)
        st.trace_accepted, st.trace_solver_iterations = ip(ta), ip(ti)
        pc, px = self._state(cams, X)
        _check(lib().ba_lm_solve(C.byref(self.desc), pc, px, C.byref(o), _stream_handle(self._stream), C.byref(st)),
               "ba_lm_solve")
        n = st.iterations
        return cams, X, LMStats(st.iterations, st.accepted, st.status, st.solver_iterations, st.cost0, st.cost,
                                st.t_total_ms, st.t_solve_ms, st.t_linearize_ms, tl[:n].copy(), tc[:n].copy(),
                                ta[:n].copy(), ti[:n].copy(), ts[:n].copy())
