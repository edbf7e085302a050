"""FP64 CPU oracle (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The product path (``paper_2110_04015_amd``) never imports it and
shares no code with it.

Thin ctypes wrapper around ``liboracle.so`` (plain C, OpenMP), built from
``ba_oracle.c`` by ``oracle.build_lib()`` or the repository's ``build()``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ba_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, MAXITER = 0, 1
ERR_INVALID, ERR_NONFINITE, ERR_NOT_SPD, ERR_BREAKDOWN = -1, -2, -3, -4


def build_lib(extra_flags=()) -> str:
    """Compile ba_oracle.c into liboracle.so with gcc (FP64, no fast-math)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-Wall", *extra_flags,
           "-o", _LIB, _SRC, "-lm"]
    subprocess.check_call(cmd)
    return _LIB


def build_variant(out_path: str, defines=()) -> str:
    """Compile a variant of the oracle with extra -D flags (used by mutation tests)."""
    cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", *[f"-D{d}" for d in defines],
           "-o", out_path, _SRC, "-lm"]
    subprocess.check_call(cmd)
    return out_path


class _Stats(C.Structure):
    _fields_ = [("iterations", C.c_int), ("multi_steps", C.c_int), ("history_cols", C.c_int),
                ("status", C.c_int), ("rel_res_recursive", C.c_double),
                ("rel_res_true", C.c_double)]


@dataclass
class Stats:
    iterations: int
    multi_steps: int
    history_cols: int
    status: int
    rel_res_recursive: float
    rel_res_true: float


_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int)


def _ptr(a: Optional[np.ndarray], t=_dp):
    if a is None:
        return None
    return a.ctypes.data_as(t)


def load(path: Optional[str] = None) -> C.CDLL:
    path = path or _LIB
    if not os.path.exists(path):
        build_lib()
    lib = C.CDLL(path)
    lib.or_build.restype = C.c_void_p
    lib.or_build.argtypes = [C.c_int, C.c_int, C.c_int64, _ip, _ip, _dp, _dp, _dp, C.c_double, _ip]
    lib.or_build_dp.restype = C.c_void_p
    lib.or_build_dp.argtypes = [C.c_int, C.c_int, C.c_int64, _ip, _ip, _dp, _dp, _dp, C.c_double, C.c_int, _ip]
    lib.or_dp.argtypes = [C.c_void_p]
    lib.or_free.argtypes = [C.c_void_p]
    lib.or_n.argtypes = [C.c_void_p]
    for name in ("or_get_rhs", "or_get_U", "or_get_Vinv", "or_get_Dblocks"):
        getattr(lib, name).argtypes = [C.c_void_p, _dp]
    lib.or_get_bp_bl.argtypes = [C.c_void_p, _dp, _dp]
    lib.or_schur_matvec.argtypes = [C.c_void_p, _dp, _dp]
    lib.or_precond_apply.argtypes = [C.c_void_p, _dp, _dp]
    lib.or_back_substitute.argtypes = [C.c_void_p, _dp, _dp]
    lib.or_pinv.argtypes = [C.c_int, _dp, _dp, _dp]
    lib.or_pinv.restype = C.c_int
    lib.or_partition.argtypes = [C.c_int, C.c_int, _ip]
    lib.or_pcg.argtypes = [C.c_void_p, _dp, _dp, C.c_double, C.c_int, C.POINTER(_Stats), _dp]
    lib.or_pcg.restype = C.c_int
    lib.or_mcg.argtypes = [C.c_void_p, C.c_int, C.c_double, _dp, _dp, C.c_double, C.c_int,
                           C.c_int, C.POINTER(_Stats), _dp, _dp, C.c_int64]
    lib.or_mcg.restype = C.c_int
    lib.or_num_threads.restype = C.c_int
    lib.or_set_lowrank.argtypes = [C.c_void_p, _dp, C.c_int]
    lib.or_set_lowrank.restype = C.c_int
    return lib


_default = None


def lib() -> C.CDLL:
    global _default
    if _default is None:
        _default = load()
    return _default


class OracleError(RuntimeError):
    def __init__(self, status: int):
        super().__init__(f"oracle status {status}")
        self.status = status


class System:
    """The oracle's damped normal equation and reduced camera system for one problem;
    the pose dimension d_p (6 or 9, Sec. 3.1) is the last axis of J_p."""

    def __init__(self, problem, lam: Optional[float] = None, libobj: Optional[C.CDLL] = None):
        self.lib = libobj or lib()
        p = problem
        self.n_cams, self.n_lms = p.n_cams, p.n_lms
        self.dp = int(np.shape(p.J_p)[-1])
        self.n = self.dp * p.n_cams
        self._keep = [np.ascontiguousarray(p.obs_cam, dtype=np.int32),
                      np.ascontiguousarray(p.obs_lm, dtype=np.int32),
                      np.ascontiguousarray(p.J_p, dtype=np.float64),
                      np.ascontiguousarray(p.J_l, dtype=np.float64),
                      np.ascontiguousarray(p.r, dtype=np.float64)]
        cam, lm, Jp, Jl, r = self._keep
        st = C.c_int(0)
        self.h = self.lib.or_build_dp(p.n_cams, p.n_lms, cam.shape[0], _ptr(cam, _ip), _ptr(lm, _ip),
                                      _ptr(Jp), _ptr(Jl), _ptr(r),
                                      float(p.lam if lam is None else lam), self.dp, C.byref(st))
        self._keep = None
        if not self.h:
            raise OracleError(st.value)

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.or_free(h)
            self.h = None

    # -- blocks ----------------------------------------------------------
    def rhs(self) -> np.ndarray:
        out = np.empty(self.n)
        self.lib.or_get_rhs(self.h, _ptr(out))
        return out

    def bp_bl(self):
        bp, bl = np.empty(self.n), np.empty(3 * self.n_lms)
        self.lib.or_get_bp_bl(self.h, _ptr(bp), _ptr(bl))
        return bp, bl

    def U_blocks(self) -> np.ndarray:
        out = np.empty((self.n_cams, self.dp, self.dp))
        self.lib.or_get_U(self.h, _ptr(out))
        return out

    def Vinv_blocks(self) -> np.ndarray:
        out = np.empty((self.n_lms, 3, 3))
        self.lib.or_get_Vinv(self.h, _ptr(out))
        return out

    def D_blocks(self) -> np.ndarray:
        out = np.empty((self.n_cams, self.dp, self.dp))
        self.lib.or_get_Dblocks(self.h, _ptr(out))
        return out

    def set_lowrank(self, U: Optional[np.ndarray]):
        """Use M^-1 = D^-1 + U U^T (U: n x rank) in precond/pcg/mcg; None restores block Jacobi."""
        if U is None:
            self.lib.or_set_lowrank(self.h, None, 0)
            return
        U = np.ascontiguousarray(U, dtype=np.float64)
        st = self.lib.or_set_lowrank(self.h, _ptr(U), int(U.shape[1]))
        if st != OK:
            raise OracleError(st)

    # -- operators -------------------------------------------------------
    def matvec(self, v: np.ndarray) -> np.ndarray:
        v = np.ascontiguousarray(v, dtype=np.float64)
        y = np.empty(self.n)
        self.lib.or_schur_matvec(self.h, _ptr(v), _ptr(y))
        return y

    def precond(self, r: np.ndarray) -> np.ndarray:
        r = np.ascontiguousarray(r, dtype=np.float64)
        z = np.empty(self.n)
        self.lib.or_precond_apply(self.h, _ptr(r), _ptr(z))
        return z

    def back_substitute(self, dxp: np.ndarray) -> np.ndarray:
        dxp = np.ascontiguousarray(dxp, dtype=np.float64)
        out = np.empty(3 * self.n_lms)
        self.lib.or_back_substitute(self.h, _ptr(dxp), _ptr(out))
        return out

    def dense_S(self) -> np.ndarray:
        """S column by column through the operator (tiny problems only)."""
        n = self.n
        S = np.empty((n, n))
        e = np.zeros(n)
        for j in range(n):
            e[:] = 0.0
            e[j] = 1.0
            S[:, j] = self.matvec(e)
        return S

    # -- solvers ---------------------------------------------------------
    def pcg(self, eps=1e-6, imax=1000, x0=None, trace=False):
        x = np.empty(self.n)
        st = _Stats()
        tr = np.full(max(imax, 1), np.nan) if trace else None
        x0c = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        self.lib.or_pcg(self.h, _ptr(x0c), _ptr(x), float(eps), int(imax), C.byref(st), _ptr(tr))
        s = Stats(st.iterations, st.multi_steps, st.history_cols, st.status,
                  st.rel_res_recursive, st.rel_res_true)
        if trace:
            return x, s, tr[:s.iterations]
        return x, s

    def mcg(self, N, tau, eps=1e-6, imax=1000, x0=None, q_mode=0, trace=False, history=False,
            history_cap=None):
        x = np.empty(self.n)
        st = _Stats()
        tr = np.full((max(imax, 1), 3), np.nan) if trace else None
        cap = 0
        Pout = None
        if history:
            cap = history_cap or (1 + imax * N)
            Pout = np.zeros((cap, self.n))
        x0c = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
        self.lib.or_mcg(self.h, int(N), float(tau), _ptr(x0c), _ptr(x), float(eps), int(imax),
                        int(q_mode), C.byref(st), _ptr(tr), _ptr(Pout), C.c_int64(cap))
        s = Stats(st.iterations, st.multi_steps, st.history_cols, st.status,
                  st.rel_res_recursive, st.rel_res_true)
        out = [x, s]
        if trace:
            out.append(tr[:s.iterations])
        if history:
            out.append(Pout[:min(cap, s.history_cols)].T.copy())
        return tuple(out)


def pinv(A: np.ndarray):
    """Symmetric pseudo-inverse (cyclic Jacobi eigendecomposition); returns (A^+, rank, eigs)."""
    A = np.ascontiguousarray(A, dtype=np.float64)
    k = A.shape[0]
    out = np.empty((k, k))
    eig = np.empty(k)
    rank = lib().or_pinv(k, _ptr(A), _ptr(out), _ptr(eig))
    return out, rank, eig


def partition(n_cams: int, N: int) -> np.ndarray:
    g = np.empty(n_cams, dtype=np.int32)
    lib().or_partition(int(n_cams), int(N), _ptr(g, _ip))
    return g


def num_threads() -> int:
    return int(lib().or_num_threads())
