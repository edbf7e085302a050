"""FP64 oracle of the Levenberg-Marquardt outer loop around the reduced camera system.

TEST INFRASTRUCTURE (see oracle/__init__.py).  Plain NumPy, written from the
definitions below; shares nothing with the HIP kernels.  The linear solves use the
oracle's own reduced camera system (``oracle.System``) and its Algorithms 1 and 2.

State (Sec. 3.1, d_p = 9: extrinsics and intrinsics of every pose).  Camera c is
15 numbers, cams[c] = (R row-major (9), t (3), f, k1, k2); landmark l is X[l] (3).
Projection of landmark l in camera c (pinhole with two radial distortion terms):
    P = R X + t,  p = (P_x / P_z, P_y / P_z),  rho2 = p . p,
    s = 1 + k1 rho2 + k2 rho2^2,  u = f s p,
and the residual of observation o is r_o = u - u_obs[o] (two rows); the objective
is F = sum_o |r_o|^2 (eq. (1)).

Step (the 9 pose coordinates of Delta x_p, then the 3 of Delta x_l per landmark):
    R <- exp([w]x) R,  t <- exp([w]x) t + dt,  (f, k1, k2) += (df, dk1, dk2),
    X <- X + dX,
with (w, dt, df, dk1, dk2) = Delta x_p of the camera.  The rotation update is a
left increment, so P moves by w x P + dt to first order and the pose Jacobian is
    dr/dw = -A [P]x,  dr/dt = A,  dr/df = s p,  dr/dk1 = f rho2 p,  dr/dk2 = f rho2^2 p,
    dr/dX = A R,  with A = du/dP = f (s I + (2 k1 + 4 k2 rho2) p p^T) [[1/z, 0, -x/z^2], [0, 1/z, -y/z^2]].

LM loop (Sec. 4.1): lambda starts at 1e-4; every iteration solves the damped normal
equation (eq. (6)-(8), D^T D = diag(J^T J)) through the Schur complement (eq. (13)-(16))
with PCG or MCG, evaluates F at the moved state, accepts the move if F decreases
(lambda / 10) and keeps the state otherwise (lambda x 10).  It stops after 25
iterations, or after an iteration whose relative change |F - F_new| / F is below the
relative function tolerance 1e-6 (the paper gives the tolerance, not its exact form:
this reading counts accepted and rejected iterations alike), or when F is zero.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from types import SimpleNamespace
from typing import List, Optional, Tuple

import numpy as np

from . import MAXITER, OK, System

CAM_WIDTH = 15


def rotation_exp(w: np.ndarray) -> np.ndarray:
    """exp([w]x) by Rodrigues' formula, one 3 x 3 matrix per row of w (Taylor terms
    below 1e-6 rad, where the closed form loses digits)."""
    w = np.atleast_2d(np.asarray(w, dtype=np.float64))
    out = np.empty((w.shape[0], 3, 3))
    for i, v in enumerate(w):
        th = float(np.sqrt(v @ v))
        K = np.array([[0.0, -v[2], v[1]], [v[2], 0.0, -v[0]], [-v[1], v[0], 0.0]])
        if th < 1e-6:
            a = 1.0 - th * th / 6.0
            b = 0.5 - th * th / 24.0
        else:
            a = np.sin(th) / th
            b = (1.0 - np.cos(th)) / (th * th)
        out[i] = np.eye(3) + a * K + b * (K @ K)
    return out


def _split(cams: np.ndarray):
    c = np.asarray(cams, dtype=np.float64).reshape(-1, CAM_WIDTH)
    return c[:, 0:9].reshape(-1, 3, 3), c[:, 9:12], c[:, 12], c[:, 13], c[:, 14]


def project(cams: np.ndarray, X: np.ndarray, cam: np.ndarray, lm: np.ndarray) -> np.ndarray:
    """Pixel position u [m, 2] of every observation."""
    R, t, f, k1, k2 = _split(cams)
    cam = np.asarray(cam, dtype=np.int64)
    lm = np.asarray(lm, dtype=np.int64)
    P = np.einsum("mij,mj->mi", R[cam], X[lm]) + t[cam]
    p = P[:, 0:2] / P[:, 2:3]
    rho2 = (p * p).sum(1)
    s = 1.0 + k1[cam] * rho2 + k2[cam] * rho2 * rho2
    return (f[cam] * s)[:, None] * p


def residuals(cams, X, cam, lm, u_obs) -> np.ndarray:
    """r_o = u_o - u_obs[o], shape [m, 2]."""
    return project(cams, X, cam, lm) - np.asarray(u_obs, dtype=np.float64)


def cost(r: np.ndarray) -> float:
    """F = sum of squared residuals (eq. (1))."""
    r = np.asarray(r, dtype=np.float64).ravel()
    return float(r @ r)


def jacobians(cams, X, cam, lm) -> Tuple[np.ndarray, np.ndarray]:
    """(J_p [m, 2, 9], J_l [m, 2, 3]) of the residuals in the step coordinates above,
    one observation at a time."""
    R, t, f, k1, k2 = _split(cams)
    m = len(cam)
    Jp = np.empty((m, 2, 9))
    Jl = np.empty((m, 2, 3))
    for o in range(m):
        c, l = int(cam[o]), int(lm[o])
        P = R[c] @ X[l] + t[c]
        x, y, z = P
        p = np.array([x / z, y / z])
        rho2 = p @ p
        s = 1.0 + k1[c] * rho2 + k2[c] * rho2 * rho2
        dudp = f[c] * (s * np.eye(2) + (2.0 * k1[c] + 4.0 * k2[c] * rho2) * np.outer(p, p))
        dpdP = np.array([[1.0 / z, 0.0, -x / (z * z)], [0.0, 1.0 / z, -y / (z * z)]])
        A = dudp @ dpdP
        Px = np.array([[0.0, -z, y], [z, 0.0, -x], [-y, x, 0.0]])
        Jp[o, :, 0:3] = -A @ Px
        Jp[o, :, 3:6] = A
        Jp[o, :, 6] = s * p
        Jp[o, :, 7] = f[c] * rho2 * p
        Jp[o, :, 8] = f[c] * rho2 * rho2 * p
        Jl[o] = A @ R[c]
    return Jp, Jl


def apply_step(cams, X, dxp, dxl) -> Tuple[np.ndarray, np.ndarray]:
    """The state moved by (Delta x_p, Delta x_l) as defined above."""
    R, t, f, k1, k2 = _split(cams)
    d = np.asarray(dxp, dtype=np.float64).reshape(-1, 9)
    E = rotation_exp(d[:, 0:3])
    out = np.empty((R.shape[0], CAM_WIDTH))
    out[:, 0:9] = np.einsum("nij,njk->nik", E, R).reshape(-1, 9)
    out[:, 9:12] = np.einsum("nij,nj->ni", E, t) + d[:, 3:6]
    out[:, 12] = f + d[:, 6]
    out[:, 13] = k1 + d[:, 7]
    out[:, 14] = k2 + d[:, 8]
    return out, np.asarray(X, dtype=np.float64) + np.asarray(dxl, dtype=np.float64).reshape(-1, 3)


@dataclass
class LMIter:
    lam: float              # damping used by this iteration's solve
    cost_before: float      # F at the current state
    cost_new: float         # F at the moved state
    accepted: bool
    solver_iterations: int
    solver_status: int


@dataclass
class LMResult:
    cams: np.ndarray
    X: np.ndarray
    cost0: float
    cost: float
    iters: List[LMIter] = field(default_factory=list)
    status: int = OK


def linearize(cams, X, cam, lm, u_obs, lam):
    """The linearised problem of the state (the input of ``oracle.System``)."""
    Jp, Jl = jacobians(cams, X, cam, lm)
    return SimpleNamespace(n_cams=cams.shape[0], n_lms=X.shape[0], obs_cam=np.asarray(cam, np.int32),
                           obs_lm=np.asarray(lm, np.int32), J_p=Jp, J_l=Jl,
                           r=residuals(cams, X, cam, lm, u_obs), lam=lam)


def lm(cams, X, cam, lm_idx, u_obs, solver: str = "pcg", N: int = 1, tau: float = 3.3, eps: float = 1e-6,
       imax: int = 1000, max_iter: int = 25, lam0: float = 1e-4, ftol: float = 1e-6,
       factor: float = 10.0) -> LMResult:
    """The LM loop described in the module docstring; returns the final state and the
    per-iteration record."""
    cams = np.array(cams, dtype=np.float64).reshape(-1, CAM_WIDTH)
    X = np.array(X, dtype=np.float64).reshape(-1, 3)
    lam = float(lam0)
    prob = linearize(cams, X, cam, lm_idx, u_obs, lam)
    F = cost(prob.r)
    res = LMResult(cams=cams, X=X, cost0=F, cost=F)
    for _ in range(max_iter):
        if F == 0.0:
            break
        prob.lam = lam
        sysm = System(prob)
        if solver == "pcg":
            dxp, st = sysm.pcg(eps=eps, imax=imax)
        else:
            dxp, st = sysm.mcg(N, tau, eps=eps, imax=imax)
        if st.status not in (OK, MAXITER):
            res.status = st.status
            break
        dxl = sysm.back_substitute(dxp)
        c_new, X_new = apply_step(cams, X, dxp, dxl)
        F_new = cost(residuals(c_new, X_new, cam, lm_idx, u_obs))
        accepted = F_new < F
        res.iters.append(LMIter(lam, F, F_new, accepted, st.iterations, st.status))
        change = abs(F - F_new) / F
        if accepted:
            cams, X, F = c_new, X_new, F_new
            lam /= factor
            prob = linearize(cams, X, cam, lm_idx, u_obs, lam)
        else:
            lam *= factor
        if change < ftol:
            break
    res.cams, res.X, res.cost = cams, X, F
    return res
