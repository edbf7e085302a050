"""Reference for the reduced-precision S products (test infrastructure, FP64 NumPy).

Only the tests may import this module; the product path never does.

The mixed-precision solves (an addition to the paper's method: FP32 or BF16 products under
FP64 iterative refinement) apply an operator S^ that differs from S in one defined way: the
per-observation Jacobian blocks J_p and J_l are the stored ones, rounded to FP32 (or to FP32
and then to BF16, each to nearest even), while V_lambda^-1 and the damping lambda D_p^T D_p
are those of the FP64 system.  ``schur_matvec_stored`` forms S^ v in FP64 from those inputs,
following eq. (14) factor by factor (Sec. 3.1):

    e_o = J_p,o v_c(o),   g_l = sum_{o in l} J_l,o^T e_o,   h_l = V_l^-1 g_l,
    y_c = sum_{o in c} J_p,o^T (e_o - J_l,o h_l(o)) + lambda diag(U_c) v_c,

and alongside it the same sums with every factor replaced by its absolute value (and the
difference e - J_l h by the sum |e| + |J_l||h|).  A product evaluated in precision u with
FP64 accumulation differs from S^ v, per element, by at most a modest multiple of u times
that absolute sum (the standard forward error bound of a sum of products), which is how the
GPU parity tests compare the reduced products element by element.
"""
from __future__ import annotations

import numpy as np


def stored(J: np.ndarray, precision: str) -> np.ndarray:
    """The FP64 values of J as stored for the reduced products: "fp32" rounds each entry to
    the nearest FP32 value (ties to even); "bf16" then keeps the 8 leading significand bits
    of that FP32 value, again to nearest, ties to even (BF16: 1 sign, 8 exponent, 7 stored
    fraction bits).  Finite inputs only."""
    f = np.asarray(J, dtype=np.float64).astype(np.float32)
    if precision == "fp32":
        return f.astype(np.float64)
    if precision != "bf16":
        raise ValueError(precision)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    u = ((u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)) << np.uint64(16)
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def lambda_diag(U_lambda_blocks: np.ndarray, lam: float) -> np.ndarray:
    """lambda diag(U_c) per pose (n values) from the damped blocks U_lambda = U + lambda diag(U)
    (eq. (6), (9): D_p^T D_p = diag(J_p^T J_p))."""
    d = np.einsum("cii->ci", U_lambda_blocks)
    return (d * (lam / (1.0 + lam))).reshape(-1)


def schur_matvec_stored(obs_cam, obs_lm, n_cams, n_lms, Jp, Jl, Vinv, lam_diag, v):
    """(S^ v, |S^| |v|): the S product with the given Jacobian blocks (m x 2 x d_p and
    m x 2 x 3), V_lambda^-1 blocks (n_l x 3 x 3) and damping diagonal (n), and the
    element-wise sum of the absolute values of its terms."""
    cam = np.asarray(obs_cam, dtype=np.int64)
    lm = np.asarray(obs_lm, dtype=np.int64)
    dp = Jp.shape[-1]
    V = v.reshape(n_cams, dp)
    Va = np.abs(V)

    def landmark_sum(t):   # [m, 3] -> [n_l, 3]
        return np.stack([np.bincount(lm, weights=t[:, k], minlength=n_lms) for k in range(3)], axis=1)

    def camera_sum(t):     # [m, dp] -> [n_cams, dp]
        return np.stack([np.bincount(cam, weights=t[:, k], minlength=n_cams) for k in range(dp)], axis=1)

    e = np.einsum("mij,mj->mi", Jp, V[cam])
    ea = np.einsum("mij,mj->mi", np.abs(Jp), Va[cam])
    g = landmark_sum(np.einsum("mij,mi->mj", Jl, e))
    ga = landmark_sum(np.einsum("mij,mi->mj", np.abs(Jl), ea))
    h = np.einsum("lij,lj->li", Vinv, g)
    ha = np.einsum("lij,lj->li", np.abs(Vinv), ga)
    f = e - np.einsum("mij,mj->mi", Jl, h[lm])
    fa = ea + np.einsum("mij,mj->mi", np.abs(Jl), ha[lm])
    y = camera_sum(np.einsum("mij,mi->mj", Jp, f)) + lam_diag.reshape(n_cams, dp) * V
    ya = camera_sum(np.einsum("mij,mi->mj", np.abs(Jp), fa)) + np.abs(lam_diag).reshape(n_cams, dp) * Va
    return y.reshape(-1), ya.reshape(-1)
