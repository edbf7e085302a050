"""Pins of the reduced-precision product reference (oracle/reduced.py).

The stored-precision rounding is pinned to values fixed by the FP32 and BF16 formats (ties
to even, and the two-step FP64 -> FP32 -> BF16 rounding); the product to a dense Schur
complement assembled observation by observation from the same Jacobian blocks (with V^-1
and the damping of the FP64 system), and to the C oracle's explicit-W product; the absolute
sum to the triangle inequality and to the case where no term cancels.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import reduced as R


def test_stored_rounding_values():
    x = np.array([1.0, 1 + 2.0 ** -24, 1 + 3 * 2.0 ** -24, 1.0 / 3.0, -2.5, 0.0])
    # FP32 ties go to the even significand: 1 + 2^-24 -> 1, 1 + 3 2^-24 -> 1 + 2^-22
    assert R.stored(x, "fp32").tolist() == [1.0, 1.0, 1 + 2.0 ** -22, 0.3333333432674408, -2.5, 0.0]
    y = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1.0 / 3.0, -2.5, 1 + 2.0 ** -8 + 2.0 ** -40, 1 + 2.0 ** -8 + 2.0 ** -20])
    # BF16 keeps 7 fraction bits: ties to even (1 + 2^-8 -> 1, 1 + 3 2^-8 -> 1 + 2^-6), 1/3 ->
    # 0x3EAB = 0.333984375; a value whose FP32 rounding lands on a BF16 tie rounds from there
    # (1 + 2^-8 + 2^-40 -> FP32 1 + 2^-8 -> 1), one above the tie in FP32 rounds up
    assert R.stored(y, "bf16").tolist() == [1.0, 1 + 2.0 ** -6, 0.333984375, -2.5, 1.0, 1 + 2.0 ** -7]
    with pytest.raises(ValueError):
        R.stored(x, "fp16")


def _dense_parts(p, Jp, Jl):
    """Dense J_p^T J_p, J_p^T J_l and J_l^T J_l from the given blocks, observation by observation."""
    m, dp, n, nl = p.n_obs, p.d_p, p.n, p.n_lms
    Jc = np.zeros((2 * m, n))
    Jm = np.zeros((2 * m, 3 * nl))
    for o in range(m):
        c, l = int(p.obs_cam[o]), int(p.obs_lm[o])
        Jc[2 * o:2 * o + 2, dp * c:dp * c + dp] = Jp[o]
        Jm[2 * o:2 * o + 2, 3 * l:3 * l + 3] = Jl[o]
    return Jc.T @ Jc, Jc.T @ Jm, Jm.T @ Jm


@pytest.mark.parametrize("dp", [9, 6])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16"])
def test_product_matches_dense_schur(dp, prec):
    """S^ = Jh_p^T Jh_p + lam diag(J_p^T J_p) - Jh_p^T Jh_l V^-1 Jh_l^T Jh_p, with V^-1 the
    inverse of the damped J_l^T J_l blocks of the unrounded J (dense, from scratch)."""
    p = synth.tiny(n_cams=5, n_lms=40, seed=2, c_hi=5)
    if dp == 6:
        p = synth.extrinsics_only(p)
    Jp = p.J_p if prec == "fp64" else R.stored(p.J_p, prec)
    Jl = p.J_l if prec == "fp64" else R.stored(p.J_l, prec)
    App, _, _ = _dense_parts(p, p.J_p, p.J_l)
    _, _, All = _dense_parts(p, p.J_p, p.J_l)
    Vinv = np.zeros((p.n_lms, 3, 3))
    for l in range(p.n_lms):
        B = All[3 * l:3 * l + 3, 3 * l:3 * l + 3]
        Vinv[l] = np.linalg.inv(B + p.lam * np.diag(np.diag(B)))
    Hpp, Hpl, _ = _dense_parts(p, Jp, Jl)
    Vd = np.zeros((3 * p.n_lms, 3 * p.n_lms))
    for l in range(p.n_lms):
        Vd[3 * l:3 * l + 3, 3 * l:3 * l + 3] = Vinv[l]
    lamd = p.lam * np.diag(App)
    S = Hpp + np.diag(lamd) - Hpl @ Vd @ Hpl.T
    v = np.random.default_rng(5).standard_normal(p.n)
    y, ya = R.schur_matvec_stored(p.obs_cam, p.obs_lm, p.n_cams, p.n_lms, Jp, Jl, Vinv, lamd, v)
    assert np.abs(y - S @ v).max() <= 1e-12 * np.abs(S @ v).max()
    assert np.all(ya >= np.abs(y) * (1 - 1e-12))
    # with the oracle's own V^-1 and damping (read from the C oracle) the same product
    o = oracle.System(p)
    y2, _ = R.schur_matvec_stored(p.obs_cam, p.obs_lm, p.n_cams, p.n_lms, Jp, Jl, o.Vinv_blocks(),
                                  R.lambda_diag(o.U_blocks(), p.lam), v)
    assert np.abs(y2 - y).max() <= 1e-12 * np.abs(y).max()
    if prec == "fp64":
        assert np.abs(y2 - o.matvec(v)).max() <= 1e-12 * np.abs(y).max()


def test_product_matches_c_oracle_at_size():
    p = synth.config0(seed=1)
    o = oracle.System(p)
    v = np.random.default_rng(6).standard_normal(o.n)
    y, ya = R.schur_matvec_stored(p.obs_cam, p.obs_lm, p.n_cams, p.n_lms, p.J_p, p.J_l, o.Vinv_blocks(),
                                  R.lambda_diag(o.U_blocks(), p.lam), v)
    ref = o.matvec(v)
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    assert np.all(ya >= np.abs(y) * (1 - 1e-12))


def test_absolute_sum_without_cancellation():
    """With J_l = 0 no landmark term enters and, for non-negative J_p and v, no term cancels:
    the absolute sum equals the product (J_p^T J_p + lam diag) v."""
    p = synth.tiny(n_cams=4, n_lms=30, seed=1)
    Jp = np.abs(p.J_p)
    Jl = np.zeros_like(p.J_l)
    v = np.abs(np.random.default_rng(2).standard_normal(p.n))
    lamd = np.full(p.n, 0.5)
    y, ya = R.schur_matvec_stored(p.obs_cam, p.obs_lm, p.n_cams, p.n_lms, Jp, Jl, np.zeros((p.n_lms, 3, 3)),
                                  lamd, v)
    Hpp, _, _ = _dense_parts(p, Jp, Jl)
    assert np.abs(y - (Hpp @ v + lamd * v)).max() <= 1e-12 * y.max()
    assert np.abs(ya - y).max() <= 1e-12 * y.max()
