"""Pins of the FP64 oracle of the learned low-rank preconditioner (oracle/learned.py)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import learned as L


@pytest.fixture(scope="module")
def small():
    p = synth.tiny(n_cams=6, n_lms=80, seed=3, c_hi=5)
    o = oracle.System(p)
    D = o.D_blocks()
    deg = L.covisibility_degree(p.n_cams, p.obs_cam, p.obs_lm)
    return p, o, D, deg


def test_degree_matches_schur_block_pattern(small):
    p, o, D, deg = small
    S = o.dense_S()
    blocks = np.abs(S.reshape(p.n_cams, 9, p.n_cams, 9)).max(axis=(1, 3)) > 0
    np.fill_diagonal(blocks, False)
    assert np.array_equal(deg, blocks.sum(1))


def test_features_are_scale_free(small):
    p, o, D, deg = small
    F = L.features(D, deg, 1e-4)
    assert F.shape == (p.n_cams, 47)
    assert np.allclose(L.features(37.5 * D, deg, 1e-4), F, atol=1e-12)
    assert np.all(np.abs(F[:, :36]) <= 1.0 + 1e-12)
    assert np.allclose(F[:, 36:45].sum(1), 0.0, atol=1e-12)


def test_zero_correction_is_block_jacobi(small):
    p, o, D, deg = small
    r = np.random.default_rng(0).standard_normal(p.n)
    assert np.allclose(L.apply_precond(D, np.zeros((p.n, 8)), r), o.precond(r), rtol=1e-12, atol=0)


def test_preconditioner_spd_for_any_weights(small):
    p, o, D, deg = small
    F = L.features(D, deg, 1e-4)
    Lc = L.chol_blocks(D)
    for seed in range(3):
        w = L.init_weights(seed, scale_out=1.0)
        _, _, out = L.mlp_forward(w, F)
        U = L.U_from_out(out, Lc)
        M = np.stack([L.apply_precond(D, U, e) for e in np.eye(p.n)], 1)
        assert np.abs(M - M.T).max() <= 1e-10 * np.abs(M).max()
        assert np.linalg.eigvalsh(0.5 * (M + M.T)).min() > 0


def test_loss_estimates_frobenius_norm(small):
    """The probe loss is an unbiased estimate of |I - (I + Uh Uh^T) Sh|_F^2 / n."""
    p, o, D, deg = small
    S = o.dense_S()
    Lc = L.chol_blocks(D)
    import scipy.linalg as sl
    Lb = sl.block_diag(*Lc)
    Sh = np.linalg.solve(Lb, np.linalg.solve(Lb, S.T).T)
    w = L.init_weights(1, scale_out=0.3)
    _, _, out = L.mlp_forward(w, L.features(D, deg, 1e-4))
    Uh = out.reshape(p.n, 8)
    A = np.eye(p.n) - (np.eye(p.n) + Uh @ Uh.T) @ Sh
    exact = (A * A).sum() / p.n
    rng = np.random.default_rng(5)
    W = rng.standard_normal((p.n, 40000))
    loss, _ = L.loss_and_grad_Uh(Uh, W, Sh @ W)
    assert abs(loss - exact) < 0.02 * exact


def test_backprop_matches_central_differences(small):
    p, o, D, deg = small
    F = L.features(D, deg, 1e-4)
    rng = np.random.default_rng(7)
    W = rng.standard_normal((p.n, 6))
    Sw = rng.standard_normal((p.n, 6))
    w = L.init_weights(2, scale_out=0.5)
    loss, g = L.loss_and_grad(w, F, W, Sw)
    flat, gflat = w.flat(), g.flat()
    idx = rng.choice(flat.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        a, b = flat.copy(), flat.copy()
        a[i] += h
        b[i] -= h
        fd = (L.loss_and_grad(L.Weights.from_flat(a), F, W, Sw)[0] -
              L.loss_and_grad(L.Weights.from_flat(b), F, W, Sw)[0]) / (2 * h)
        assert abs(fd - gflat[i]) <= 1e-6 * max(1.0, abs(gflat[i])) + 1e-9, (i, fd, gflat[i])


def test_adam_decreases_the_loss(small):
    p, o, D, deg = small
    F = L.features(D, deg, 1e-4)
    S = o.dense_S()
    Lc = L.chol_blocks(D)
    import scipy.linalg as sl
    Lb = sl.block_diag(*Lc)
    Sh = np.linalg.solve(Lb, np.linalg.solve(Lb, S.T).T)
    rng = np.random.default_rng(9)
    W = rng.standard_normal((p.n, 32))
    Sw = Sh @ W
    w = L.init_weights(3)
    m = np.zeros(L.n_params())
    v = np.zeros(L.n_params())
    l0 = L.loss_and_grad(w, F, W, Sw)[0]
    for t in range(1, 201):
        _, g = L.loss_and_grad(w, F, W, Sw)
        w = L.adam_step(w, g, m, v, t, lr=3e-3)
    assert L.loss_and_grad(w, F, W, Sw)[0] < l0
    assert L.n_params() == 15432
