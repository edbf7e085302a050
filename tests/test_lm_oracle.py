"""Pins of the LM oracle (oracle/lm.py): the camera model, its Jacobians, the step and
the loop of Sec. 4.1, each against something other than the oracle itself (hand-worked
projections, central finite differences, an independent implementation of the model,
the dense damped least-squares step of eq. (6), and convergence to the exact solution
of a noise-free scene)."""
import numpy as np
import pytest

import oracle
import synth
from oracle import lm as olm


def _scene(p):
    return synth.camera_array(p.cams), p.points, p.obs_cam, p.obs_lm, p.u_obs


def test_rotation_exp_closed_forms():
    R = olm.rotation_exp(np.array([[0.0, 0.0, np.pi / 2]]))[0]
    assert np.allclose(R, [[0.0, -1.0, 0.0], [1.0, 0.0, 0.0], [0.0, 0.0, 1.0]], atol=1e-15)
    rng = np.random.default_rng(0)
    W = rng.standard_normal((20, 3))
    for w, E, Em in zip(W, olm.rotation_exp(W), olm.rotation_exp(-W)):
        assert np.abs(E.T @ E - np.eye(3)).max() < 1e-14
        assert abs(np.linalg.det(E) - 1.0) < 1e-14
        assert np.abs(E @ Em - np.eye(3)).max() < 1e-14
        assert np.abs(E @ w - w).max() < 1e-14 * (1 + np.linalg.norm(w))      # the axis is fixed
    w = np.array([3e-7, -1e-7, 2e-7])                                          # Taylor branch
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    assert np.abs(olm.rotation_exp(w)[0] - (np.eye(3) + K + 0.5 * K @ K)).max() < 1e-20


def test_projection_hand_worked():
    # R = I, t = 0, f = 500, k1 = 0.1, k2 = 0.01, X = (1, 2, 4): p = (1/4, 1/2), rho2 = 5/16,
    # s = 1 + 0.1 * 5/16 + 0.01 * 25/256 = 1.0322265625, u = 500 s p
    cam = np.array([[1, 0, 0, 0, 1, 0, 0, 0, 1, 0, 0, 0, 500.0, 0.1, 0.01]])
    u = olm.project(cam, np.array([[1.0, 2.0, 4.0]]), [0], [0])
    assert np.allclose(u, [[129.0283203125, 258.056640625]], rtol=1e-15)
    # quarter turn about z, t = (0, 0, 2), f = 1, no distortion: X = (1, 0, 2) -> P = (0, 1, 4)
    cam = np.array([[0, -1, 0, 1, 0, 0, 0, 0, 1, 0, 0, 2.0, 1.0, 0.0, 0.0]])
    assert np.allclose(olm.project(cam, np.array([[1.0, 0.0, 2.0]]), [0], [0]), [[0.0, 0.25]], atol=1e-16)


def test_model_agrees_with_the_input_generator():
    """Two independent implementations of the model: the oracle's and the generator's."""
    p = synth.ring_problem(n_cams=8, n_lms=60, c_lo=2, c_hi=5, seed=4)
    cams, X, cam, lm, u_obs = _scene(p)
    r = olm.residuals(cams, X, cam, lm, u_obs)
    assert np.abs(r - p.r).max() < 1e-12 * np.abs(p.r).max()
    Jp, Jl = olm.jacobians(cams, X, cam, lm)
    assert np.abs(Jp - p.J_p).max() < 1e-12 * np.abs(p.J_p).max()
    assert np.abs(Jl - p.J_l).max() < 1e-12 * np.abs(p.J_l).max()


def _fd_error(jac_fn, h):
    """max |(r(x + h d) - r(x - h d)) / 2h - J d| over random directions d."""
    p = synth.ring_problem(n_cams=6, n_lms=40, c_lo=2, c_hi=4, seed=9)
    cams, X, cam, lm, u_obs = _scene(p)
    Jp, Jl = jac_fn(cams, X, cam, lm)
    rng = np.random.default_rng(3)
    scale = np.tile([1e-2, 1e-2, 1e-2, 1e-1, 1e-1, 1e-1, 1.0, 1e-2, 1e-3], p.n_cams)
    worst, ref = 0.0, 0.0
    for _ in range(4):
        dp = rng.standard_normal(p.n) * scale
        dl = rng.standard_normal(3 * p.n_lms) * 1e-1
        lin = np.einsum("mij,mj->mi", Jp, dp.reshape(-1, 9)[cam]) + np.einsum("mij,mj->mi", Jl, dl.reshape(-1, 3)[lm])
        cp, Xp = olm.apply_step(cams, X, h * dp, h * dl)
        cm, Xm = olm.apply_step(cams, X, -h * dp, -h * dl)
        fd = (olm.residuals(cp, Xp, cam, lm, u_obs) - olm.residuals(cm, Xm, cam, lm, u_obs)) / (2 * h)
        worst = max(worst, np.abs(fd - lin).max())
        ref = max(ref, np.abs(lin).max())
    return worst, ref


def test_jacobians_match_central_differences():
    e2, ref = _fd_error(olm.jacobians, 1e-2)
    e3, _ = _fd_error(olm.jacobians, 1e-3)
    assert e3 < 1e-5 * ref
    assert e3 < e2 / 50                   # O(h^2): the step and the Jacobian describe the same motion


@pytest.mark.parametrize("mutation", ["rotation_sign", "k2_power", "landmark_R_transposed"])
def test_a_planted_jacobian_mistake_fails_the_difference_check(mutation):
    def bad(cams, X, cam, lm):
        Jp, Jl = olm.jacobians(cams, X, cam, lm)
        Jp, Jl = Jp.copy(), Jl.copy()
        if mutation == "rotation_sign":
            Jp[:, :, 0:3] *= -1.0
        elif mutation == "k2_power":
            Jp[:, :, 8] = Jp[:, :, 7]
        else:
            R = np.asarray(cams)[:, 0:9].reshape(-1, 3, 3)[np.asarray(cam)]
            A = np.einsum("mij,mkj->mik", Jl, R)            # undo A R, then apply R^T
            Jl = np.einsum("mij,mkj->mik", A, R)
        return Jp, Jl
    e, ref = _fd_error(bad, 1e-3)
    assert e > 1e-3 * ref


def test_first_step_is_the_dense_damped_least_squares_step():
    """eq. (6): minimise |r + J dx|^2 + lambda |D dx|^2 with D^T D = diag(J^T J); the
    oracle's Schur solve and back-substitution give the same dx as the stacked dense
    least-squares problem."""
    p = synth.ring_problem(n_cams=5, n_lms=30, c_lo=2, c_hi=4, seed=5)
    cams, X, cam, lm, u_obs = _scene(p)
    lam = 1e-3
    prob = olm.linearize(cams, X, cam, lm, u_obs, lam)
    m = len(cam)
    J = np.zeros((2 * m, prob.n_cams * 9 + 3 * prob.n_lms))
    for o in range(m):
        J[2 * o:2 * o + 2, 9 * cam[o]:9 * cam[o] + 9] = prob.J_p[o]
        J[2 * o:2 * o + 2, 9 * prob.n_cams + 3 * lm[o]:9 * prob.n_cams + 3 * lm[o] + 3] = prob.J_l[o]
    d = np.sqrt(lam * (J * J).sum(0))
    A = np.vstack([J, np.diag(d)])
    b = -np.concatenate([prob.r.ravel(), np.zeros(J.shape[1])])
    dx = np.linalg.lstsq(A, b, rcond=None)[0]
    o = oracle.System(prob)
    dxp, st = o.pcg(eps=1e-14, imax=5000)
    dxl = o.back_substitute(dxp)
    assert np.abs(dxp - dx[:9 * prob.n_cams]).max() < 1e-7 * np.abs(dx).max()
    assert np.abs(dxl - dx[9 * prob.n_cams:]).max() < 1e-7 * np.abs(dx).max()


@pytest.mark.parametrize("solver", ["pcg", "mcg"])
def test_lm_reaches_the_exact_solution_of_a_noise_free_scene(solver):
    p = synth.ring_problem(n_cams=8, n_lms=120, c_lo=3, c_hi=6, seed=11, noise_px=0.0)
    cams, X, cam, lm, u_obs = _scene(p)
    res = olm.lm(cams, X, cam, lm, u_obs, solver=solver, N=2, tau=3.3, eps=1e-10, ftol=0.0)
    assert res.cost0 > 1.0
    assert res.cost < 1e-18 * res.cost0 * len(cam) or res.cost < 1e-16
    # accepted moves decrease F; lambda follows the accept/reject rule
    lam = 1e-4
    F = res.cost0
    for it in res.iters:
        assert it.lam == pytest.approx(lam, rel=1e-15) and it.cost_before == F
        if it.accepted:
            assert it.cost_new < F
            F = it.cost_new
            lam /= 10.0
        else:
            assert it.cost_new >= F
            lam *= 10.0


def test_lm_stops_on_the_relative_function_tolerance():
    p = synth.ring_problem(n_cams=8, n_lms=200, c_lo=3, c_hi=6, seed=12)
    cams, X, cam, lm, u_obs = _scene(p)
    res = olm.lm(cams, X, cam, lm, u_obs, solver="pcg", ftol=1e-6)
    last = res.iters[-1]
    assert len(res.iters) < 25
    assert abs(last.cost_before - last.cost_new) / last.cost_before < 1e-6
    for it in res.iters[:-1]:
        assert abs(it.cost_before - it.cost_new) / it.cost_before >= 1e-6
    # noisy observations: the optimum keeps the noise, about 1 px^2 per residual row
    assert 0.3 < res.cost / (2 * len(cam)) < 1.5
