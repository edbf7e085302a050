"""The outer Levenberg-Marquardt support of the input generator (Sec. 4.1): moving the
state by a solved step and linearising again (synth.relinearize)."""
import numpy as np

import oracle
import synth


def test_zero_step_reproduces_the_linearisation():
    p = synth.tiny(n_cams=5, n_lms=40, seed=2, c_hi=5)
    q = synth.relinearize(p, np.zeros(p.n), np.zeros(3 * p.n_lms))
    assert np.array_equal(q.J_p, p.J_p) and np.array_equal(q.J_l, p.J_l) and np.array_equal(q.r, p.r)


def test_step_parametrisation_matches_the_jacobian():
    """r(x + h d) - r(x - h d) = 2 h J d + O(h^3): the update moves the state along the
    directions J_p and J_l differentiate (left rigid motion, f, k1, k2, points)."""
    p = synth.ring_problem(n_cams=8, n_lms=60, c_lo=2, c_hi=5, seed=4)
    rng = np.random.default_rng(1)
    d_p = rng.standard_normal(p.n) * np.tile([1e-2, 1e-2, 1e-2, 1e-1, 1e-1, 1e-1, 1.0, 1e-2, 1e-3], p.n_cams)
    d_l = rng.standard_normal(3 * p.n_lms) * 1e-1
    lin = np.einsum("mij,mj->mi", p.J_p, d_p.reshape(p.n_cams, 9)[p.obs_cam]) + \
        np.einsum("mij,mj->mi", p.J_l, d_l.reshape(p.n_lms, 3)[p.obs_lm])
    errs = []
    for h in (1e-2, 1e-3):
        rp = synth.relinearize(p, h * d_p, h * d_l).r
        rm = synth.relinearize(p, -h * d_p, -h * d_l).r
        errs.append(np.abs((rp - rm) / (2 * h) - lin).max())
    assert errs[1] < 1e-4 * np.abs(lin).max()
    assert errs[1] < errs[0] / 50          # second-order convergence of the central difference (h^2)


def test_lm_steps_from_the_oracle_decrease_the_cost():
    p = synth.ring_problem(n_cams=12, n_lms=300, c_lo=2, c_hi=6, seed=7)
    f0 = synth.cost(p)
    costs = [f0]
    for _ in range(3):
        o = oracle.System(p)
        x, st = o.pcg(eps=1e-10, imax=2000)
        dxl = o.back_substitute(x)
        p = synth.relinearize(p, x, dxl)
        costs.append(synth.cost(p))
    assert all(b < a for a, b in zip(costs, costs[1:]))
    # noise floor: 2 pixel coordinates per observation with 1 px noise
    assert costs[-1] < 3.0 * 2 * p.n_obs and f0 > 10 * costs[-1]
