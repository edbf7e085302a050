"""LM outer loop on the GPU (ba_project, ba_apply_step, ba_update_system, ba_lm_solve)
against the LM oracle (oracle/lm.py).

Bars: residuals, Jacobians and the moved state 1e-12 relative (one evaluation of the
same closed forms, rounding only); F at the moved state of every LM iteration within
1e-8 of F at the state it moved from (each step comes from an iterative solve whose
GPU and oracle iterates agree to about 1e-9 relative; F at a point off the
linearisation's minimum moves to first order with the step, on the scale of the F
it decreases from), or within 4 x the spread of correct FP64 runs where that is
larger: the largest difference between the oracle and the oracle on the same scene
with its landmarks relabelled and its observations reordered (four such orders), which
changes nothing but the order of the sums.  A solve that
runs for more iterations than S has rows (the small ring scenes at small lambda, where
the scene's gauge leaves S nearly singular) amplifies rounding differences that far.
The accept/reject sequence and the damping sequence are identical.
The final states are compared through their residual vectors: BA leaves a similarity
transform of the whole scene (gauge) unfixed, along which the two paths may drift
apart without changing any residual.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import lm as olm

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ba = pytest.importorskip("paper_2110_04015_amd")


def _h(t):
    return t.detach().cpu().numpy()


def _dev(a, dt=None):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=dt or torch.float64)


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


SCENES = {
    "ring12": lambda: synth.ring_problem(n_cams=12, n_lms=400, c_lo=2, c_hi=6, seed=7, name="ring12"),
    "walk60": lambda: synth.walk_problem(n_cams=60, n_lms=3000, seed=3, name="walk60"),
    "ring_ragged": lambda: synth.ring_problem(n_cams=9, n_lms=77, c_lo=2, c_hi=4, seed=5, shuffle=True),
}


@pytest.fixture(scope="module", params=list(SCENES))
def scene(request):
    p = SCENES[request.param]()
    sc, cams, X = ba.Scene.from_problem(p)
    return request.param, p, sc, cams, X


def test_residuals_and_jacobians(scene):
    name, p, sc, cams, X = scene
    c = synth.camera_array(p.cams)
    r, Jp, Jl, F = sc.project(cams, X)
    ro = olm.residuals(c, p.points, p.obs_cam, p.obs_lm, p.u_obs)
    Jpo, Jlo = olm.jacobians(c, p.points, p.obs_cam, p.obs_lm)
    assert rel(_h(r), ro) < 1e-12
    assert rel(_h(Jp), Jpo) < 1e-12
    assert rel(_h(Jl), Jlo) < 1e-12
    assert abs(F - olm.cost(ro)) < 1e-12 * olm.cost(ro)
    r2, Jp2, Jl2, F2 = sc.project(cams, X, jacobians=False)
    assert torch.equal(r, r2) and F2 == F and Jp2 is None


def test_moved_state(scene):
    name, p, sc, cams, X = scene
    rng = np.random.default_rng(0)
    dxp = rng.standard_normal(9 * p.n_cams) * np.tile([1e-2] * 3 + [1e-1] * 3 + [1.0, 1e-3, 1e-4], p.n_cams)
    dxp[:9] *= 1e-6                                   # one camera on the small-angle branch
    dxl = rng.standard_normal(3 * p.n_lms) * 1e-1
    co, Xo = sc.apply_step(cams, X, _dev(dxp), _dev(dxl))
    c_ref, X_ref = olm.apply_step(synth.camera_array(p.cams), p.points, dxp, dxl)
    assert rel(_h(co), c_ref) < 1e-12
    assert rel(_h(Xo), X_ref) < 1e-14


def test_update_equals_a_fresh_build(scene):
    """A system updated in place (new linearisation and lambda) gives bit-identical
    products, right-hand side and preconditioner to one built from the same values."""
    name, p, sc, cams, X = scene
    r, Jp, Jl, F = sc.project(cams, X)
    oc, ol = _dev(p.obs_cam, torch.int32), _dev(p.obs_lm, torch.int32)
    g = ba.System(p.n_cams, p.n_lms, oc, ol, _dev(p.J_p) * 1.5, _dev(p.J_l), _dev(p.r), 1e-2, store_fp32=True)
    g.update(Jp, Jl, r, 3e-3)
    fresh = ba.System(p.n_cams, p.n_lms, oc, ol, Jp, Jl, r, 3e-3, store_fp32=True)
    v = _dev(np.random.default_rng(1).standard_normal(9 * p.n_cams))
    assert torch.equal(g.matvec(v), fresh.matvec(v))
    assert torch.equal(g.matvec(v, precision="fp32"), fresh.matvec(v, precision="fp32"))
    assert torch.equal(g.rhs(), fresh.rhs())
    assert torch.equal(g.precond(v), fresh.precond(v))
    o = oracle.System(olm.linearize(synth.camera_array(p.cams), p.points, p.obs_cam, p.obs_lm, p.u_obs, 3e-3))
    ref = o.matvec(_h(v))
    assert rel(_h(g.matvec(v)), ref) < 1e-12
    bad = r.clone()
    bad[0, 0] = float("nan")
    with pytest.raises(ba.BAError) as e:
        g.update(Jp, Jl, bad, 1e-3)
    assert e.value.status == ba.BA_ERR_NONFINITE
    assert torch.equal(g.matvec(v), fresh.matvec(v))        # nothing changed
    g.close()
    fresh.close()


def _relabelled_oracle_lm(p, seed, **kw):
    """The oracle's LM loop on the same scene with the landmarks relabelled and the
    observations reordered: the same arithmetic summed in another order."""
    rng = np.random.default_rng(seed)
    perm = rng.permutation(p.n_lms)
    inv = np.empty_like(perm)
    inv[perm] = np.arange(p.n_lms)
    order = rng.permutation(p.n_obs)
    return olm.lm(synth.camera_array(p.cams), p.points[perm], p.obs_cam[order], inv[p.obs_lm[order]],
                  p.u_obs[order], **kw)


@pytest.mark.parametrize("solver,N", [("pcg", 1), ("mcg", 4)])
def test_lm_loop_matches_the_oracle(scene, solver, N):
    name, p, sc, cams, X = scene
    N = min(N, p.n_cams)
    c1, X1, st = sc.lm(cams, X, solver=solver, N=N, tau=3.3)
    ref = olm.lm(synth.camera_array(p.cams), p.points, p.obs_cam, p.obs_lm, p.u_obs, solver=solver, N=N, tau=3.3)
    alts = [_relabelled_oracle_lm(p, seed, solver=solver, N=N, tau=3.3) for seed in range(4)]
    assert st.status == ba.BA_OK
    assert st.iterations == len(ref.iters)
    assert all(len(a.iters) == len(ref.iters) for a in alts)
    assert abs(st.cost0 - ref.cost0) < 1e-12 * ref.cost0
    assert [bool(a) for a in st.trace_accepted] == [it.accepted for it in ref.iters]
    assert np.array_equal(st.trace_lambda, [it.lam for it in ref.iters])
    for i, (got, it) in enumerate(zip(st.trace_cost, ref.iters)):
        spread = max(abs(a.iters[i].cost_new - it.cost_new) for a in alts)
        assert abs(got - it.cost_new) < max(1e-8 * it.cost_before, 4.0 * spread), i
    spread = max(abs(a.cost - ref.cost) for a in alts)
    assert abs(st.cost - ref.cost) < max(1e-8 * ref.iters[-1].cost_before, 4.0 * spread)
    assert st.accepted == sum(it.accepted for it in ref.iters)
    r1 = _h(sc.project(c1, X1, jacobians=False)[0])
    assert rel(r1, olm.residuals(ref.cams, ref.X, p.obs_cam, p.obs_lm, p.u_obs)) < 1e-6
    assert st.t_solve_ms > 0 and st.t_total_ms >= st.t_solve_ms


def test_lm_noise_free_scene_reaches_zero():
    p = synth.ring_problem(n_cams=8, n_lms=120, c_lo=3, c_hi=6, seed=11, noise_px=0.0)
    sc, cams, X = ba.Scene.from_problem(p)
    c1, X1, st = sc.lm(cams, X, solver="mcg", N=2, eps=1e-10, ftol=0.0, max_iter=8)
    assert st.cost0 > 1.0 and st.cost < 1e-16 * len(p.obs_cam)
    r, _, _, F = sc.project(c1, X1, jacobians=False)
    assert F == st.cost


def test_lm_zero_iterations_and_bad_arguments():
    p = synth.ring_problem(n_cams=6, n_lms=50, c_lo=2, c_hi=4, seed=2)
    sc, cams, X = ba.Scene.from_problem(p)
    c1, X1, st = sc.lm(cams, X, max_iter=0)
    assert st.iterations == 0 and torch.equal(c1, cams) and st.cost == st.cost0
    with pytest.raises(ba.BAError) as e:
        sc.lm(cams, X, lambda_factor=1.0)
    assert e.value.status == ba.BA_ERR_INVALID_ARG
    with pytest.raises(ba.BAError) as e:
        sc.lm(cams, X, solver="mcg", N=0)
    assert e.value.status == ba.BA_ERR_INVALID_ARG
