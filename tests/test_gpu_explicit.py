"""Explicit block-sparse S (ba_build_opts.explicit_schur) against the FP64 oracle.

S is assembled from the same W_jl V_l^-1 W_kl^T blocks the implicit products apply,
so the operator bars are those of the implicit path: S v and the grouped product
1e-12; solver iterates after a fixed number of iterations 1e-9; converged solves
reach the 1e-6 residual.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ba = pytest.importorskip("paper_2110_04015_amd")


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=torch.float64)


def _h(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def relnorm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def covis(p):
    """Covisibility pattern (camera pairs sharing a landmark, diagonal included)."""
    A = np.zeros((p.n_cams, p.n_cams), dtype=bool)
    order = np.argsort(p.obs_lm, kind="stable")
    cam, lm = p.obs_cam[order], p.obs_lm[order]
    starts = np.flatnonzero(np.r_[True, lm[1:] != lm[:-1]])
    for a, b in zip(starts, np.r_[starts[1:], lm.shape[0]]):
        c = cam[a:b]
        A[np.ix_(c, c)] = True
    return A


PROBLEMS = {
    "tiny": lambda: synth.tiny(n_cams=5, n_lms=40, seed=2, c_hi=5, shuffle=True),
    "ring50": lambda: synth.config0(seed=0),
    "walk200": lambda: synth.walk_problem(n_cams=200, n_lms=20000, seed=1, name="walk200"),
    "cap120": lambda: synth.cap_problem(n_cams=120, n_lms=6000, seed=2, name="cap120"),
}


@pytest.fixture(scope="module", params=list(PROBLEMS))
def pair(request):
    p = PROBLEMS[request.param]()
    o = oracle.System(p)
    g = ba.System.from_problem(p, explicit_schur=True)
    yield request.param, p, o, g
    g.close()


def test_pattern_and_products(pair):
    name, p, o, g = pair
    info = g.explicit_schur_info()
    assert info["nnz_blocks"] == int(covis(p).sum())
    assert info["bytes"] == info["nnz_blocks"] * 81 * 8
    v = np.random.default_rng(0).standard_normal(g.n)
    y = _h(g.matvec(_dev(v)))
    assert rel(y, o.matvec(v)) < 1e-12
    assert np.array_equal(y, _h(g.matvec(_dev(v))))           # deterministic
    for N in (4, 16):
        if N > p.n_cams:
            continue
        Y = _h(g.matmat_grouped(N, _dev(v)))
        grp = np.repeat(oracle.partition(p.n_cams, N), 9)
        for q in range(N):
            assert rel(Y[q], o.matvec(np.where(grp == q, v, 0.0))) < 1e-12, q


def test_assembly_is_reproducible(pair):
    name, p, o, g = pair
    g2 = ba.System.from_problem(p, explicit_schur=True)
    v = _dev(np.random.default_rng(1).standard_normal(g.n))
    assert torch.equal(g.matvec(v), g2.matvec(v))
    g2.close()


def test_solver_iterates(pair):
    name, p, o, g = pair
    x, st = g.pcg(eps=0.0, max_iter=20)
    xo, so = o.pcg(eps=0.0, imax=20)
    assert relnorm(_h(x), xo) < 1e-9
    N = min(4, p.n_cams)
    x, st = g.mcg(N, 10.0, eps=0.0, max_iter=8, trace=True)
    xo, so, tro = o.mcg(N, 10.0, eps=0.0, imax=8, trace=True)
    assert st.multi_steps == so.multi_steps
    assert relnorm(_h(x), xo) < 1e-9
    x, st = g.mcg(N, 10.0)
    assert st.status == ba.BA_OK and st.rel_res_true < 1.05e-6


def test_rows_beyond_one_wavefront_lds():
    """Rows wider than one wavefront's LDS (251 blocks) are assembled in pieces by several
    wavefronts; the products still equal the oracle's operator."""
    p = synth.cap_problem(n_cams=300, n_lms=3000, c_min=30, c_max=40, zipf_s=0.2, seed=7, name="dense300")
    if covis(p).sum(1).max() * (81 * 8 + 4) <= 163840:
        pytest.skip("every row fits in LDS on this problem")
    o = oracle.System(p)
    g = ba.System.from_problem(p, explicit_schur=True)
    v = np.random.default_rng(3).standard_normal(g.n)
    ref = o.matvec(v)
    y = g.matvec(torch.from_numpy(v).cuda()).cpu().numpy()
    assert np.abs(y - ref).max() <= 1e-12 * np.abs(ref).max()
    x, st = g.pcg(eps=0.0, max_iter=5)
    xo, so = o.pcg(eps=0.0, imax=5)
    assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) < 1e-9
    g.close()


@pytest.mark.parametrize("explicit", [False, True])
def test_timed_products_equal_the_product(explicit):
    """ba_schur_matvec_timed (back-to-back launches for measurement) leaves the same y as
    ba_schur_matvec and reports a positive time; reps < 1 is refused."""
    p = synth.walk_problem(n_cams=120, n_lms=6000, seed=4, name="walk120")
    g = ba.System.from_problem(p, explicit_schur=explicit)
    v = torch.from_numpy(np.random.default_rng(5).standard_normal(g.n)).cuda()
    y0 = g.matvec(v)
    y1 = torch.empty_like(y0)
    ms = g.matvec_timed(v, reps=7, out=y1)
    assert ms > 0.0 and torch.equal(y0, y1)
    with pytest.raises(ba.BAError):
        g.matvec_timed(v, reps=0)
    g.close()
