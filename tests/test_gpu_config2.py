"""Parity at the full size of the dense-Schur workload.

cap571: the Alamo-shaped synthetic problem (Table 1's Alamo row: 571 poses, about
0.9M projections; 100k landmarks, 5-40 observers per landmark drawn with Zipf(1.2)
popularity, Schur block density near 0.8), with the paper's settings for that row,
N = 47 and tau = 10 (Table 1, Sec. 4.1).

  - S v in FP64 element by element against the oracle (max-abs relative 1e-12);
    FP32 and BF16 products against it per element, relative to the largest entry.
  - Eight iterations of Alg. 1 and Alg. 2 against the oracle's: iterates within 1e-9,
    equal branch sequences.
  - FP64 PCG and MCG, and MCG with FP32 products and with BF16-stored Jacobians under
    FP64 refinement, each run to a 1e-10 true residual: energy-norm error against the
    oracle's solution (PCG to 1e-12) at most 1e-6, and each to 1e-6 with the true
    residual recomputed by the oracle.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import reduced as R

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ba = pytest.importorskip("paper_2110_04015_amd")

N, TAU = 47, 10.0


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=torch.float64)


def _h(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def cap():
    print("\n[case] problem=cap571 (dense Schur, full size)", flush=True)
    p = synth.config2(seed=0)
    o = oracle.System(p)
    g = ba.System.from_problem(p, store_fp32=True, store_bf16=True)
    xs, so = o.pcg(eps=1e-12, imax=5000)
    assert so.status == 0
    yield p, o, g, xs
    g.close()


def _energy(o, x, xs):
    e = x - xs
    return float(np.sqrt(max(e @ o.matvec(e), 0.0) / (xs @ o.matvec(xs))))


def test_density_is_dense(cap):
    p, o, g, xs = cap
    assert synth.schur_block_density(p) > 0.3


def test_matvec(cap):
    p, o, g, xs = cap
    v = np.random.default_rng(0).standard_normal(g.n)
    ref = o.matvec(v)
    scale = np.abs(ref).max()
    y = _h(g.matvec(_dev(v)))
    assert np.abs(y - ref).max() / scale < 1e-12
    # reduced precision: per element against the largest entry (FP32: unit roundoff
    # 6e-8 times the cancellation of U v against W V^-1 W^T v; BF16: 3.9e-3 likewise)
    y32 = _h(g.matvec(_dev(v), precision="fp32"))
    assert np.abs(y32 - ref).max() / scale < 2e-5
    y16 = _h(g.matvec(_dev(v), precision="bf16"))
    assert np.abs(y16 - ref).max() / scale < 3e-2
    # and per element against the FP64 product with the stored blocks, within 64 u32 of
    # the absolute sum of its terms (the bound of the parity tests' reduced products)
    lamd = R.lambda_diag(o.U_blocks(), p.lam)
    for prec, y in (("fp32", y32), ("bf16", y16)):
        yr, ya = R.schur_matvec_stored(p.obs_cam, p.obs_lm, p.n_cams, p.n_lms, R.stored(p.J_p, prec),
                                       R.stored(p.J_l, prec), o.Vinv_blocks(), lamd, v)
        assert np.all(np.abs(y - yr) <= 64 * 2.0 ** -24 * ya), prec


def test_fixed_iterations(cap):
    p, o, g, xs = cap
    x, st = g.pcg(eps=0.0, max_iter=8)
    xo, so = o.pcg(eps=0.0, imax=8)
    assert np.linalg.norm(_h(x) - xo) / np.linalg.norm(xo) < 1e-9
    x, st = g.mcg(N, TAU, eps=0.0, max_iter=8, trace=True)
    xo, so, tro = o.mcg(N, TAU, eps=0.0, imax=8, trace=True)
    assert st.iterations == so.iterations == 8
    assert st.multi_steps == so.multi_steps
    assert np.array_equal(st.trace_k, tro[:, 2].astype(np.int32))
    assert np.linalg.norm(_h(x) - xo) / np.linalg.norm(xo) < 1e-9


@pytest.mark.parametrize("solver,prec", [("pcg", "fp64"), ("mcg", "fp64"), ("mcg", "fp32"), ("mcg", "bf16")])
def test_converged_solves(cap, solver, prec):
    p, o, g, xs = cap
    bt = o.rhs()
    run = (lambda **kw: g.pcg(**kw)) if solver == "pcg" else (lambda **kw: g.mcg(N, TAU, **kw))
    x, st = run(eps=1e-10, precision=prec)
    assert st.status == ba.BA_OK, st
    res = np.linalg.norm(-bt - o.matvec(_h(x))) / np.linalg.norm(bt)
    assert res < 1.05e-10
    err = _energy(o, _h(x), xs)
    print(f"{solver} {prec}: {st.iterations} iterations, {st.refinement_steps} refinement steps, "
          f"energy error {err:.2e}", flush=True)
    assert err <= 1e-6
    x, st = run(eps=1e-6, precision=prec)
    assert st.status == ba.BA_OK
    res = np.linalg.norm(-bt - o.matvec(_h(x))) / np.linalg.norm(bt)
    assert res < 1.05e-6
    assert abs(res - st.rel_res_true) <= 1e-9


def test_explicit_schur_dense_rows(cap):
    """The explicit S of the dense problem: rows of up to 571 blocks, assembled in pieces."""
    p, o, g, xs = cap
    ge = ba.System.from_problem(p, explicit_schur=True)
    info = ge.explicit_schur_info()
    assert info["nnz_blocks"] > 0.3 * p.n_cams ** 2
    v = np.random.default_rng(1).standard_normal(g.n)
    ref = o.matvec(v)
    y = _h(ge.matvec(_dev(v)))
    assert np.abs(y - ref).max() / np.abs(ref).max() < 1e-12
    assert np.array_equal(y, _h(ge.matvec(_dev(v))))          # run twice, bit for bit
    Y = _h(ge.matmat_grouped(N, _dev(v)))
    part = oracle.partition(p.n_cams, N)
    for q in range(N):
        zq = np.where(np.repeat(part == q, 9), v, 0.0)
        rq = o.matvec(zq)
        assert np.abs(Y[q] - rq).max() <= 1e-12 * np.abs(ref).max()
    x, st = ge.mcg(N, TAU, eps=0.0, max_iter=8, trace=True)
    xo, so, tro = o.mcg(N, TAU, eps=0.0, imax=8, trace=True)
    assert np.array_equal(st.trace_k, tro[:, 2].astype(np.int32))
    assert np.linalg.norm(_h(x) - xo) / np.linalg.norm(xo) < 1e-9
    x, st = ge.pcg(eps=1e-10)
    assert st.status == ba.BA_OK and _energy(o, _h(x), xs) <= 1e-6
    ge.close()
