"""Parity at the full size of the benchmark workload.

walk1936 (1,936 cameras, 650k landmarks, 5.08M observations, seed 0) in the
configuration the benchmark times (FP64, adaptive chunking, MCG with N = 16 and
tau = 3.3): the whole of S v against the oracle's operator, eight MCG iterations
(Alg. 2) against the oracle's, element by element, and the converged solve's true
residual computed by the oracle (the stop test of Alg. 2 at 1e-6).
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


@pytest.fixture(scope="module")
def full():
    print("\n[case] problem=walk1936 (full size)", flush=True)
    p = synth.config1(seed=0)
    o = oracle.System(p)
    g = ba.System.from_problem(p)
    yield p, o, g
    g.close()


def test_fullsize_matvec(full):
    p, o, g = full
    v = np.random.default_rng(0).standard_normal(g.n)
    y = _h(g.matvec(_dev(v)))
    ref = o.matvec(v)
    assert float(np.abs(y - ref).max() / np.abs(ref).max()) < 1e-12


def test_fullsize_mcg_fixed_iterations(full):
    p, o, g = full
    k = 8
    x, st = g.mcg(16, 3.3, eps=0.0, max_iter=k, trace=True)
    xo, so, tro = o.mcg(16, 3.3, eps=0.0, imax=k, trace=True)
    assert st.iterations == so.iterations == k
    assert np.array_equal(st.trace_k, tro[:, 2].astype(np.int32))
    xh = _h(x)
    assert np.linalg.norm(xh - xo) / np.linalg.norm(xo) < 1e-9


def test_fullsize_mcg_to_1e6(full):
    p, o, g = full
    x, st = g.mcg(16, 3.3)
    assert st.status == ba.BA_OK
    bt = o.rhs()
    res = np.linalg.norm(-bt - o.matvec(_h(x))) / np.linalg.norm(bt)
    assert res < 1.05e-6
    assert abs(res - st.rel_res_true) <= 1e-9
