"""Parity at the full size of the benchmark workload.

walk1936 (1,936 cameras, 650k landmarks, 5.08M observations, seed 0) in the
configuration the benchmark times (FP64, adaptive chunking, MCG with N = 16 and
tau = 3.3): the whole of S v against the oracle's operator, eight MCG iterations
(Alg. 2) against the oracle's, element by element, and the converged solve's true
residual computed by the oracle (the stop test of Alg. 2 at 1e-6).  The whole solve to
1e-6 is also compared with the oracle's own run to 1e-6 on this problem, stored by
tests/golden/make_walk1936_mcg.py (a few minutes of host time): iteration count within
2 %, equal multidirectional step count, the tau-test branch of every iteration equal
wherever t_i is not within 1e-6 of tau, the first residual-history entries within 1e-6;
and the same for PCG (Alg. 1).
"""
import json
import os

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


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "walk1936_mcg.json")


def test_fullsize_mcg_path_matches_oracle_run(full):
    p, o, g = full
    ref = json.load(open(GOLDEN))["mcg_N16_tau3.3"]
    x, st = g.mcg(16, 3.3, trace=True)
    assert st.status == ba.BA_OK and ref["status"] == 0
    assert abs(st.iterations - ref["iterations"]) <= max(1, 0.02 * ref["iterations"])
    assert st.multi_steps == ref["multi_steps"]
    t = np.array([np.nan if v is None else v for v in ref["trace_t"]])
    n = min(len(st.trace_k), len(ref["trace_k"])) - 1
    near = np.abs(t[:n] - 3.3) <= 1e-6 * 3.3
    assert np.all((st.trace_k[:n] == np.array(ref["trace_k"][:n])) | near)
    m = min(len(st.trace_res), 20)
    assert np.allclose(st.trace_res[:m], ref["trace_res"][:m], rtol=1e-6, atol=0)


def test_fullsize_pcg_path_matches_oracle_run(full):
    p, o, g = full
    ref = json.load(open(GOLDEN))["pcg"]
    x, st = g.pcg(trace=True)
    assert st.status == ba.BA_OK
    assert abs(st.iterations - ref["iterations"]) <= max(1, 0.02 * ref["iterations"])
    m = min(len(st.trace_res), 20)
    assert np.allclose(st.trace_res[:m], ref["trace_res"][:m], rtol=1e-6, atol=0)
