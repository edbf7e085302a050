"""Batched Algorithm 2 (ba_batch_*) against the FP64 oracle, problem by problem.

The batch solves independent problems of different sizes at once.  Each problem
must follow its own Algorithm 2: the same parity bars as single solves apply per
problem (S products 1e-12, iterates after a fixed number of iterations 1e-9 with
equal multidirectional step counts, true residual below 1.05e-6 at eps = 1e-6).
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ba = pytest.importorskip("paper_2110_04015_amd")


def _h(t):
    return t.detach().cpu().numpy()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=torch.float64)


def relnorm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.fixture(scope="module")
def batch():
    probs = [synth.ring_problem(n_cams=24, n_lms=1500, c_lo=2, c_hi=6, seed=1, name="ring24"),
             synth.walk_problem(n_cams=90, n_lms=9000, seed=2, name="walk90"),
             synth.ring_problem(n_cams=40, n_lms=3000, c_lo=2, c_hi=8, seed=3, name="ring40"),
             synth.cap_problem(n_cams=60, n_lms=3000, seed=4, name="cap60")]
    orc = [oracle.System(p) for p in probs]
    b = ba.Batch(probs, store_fp32=True)
    yield probs, orc, b
    b.close()


def test_block_diagonal_products(batch):
    probs, orc, b = batch
    v = np.random.default_rng(0).standard_normal(b.n)
    y = _h(b.system.matvec(_dev(v)))
    for p, o, a, c in zip(probs, orc, b.row0, b.cams):
        seg = slice(int(a), int(a) + 9 * int(c))
        ref = o.matvec(v[seg])
        assert np.abs(y[seg] - ref).max() <= 1e-12 * np.abs(ref).max()
    bt = _h(b.system.rhs())
    for o, a, c in zip(orc, b.row0, b.cams):
        ref = o.rhs()
        assert np.abs(bt[int(a):int(a) + 9 * int(c)] - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("N,tau,k", [(4, 10.0, 6), (8, 3.3, 10), (1, 3.3, 12)])
def test_fixed_iterations_match_the_oracle(batch, N, tau, k):
    probs, orc, b = batch
    x, stats, ms, rc = b.mcg(N, tau, eps=0.0, max_iter=k)
    assert rc == ba.BA_MAXITER
    for o, xs, st in zip(orc, b.split(_h(x)), stats):
        xo, so = o.mcg(N, tau, eps=0.0, imax=k)
        assert st.iterations == so.iterations == k
        assert st.multi_steps == so.multi_steps
        assert relnorm(xs, xo) < 1e-9


@pytest.mark.parametrize("window", [0, 8])
def test_solve_to_1e6(batch, window):
    probs, orc, b = batch
    x, stats, ms, rc = b.mcg(4, 10.0, graph_window=window)
    assert rc == ba.BA_OK
    for o, xs, st in zip(orc, b.split(_h(x)), stats):
        so = o.mcg(4, 10.0)[1]
        bt = o.rhs()
        true = np.linalg.norm(-bt - o.matvec(xs)) / np.linalg.norm(bt)
        assert st.status == ba.BA_OK and true < 1.05e-6 and abs(true - st.rel_res_true) < 1e-9
        assert abs(st.iterations - so.iterations) <= max(1, 0.02 * so.iterations)
        assert 0.0 < st.done_ms <= ms


def test_graph_and_eager_agree_bitwise(batch):
    probs, orc, b = batch
    x0 = _h(b.mcg(8, 3.3, eps=0.0, max_iter=9, graph_window=0)[0])
    x1 = _h(b.mcg(8, 3.3, eps=0.0, max_iter=9, graph_window=4)[0])
    assert np.array_equal(x0, x1)


def test_mixed_precision_refinement(batch):
    probs, orc, b = batch
    x, stats, ms, rc = b.mcg(4, 10.0, precision="fp32")
    assert rc == ba.BA_OK
    for o, xs, st in zip(orc, b.split(_h(x)), stats):
        bt = o.rhs()
        true = np.linalg.norm(-bt - o.matvec(xs)) / np.linalg.norm(bt)
        assert st.status == ba.BA_OK and true < 1e-6 and st.refinement_steps >= 1


def test_mixed_precision_graph_and_eager(batch):
    """The refinement restarts each problem's inner solve on its own; graph replays and
    eager launches take the same steps."""
    probs, orc, b = batch
    x0, s0, _, rc0 = b.mcg(4, 10.0, precision="fp32", graph_window=0)
    x1, s1, _, rc1 = b.mcg(4, 10.0, precision="fp32", graph_window=8)
    assert rc0 == rc1 == ba.BA_OK
    assert np.array_equal(_h(x0), _h(x1))
    assert [s.iterations for s in s0] == [s.iterations for s in s1]
    assert [s.refinement_steps for s in s0] == [s.refinement_steps for s in s1]


def test_bad_arguments(batch):
    probs, orc, b = batch
    with pytest.raises(ba.BAError) as e:
        b.mcg(25, 3.3)          # more subsets than the smallest problem's cameras
    assert e.value.status == ba.BA_ERR_INVALID_ARG
    q = synth.ring_problem(n_cams=10, n_lms=200, seed=5)
    q.lam = 1e-3
    with pytest.raises(ValueError):
        ba.Batch([probs[0], q])
