"""The batched solver at the full size of the serving workload, in the launch shape the
benchmark times.

64 uneven problems (cameras U{50..800}, 200 landmarks per camera, 2-20 observers per
landmark, about 61M observations), chunk shape from the autotuner, MCG with N = 16 and
tau = 3.3, 8-iteration graph windows.  Problems sampled across the size range (the
smallest, the median and the largest) are compared with the oracle run on that problem
alone: iterates after six FP64 iterations within 1e-9 with equal multidirectional step
counts, and, after the FP32-product solve with FP64 refinement to 1e-6, the true residual
recomputed by the oracle below 1.05e-6 and equal to the library's figure within 1e-9.
"""
import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ba = pytest.importorskip("paper_2110_04015_amd")

N, TAU = 16, 3.3


def _h(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def full():
    from paper_2110_04015_amd import tune
    print("\n[case] batch of 64 problems (serving workload, full size)", flush=True)
    probs = synth.config4(seed=0, workers=16)
    order = np.argsort([p.n_cams for p in probs])
    tn = tune.tune_chunks([probs[i] for i in order[::8]], "fp32")
    print(f"[case] autotuned shape {tn['max_slots']} x {tn['max_tiles']}", flush=True)
    b = ba.Batch(probs, max_slots=tn["max_slots"], max_tiles=tn["max_tiles"], store_fp32=True)
    sample = [int(order[0]), int(order[len(order) // 2]), int(order[-1])]
    yield probs, b, sample
    b.close()


def test_fixed_iterations_sampled(full):
    probs, b, sample = full
    x, stats, ms, rc = b.mcg(N, TAU, eps=0.0, max_iter=6, graph_window=8)
    xs = b.split(_h(x))
    for i in sample:
        xo, so = oracle.System(probs[i]).mcg(N, TAU, eps=0.0, imax=6)
        assert stats[i].iterations == so.iterations == 6
        assert stats[i].multi_steps == so.multi_steps
        assert np.linalg.norm(xs[i] - xo) / np.linalg.norm(xo) < 1e-9, i


def test_mixed_solve_sampled(full):
    probs, b, sample = full
    x, stats, ms, rc = b.mcg(N, TAU, precision="fp32", max_inner=300, graph_window=8)
    assert rc == ba.BA_OK
    assert all(s.status == ba.BA_OK for s in stats)
    # problems retire when each one's own refinement reaches eps, not all at the end
    done = sorted(s.done_ms for s in stats)
    assert done[0] < done[-1] <= ms
    xs = b.split(_h(x))
    for i in sample:
        o = oracle.System(probs[i])
        bt = o.rhs()
        true = np.linalg.norm(-bt - o.matvec(xs[i])) / np.linalg.norm(bt)
        assert true < 1.05e-6 and abs(true - stats[i].rel_res_true) <= 1e-9, i
