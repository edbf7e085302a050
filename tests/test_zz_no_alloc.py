"""The allocation-free Schur product (ba_schur_matvec_noalloc) against ba_schur_matvec.

Both run the same kernels in the same order; only the buffer of the partial camera
rows differs (a file-scope device array instead of the system's own), so the two
results must agree bit for bit.  Two calls in a row on different systems, the second
smaller, check that the shared array's leftovers from the first call do not leak into
the second.  The calls go through the C ABI (ctypes).
"""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _ba():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2110_04015_amd as ba
    return ba, torch


def _pair(ba, torch, g, seed, precision):
    v = torch.from_numpy(np.random.default_rng(seed).standard_normal(g.n)).cuda()
    y_ref = g.matvec(v, precision=precision)
    y = torch.full((g.n,), float("nan"), dtype=torch.float64, device="cuda")
    g.matvec_noalloc(v, y, precision=precision)
    torch.cuda.synchronize()
    return y_ref.cpu().numpy(), y.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
def test_noalloc_equals_matvec_two_calls(precision):
    ba, torch = _ba()
    print(f"no-alloc product, precision {precision}", flush=True)
    big = ba.System.from_problem(synth.walk_problem(n_cams=200, n_lms=40_000, seed=1), store_fp32=True,
                                 store_bf16=True)
    small = ba.System.from_problem(synth.tiny(n_cams=5, n_lms=40, seed=2, c_hi=5), store_fp32=True,
                                   store_bf16=True)
    assert small.n < big.n
    for g, seed in ((big, 0), (small, 1), (big, 2)):
        a, b = _pair(ba, torch, g, seed, precision)
        assert np.isfinite(b).all()
        assert np.array_equal(a, b), np.abs(a - b).max()
    big.close()
    small.close()


def test_noalloc_explicit_schur_and_dp6():
    ba, torch = _ba()
    print("no-alloc product, explicit S and d_p = 6", flush=True)
    p = synth.ring_problem(n_cams=50, n_lms=3000, seed=4)
    ex = ba.System.from_problem(p, explicit_schur=True)
    a, b = _pair(ba, torch, ex, 3, "fp64")
    assert np.array_equal(a, b)
    ex.close()
    p6 = synth.extrinsics_only(synth.tiny(n_cams=6, n_lms=60, seed=5, c_hi=5))
    g6 = ba.System.from_problem(p6)
    a, b = _pair(ba, torch, g6, 4, "fp64")
    assert np.array_equal(a, b)
    g6.close()


def test_noalloc_refuses_missing_precision_copy():
    ba, torch = _ba()
    g = ba.System.from_problem(synth.tiny(n_cams=5, n_lms=40, seed=2, c_hi=5))
    v = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    y = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    with pytest.raises(ba.BAError) as e:
        g.matvec_noalloc(v, y, precision="fp32")
    assert e.value.status == ba.BA_ERR_UNSUPPORTED
    # after an ordinary FP32 product the copy exists and the call goes through
    y_ref = g.matvec(v + 1.0, precision="fp32")
    g.matvec_noalloc(v + 1.0, y, precision="fp32")
    assert torch.equal(y, y_ref)
    g.close()
