"""ba_set_lambda: a new damping lambda for the same linearisation (the LM loop's step
after a rejected move, Sec. 4.1) from the undamped blocks kept at build and the packed
Jacobian stream, without reading J or r again.

Bar: bit-for-bit equal to a fresh build of the same J and r at the new lambda (the
same kernels run on the same lambda-free sums), for every value a solve reads -- S v in
FP64, FP32 and BF16, the multidirectional product, b~, the D(S) blocks and their
Cholesky solves, the back-substitution -- and for PCG and MCG iterates; and 1e-12
against the oracle built at the new lambda.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
ba = pytest.importorskip("paper_2110_04015_amd")

PROBLEMS = {
    "tiny": lambda: synth.tiny(n_cams=5, n_lms=40, seed=2, c_hi=5),
    "ring50": lambda: synth.config0(seed=1),
    "walk200": lambda: synth.walk_problem(n_cams=200, n_lms=20_000, seed=3),
    "cap120": lambda: synth.cap_problem(n_cams=120, n_lms=5000, seed=4),
    "ring50_dp6": lambda: synth.extrinsics_only(synth.config0(seed=2)),
}


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=torch.float64)


def _h(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def _same(a, b):
    torch.cuda.synchronize()
    return torch.equal(a, b)


@pytest.mark.parametrize("name", list(PROBLEMS))
def test_set_lambda_equals_fresh_build(name):
    print(f"\n[case] set_lambda problem={name}", flush=True)
    p = PROBLEMS[name]()
    kw = dict(store_fp32=True, store_bf16=True)
    lam1 = 3e-2
    g = ba.System.from_problem(p, **kw)            # built at p.lam = 1e-4
    g.set_lambda(lam1)
    p1 = dataclasses.replace(p, lam=lam1)
    fresh = ba.System.from_problem(p1, **kw)
    n = g.n
    v = _dev(np.random.default_rng(1).standard_normal(n))
    for prec in ("fp64", "fp32", "bf16"):
        assert _same(g.matvec(v, precision=prec), fresh.matvec(v, precision=prec)), prec
    assert _same(g.rhs(), fresh.rhs())
    assert _same(g.precond_blocks(), fresh.precond_blocks())
    assert _same(g.precond(v), fresh.precond(v))
    assert _same(g.back_substitute(v), fresh.back_substitute(v))
    N = min(4, p.n_cams)
    assert _same(g.matmat_grouped(N, v), fresh.matmat_grouped(N, v))
    xa, sa = g.pcg(eps=0.0, max_iter=7)
    xb, sb = fresh.pcg(eps=0.0, max_iter=7)
    assert _same(xa, xb)
    xa, sa = g.mcg(N, 10.0, eps=0.0, max_iter=6)
    xb, sb = fresh.mcg(N, 10.0, eps=0.0, max_iter=6)
    assert _same(xa, xb) and sa.multi_steps == sb.multi_steps
    # against the oracle at the new lambda
    o = oracle.System(p1)
    assert rel(_h(g.matvec(v)), o.matvec(_h(v))) < 1e-12
    assert rel(_h(g.rhs()), o.rhs()) < 1e-12
    D = _h(g.precond_blocks())
    assert rel(D, o.D_blocks().reshape(D.shape)) < 1e-12
    # and back: the first lambda again equals the first build
    g.set_lambda(p.lam)
    first = ba.System.from_problem(p, **kw)
    assert _same(g.matvec(v), first.matvec(v)) and _same(g.rhs(), first.rhs())
    assert _same(g.precond(v), first.precond(v))
    for s in (g, fresh, first):
        s.close()


def test_set_lambda_explicit_schur():
    print("\n[case] set_lambda explicit S", flush=True)
    p = synth.walk_problem(n_cams=120, n_lms=10_000, seed=6)
    g = ba.System.from_problem(p, explicit_schur=True)
    g.set_lambda(1e-1)
    p1 = dataclasses.replace(p, lam=1e-1)
    fresh = ba.System.from_problem(p1, explicit_schur=True)
    v = _dev(np.random.default_rng(2).standard_normal(g.n))
    assert _same(g.matvec(v), fresh.matvec(v))
    assert _same(g.matmat_grouped(8, v), fresh.matmat_grouped(8, v))
    o = oracle.System(p1)
    assert rel(_h(g.matvec(v)), o.matvec(_h(v))) < 1e-12
    g.close()
    fresh.close()


def test_set_lambda_errors_change_nothing():
    p = synth.tiny(n_cams=5, n_lms=40, seed=2, c_hi=5)
    g = ba.System.from_problem(p)
    v = _dev(np.random.default_rng(3).standard_normal(g.n))
    y0 = g.matvec(v).clone()
    for bad, status in ((-1.0, ba.BA_ERR_INVALID_ARG), (float("nan"), ba.BA_ERR_NONFINITE),
                        (float("inf"), ba.BA_ERR_NONFINITE)):
        with pytest.raises(ba.BAError) as e:
            g.set_lambda(bad)
        assert e.value.status == status
    assert _same(g.matvec(v), y0)
    g.close()
