"""GPU path (libba.so through the C ABI) against the FP64 CPU oracle.

Tolerances (FP64 path):
  - single operators (S v, S Z, D^-1 r, b~, D(S), back-substitution, pinv):
    1e-12 relative in max norm -- a few hundred roundings of O(1) terms;
  - solver iterates after a fixed number of iterations: 1e-9 relative (the
    stated FP64 target);
  - solves run to eps = 1e-10: the GPU solution's energy-norm distance to the
    dense solution x* is at most 4 x the largest of the oracle's and that of two
    textbook dense NumPy PCG forms run to the same eps (at least 1e-9). The two
    textbook forms alone land 14 x apart on the tiny problem (kappa(S) = 3e9),
    and the bound a residual of eps guarantees, sqrt(kappa) eps, is looser still;
  - solves stopped at eps = 1e-6: true residual below 1.05e-6, iteration count
    within 2 % (at least 1) of the oracle's, residual histories equal to 1e-6
    over the first 20 iterations (PCG) or 5 iterations (MCG, whose later Gram
    blocks become numerically rank deficient on the smallest problem).
  Two correct FP64 implementations (the oracle and a dense NumPy PCG) differ by
  up to 5e-8 in x at eps = 1e-10 and up to 5e-7 (energy norm) at eps = 1e-6 on
  these problems: the gauge directions of S are damped only by lambda, so a
  1e-9 gate on such iterates would measure summation order, not correctness.
Reduced-precision products (FP32 arithmetic on FP32 or BF16 Jacobian blocks, FP64 sums):
  per element against the FP64 product with the stored blocks (oracle/reduced.py), within
  64 u (u = 2^-24) times the sum of the absolute values of the terms. The longest chain
  of FP32 roundings behind one term has about 25 (the FP32 casts of v, V^-1 and g, the
  9-term e = J_p v, the 3-term V^-1 g, J_l h and the difference, the 2-term J_p^T f), so
  the first-order bound is about 25 u; 64 u leaves room. A wrong index, sign or dropped
  term moves elements by the size of the terms, far above it.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import reduced as R

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

ba = pytest.importorskip("paper_2110_04015_amd")


def _dev(a, dt=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype=dt)


def _h(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def relnorm(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


U32 = 2.0 ** -24


def stored_product(p, o, prec, v):
    """(S^ v, |S^||v|) of the reduced-precision operator: the blocks as stored, V^-1 and the
    damping of the FP64 system."""
    return R.schur_matvec_stored(p.obs_cam, p.obs_lm, p.n_cams, p.n_lms, R.stored(p.J_p, prec),
                                 R.stored(p.J_l, prec), o.Vinv_blocks(), R.lambda_diag(o.U_blocks(), p.lam), v)


def assert_within_rounding(y, ref, bound, what=""):
    err = np.abs(y - ref)
    i = int(np.argmax(err / np.maximum(bound, 1e-300)))
    assert np.all(err <= 64 * U32 * bound), (what, i, err[i], bound[i])


PROBLEMS = {
    "tiny": lambda: synth.tiny(n_cams=5, n_lms=40, seed=2, c_hi=5, shuffle=True),
    "ring50": lambda: synth.config0(seed=0),
    "walk200": lambda: synth.walk_problem(n_cams=200, n_lms=20000, seed=1, name="walk200"),
    "cap120": lambda: synth.cap_problem(n_cams=120, n_lms=6000, seed=2, name="cap120"),
}


@pytest.fixture(scope="module", params=sorted(PROBLEMS))
def pair(request):
    print(f"\n[case] problem={request.param}", flush=True)
    p = PROBLEMS[request.param]()
    o = oracle.System(p)
    g = ba.System.from_problem(p)
    yield request.param, p, o, g
    g.close()


_DENSE = {}


def dense(name, o):
    """Dense S (through the oracle operator) and x* = -S^-1 b~ for a small problem."""
    if name not in _DENSE:
        S = o.dense_S()
        S = 0.5 * (S + S.T)
        _DENSE[name] = (S, np.linalg.solve(S, -o.rhs()))
    return _DENSE[name]


def energy_err(S, x, xs):
    e = x - xs
    return float(np.sqrt(e @ S @ e) / np.sqrt(xs @ S @ xs))


_SPREAD = {}


def textbook_spread(name, o, eps=1e-10):
    """Largest energy error of two textbook PCG forms on the dense S (beta from
    Q^T z and from r^T z), block-Jacobi preconditioned, run to the same eps: how far
    correct FP64 implementations land from x* on this problem."""
    if name not in _SPREAD:
        S, xs = dense(name, o)
        b = -o.rhs()
        errs = []
        for form in ("phi", "rz"):
            x = np.zeros_like(b)
            r = b.copy()
            z = o.precond(r)
            P = z.copy()
            rz = r @ z
            for _ in range(20 * b.size):
                Q = S @ P
                d = P @ Q
                a = (P @ r) / d if form == "phi" else rz / d
                x += a * P
                r -= a * Q
                if np.linalg.norm(r) < eps * np.linalg.norm(b):
                    break
                z = o.precond(r)
                if form == "phi":
                    P = z - (Q @ z) / d * P
                else:
                    rz, rz_old = r @ z, rz
                    P = z + rz / rz_old * P
            errs.append(energy_err(S, x, xs))
        _SPREAD[name] = max(errs)
    return _SPREAD[name]


def converged_gate(name, o, S, xs, xo):
    return 4.0 * max(energy_err(S, xo, xs), textbook_spread(name, o), 1e-9 / 4)


@pytest.fixture(scope="module")
def ring():
    p = synth.config0(seed=0)
    o = oracle.System(p)
    g = ba.System.from_problem(p)
    yield p, o, g
    g.close()


# ---------------------------------------------------------------- A1 build


def test_rhs_and_preconditioner_blocks(pair):
    name, p, o, g = pair
    assert rel(_h(g.rhs()), o.rhs()) < 1e-12
    assert rel(_h(g.precond_blocks()), o.D_blocks()) < 1e-12


# ---------------------------------------------------------------- A2 S v


def test_matvec_fp64(pair):
    name, p, o, g = pair
    rng = np.random.default_rng(0)
    for _ in range(3):
        v = rng.standard_normal(g.n)
        y = _h(g.matvec(_dev(v)))
        assert rel(y, o.matvec(v)) < 1e-12


def test_matvec_deterministic(pair):
    name, p, o, g = pair
    v = _dev(np.random.default_rng(1).standard_normal(g.n))
    a, b = _h(g.matvec(v)), _h(g.matvec(v))
    assert np.array_equal(a, b)


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-5), ("bf16", 3e-2)])
def test_matvec_reduced_precision(pair, prec, tol):
    name, p, o, g = pair
    v = np.random.default_rng(2).standard_normal(g.n)
    y = _h(g.matvec(_dev(v), precision=prec))
    assert relnorm(y, o.matvec(v)) < tol
    ref, bound = stored_product(p, o, prec, v)
    assert_within_rounding(y, ref, bound, (name, prec))


# ---------------------------------------------------------------- A3 S Z


@pytest.mark.parametrize("N", [1, 3, 16])
def test_matmat_grouped(pair, N):
    name, p, o, g = pair
    if N > p.n_cams:
        pytest.skip("more subsets than cameras")
    z = np.random.default_rng(3).standard_normal(g.n)
    Y = _h(g.matmat_grouped(N, _dev(z)))
    grp = np.repeat(oracle.partition(p.n_cams, N), 9)
    for q in range(N):
        ref = o.matvec(np.where(grp == q, z, 0.0))
        assert rel(Y[q], ref) < 1e-12, q
    assert np.array_equal(grp // 1, np.repeat(ba.partition(p.n_cams, N), 9))


@pytest.mark.parametrize("max_tiles,max_tiles_multi", [(1, 1), (16, 0), (0, 3), (2, 40)])
def test_chunk_shapes(max_tiles, max_tiles_multi):
    """The chunk size (tiles per chunk of either product, fixed or sized by the plan to the
    resident wavefronts) changes only how the work is split: the products stay within
    1e-12 of the oracle."""
    p = PROBLEMS["walk200"]()
    o = oracle.System(p)
    g = ba.System.from_problem(p, max_tiles=max_tiles, max_tiles_multi=max_tiles_multi)
    rng = np.random.default_rng(11)
    v = rng.standard_normal(g.n)
    assert rel(_h(g.matvec(_dev(v))), o.matvec(v)) < 1e-12
    N = 16
    Y = _h(g.matmat_grouped(N, _dev(v)))
    grp = np.repeat(oracle.partition(p.n_cams, N), 9)
    for q in range(N):
        assert rel(Y[q], o.matvec(np.where(grp == q, v, 0.0))) < 1e-12, q
    g.close()


def test_product_timing_sampled(ring):
    """Event timing of the S product: every launch, or every k-th; a negative k is refused."""
    p, o, g = ring
    v = _dev(np.random.default_rng(5).standard_normal(g.n))
    for every, expect in ((1, 8), (4, 2), (3, 3)):
        g.profile(True, every=every)
        g.profile_read(reset=True)
        for _ in range(8):
            g.matvec(v)
        ms, n = g.profile_read(reset=True)
        g.profile(False)
        assert n == expect and ms > 0.0, (every, n, ms)
    with pytest.raises(ba.BAError):
        g.profile(True, every=-1)


@pytest.mark.parametrize("prec,tol", [("fp32", 2e-5), ("bf16", 3e-2)])
def test_matmat_grouped_reduced_precision(pair, prec, tol):
    name, p, o, g = pair
    N = min(16, p.n_cams)
    z = np.random.default_rng(7).standard_normal(g.n)
    Y = _h(g.matmat_grouped(N, _dev(z), precision=prec))
    grp = np.repeat(oracle.partition(p.n_cams, N), 9)
    for q in range(N):
        zq = np.where(grp == q, z, 0.0)
        assert relnorm(Y[q], o.matvec(zq)) < tol, q
        ref, bound = stored_product(p, o, prec, zq)
        assert_within_rounding(Y[q], ref, bound, (name, prec, q))


def test_matmat_grouped_large_lds():
    """35 observers per landmark spread over 60 subsets: a tile touches more (camera,
    subset) pairs than 64 KiB of LDS holds, so the kernel runs with a larger work-group
    allocation."""
    p = synth.cap_problem(n_cams=120, n_lms=600, c_min=30, c_max=40, seed=5, name="dense120")
    o = oracle.System(p)
    g = ba.System.from_problem(p)
    N = 60
    z = np.random.default_rng(6).standard_normal(g.n)
    Y = _h(g.matmat_grouped(N, _dev(z)))
    grp = np.repeat(oracle.partition(p.n_cams, N), 9)
    for q in range(N):
        assert rel(Y[q], o.matvec(np.where(grp == q, z, 0.0))) < 1e-12, q
    x, st = g.mcg(N, 10.0, eps=0.0, max_iter=4)
    xo, so = o.mcg(N, 10.0, eps=0.0, imax=4)
    assert st.multi_steps == so.multi_steps and relnorm(_h(x), xo) < 1e-9
    g.close()


# ---------------------------------------------------------------- A4 D^-1 r, eq. (16)


def test_precond_apply(pair):
    name, p, o, g = pair
    r = np.random.default_rng(4).standard_normal(g.n)
    assert rel(_h(g.precond(_dev(r))), o.precond(r)) < 1e-11


def test_back_substitution(pair):
    name, p, o, g = pair
    dxp = np.random.default_rng(5).standard_normal(g.n)
    assert rel(_h(g.back_substitute(_dev(dxp))), o.back_substitute(dxp)) < 1e-12


# ---------------------------------------------------------------- A6 pinv


@pytest.mark.parametrize("k,r", [(1, 1), (2, 2), (5, 5), (16, 16), (32, 32), (33, 33), (47, 47), (57, 57), (64, 64),
                                 (16, 9), (47, 30), (64, 1)])
def test_pinv(k, r):
    rng = np.random.default_rng(k * 100 + r)
    Qm, _ = np.linalg.qr(rng.standard_normal((k, k)))
    lam = np.zeros(k)
    lam[:r] = rng.uniform(0.2, 5.0, r)
    A = (Qm * lam) @ Qm.T
    A = 0.5 * (A + A.T)
    Ap, rank = ba.pinv_sym(_dev(A))
    Ao, ro, _ = oracle.pinv(A)
    assert rank == ro == r
    assert rel(_h(Ap), Ao) < 1e-11


# ---------------------------------------------------------------- A2-A10 PCG


@pytest.mark.parametrize("k", [1, 5, 30])
def test_pcg_fixed_iterations(pair, k):
    name, p, o, g = pair
    x, st = g.pcg(eps=0.0, max_iter=k)
    xo, so = o.pcg(eps=0.0, imax=k)
    assert st.iterations == so.iterations == k and st.status == ba.BA_MAXITER
    assert relnorm(_h(x), xo) < 1e-9


def test_pcg_converged(pair):
    name, p, o, g = pair
    S, xs = dense(name, o)
    x, st = g.pcg(eps=1e-10, max_iter=5000)
    xo, so = o.pcg(eps=1e-10, imax=5000)
    assert st.status == ba.BA_OK and so.status == oracle.OK
    assert energy_err(S, _h(x), xs) <= converged_gate(name, o, S, xs, xo)


def test_pcg_to_1e6(pair):
    name, p, o, g = pair
    x, st = g.pcg(trace=True)
    xo, so, tro = o.pcg(trace=True)
    assert st.status == ba.BA_OK
    assert abs(st.iterations - so.iterations) <= max(1, 0.02 * so.iterations)
    assert st.rel_res_recursive < 1e-6
    xh = _h(x)
    bt = o.rhs()
    true = np.linalg.norm(-bt - o.matvec(xh)) / np.linalg.norm(bt)
    assert true < 1.05e-6
    assert abs(true - st.rel_res_true) <= 1e-9
    n = min(len(st.trace_res), len(tro), 20)
    assert np.allclose(st.trace_res[:n], tro[:n], rtol=1e-6, atol=0)


# ---------------------------------------------------------------- Algorithm 2


@pytest.mark.parametrize("N,tau", [(1, 10.0), (4, 10.0), (16, 3.3), (16, 0.0)])
def test_mcg_fixed_iterations(pair, N, tau):
    name, p, o, g = pair
    if N > p.n_cams:
        pytest.skip("more subsets than cameras")
    k = 8
    x, st = g.mcg(N, tau, eps=0.0, max_iter=k, trace=True)
    xo, so, tro = o.mcg(N, tau, eps=0.0, imax=k, trace=True)
    assert st.iterations == so.iterations == k
    assert np.array_equal(st.trace_k, tro[:, 2].astype(np.int32))
    assert st.multi_steps == so.multi_steps
    assert relnorm(_h(x), xo) < 1e-9


@pytest.mark.parametrize("N,tau", [(4, 10.0), (16, 3.3)])
def test_mcg_converged(pair, N, tau):
    name, p, o, g = pair
    if N > p.n_cams:
        pytest.skip("more subsets than cameras")
    S, xs = dense(name, o)
    x, st = g.mcg(N, tau, eps=1e-10, max_iter=3000)
    xo, so = o.mcg(N, tau, eps=1e-10, imax=3000)
    assert st.status == ba.BA_OK and so.status == oracle.OK
    assert energy_err(S, _h(x), xs) <= converged_gate(name, o, S, xs, xo)


@pytest.mark.parametrize("N,tau", [(4, 10.0), (16, 3.3)])
def test_mcg_to_1e6(pair, N, tau):
    name, p, o, g = pair
    if N > p.n_cams:
        pytest.skip("more subsets than cameras")
    x, st = g.mcg(N, tau, trace=True)
    xo, so, tro = o.mcg(N, tau, trace=True)
    assert st.status == ba.BA_OK
    assert abs(st.iterations - so.iterations) <= max(1, 0.02 * so.iterations)
    xh = _h(x)
    bt = o.rhs()
    assert np.linalg.norm(-bt - o.matvec(xh)) / np.linalg.norm(bt) < 1.05e-6
    n = min(len(st.trace_res), len(tro), 5)
    assert np.allclose(st.trace_res[:n], tro[:n, 0], rtol=1e-6, atol=0)
    # branch decisions agree wherever t_i is not within rounding of tau
    n = min(len(st.trace_k), len(tro)) - 1
    near = np.abs(tro[:n, 1] - tau) <= 1e-6 * max(tau, 1.0)
    assert np.all((st.trace_k[:n] == tro[:n, 2]) | near)


# ---------------------------------------------------------------- edge cases


def test_zero_rhs_and_warm_start():
    p = synth.tiny(n_cams=4, n_lms=30, seed=1)
    p.r[:] = 0.0
    g = ba.System.from_problem(p)
    x, st = g.pcg()
    assert st.iterations == 0 and st.status == ba.BA_OK and not torch.any(x)
    x, st = g.mcg(2, 10.0)
    assert st.iterations == 0 and not torch.any(x)
    g.close()
    p = synth.config0(seed=3)
    o = oracle.System(p)
    g = ba.System.from_problem(p)
    xo, _ = o.pcg(eps=1e-6)
    x0 = _dev(xo)
    x, st = g.pcg(x0=x0, eps=1e-3)
    xr, sr = o.pcg(x0=xo, eps=1e-3)
    assert st.iterations == sr.iterations
    assert relnorm(_h(x), xr) < 1e-9
    g.close()


def test_single_iteration_and_every_camera_its_own_subset(ring):
    p, o, g = ring
    x, st = g.pcg(max_iter=1)
    assert st.iterations == 1 and st.status == ba.BA_MAXITER
    N = p.n_cams
    x, st = g.mcg(N, 1e9, eps=0.0, max_iter=3, trace=True)
    xo, so, tro = o.mcg(N, 1e9, eps=0.0, imax=3, trace=True)
    assert st.multi_steps == so.multi_steps == 3
    assert relnorm(_h(x), xo) < 1e-9


def test_history_capacity_error(ring):
    p, o, g = ring
    with pytest.raises(ba.BAError) as e:
        g.mcg(8, 1e9, max_iter=50, max_history_cols=10)
    assert e.value.status == ba.BA_ERR_WORKSPACE


def test_invalid_subset_count(ring):
    p, o, g = ring
    for N in (0, p.n_cams + 1):
        with pytest.raises(ba.BAError) as e:
            g.mcg(N, 1.0)
        assert e.value.status == ba.BA_ERR_INVALID_ARG
    with pytest.raises(ba.BAError):
        g.mcg(2, -1.0)


def test_build_errors():
    p = synth.tiny(n_cams=4, n_lms=20, seed=0)
    q = synth.tiny(n_cams=4, n_lms=20, seed=0)
    q.J_l[2, 0, 1] = np.inf
    with pytest.raises(ba.BAError) as e:
        ba.System.from_problem(q)
    assert e.value.status == ba.BA_ERR_NONFINITE
    q = synth.tiny(n_cams=4, n_lms=20, seed=0)
    q.obs_cam[1], q.obs_lm[1] = q.obs_cam[0], q.obs_lm[0]
    with pytest.raises(ba.BAError) as e:
        ba.System.from_problem(q)
    assert e.value.status == ba.BA_ERR_INVALID_ARG
    q = synth.tiny(n_cams=4, n_lms=20, seed=0)
    q.obs_cam[0] = 7
    with pytest.raises(ba.BAError) as e:
        ba.System.from_problem(q)
    assert e.value.status == ba.BA_ERR_INVALID_ARG
    q = synth.tiny(n_cams=4, n_lms=20, seed=0)
    q.n_cams = 5
    with pytest.raises(ba.BAError) as e:
        ba.System.from_problem(q)
    assert e.value.status == ba.BA_ERR_NOT_SPD
    q = synth.ring_problem(n_cams=70, n_lms=10, c_lo=65, c_hi=65, seed=0)
    with pytest.raises(ba.BAError) as e:
        ba.System.from_problem(q)
    assert e.value.status == ba.BA_ERR_UNSUPPORTED
    g = ba.System.from_problem(p)
    g.close()


# ---------------------------------------------------------------- A11 mixed precision


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
@pytest.mark.parametrize("solver", ["pcg", "mcg", "mcg_h32"])
def test_mixed_precision_refinement(pair, prec, solver):
    """FP64 refinement around reduced-precision S products: the result meets the FP64
    residual target, and run to 1e-10 its error against the dense solution is <= 1e-6
    (energy norm) -- the stated bound for the mixed form.  mcg_h32: MCG whose
    reorthogonalisation reads the FP32 copy of the history (ba_solve_opts.history_fp32, the
    default), mcg: the FP64 history."""
    name, p, o, g = pair
    N = min(4, p.n_cams)
    run = (lambda **kw: g.pcg(precision=prec, **kw)) if solver == "pcg" else \
        (lambda **kw: g.mcg(N, 10.0, precision=prec, history_fp32=solver == "mcg_h32", **kw))   # mcg: FP64 history
    x, st = run(max_iter=5000, max_outer=40)
    bt = o.rhs()
    xh = _h(x)
    true = np.linalg.norm(-bt - o.matvec(xh)) / np.linalg.norm(bt)
    assert abs(true - st.rel_res_true) <= 1e-9 + 1e-9 * true      # the reported residual is the true one
    if prec == "bf16" and name == "tiny":
        # kappa(S) = 3e9: the BF16 operator's relative error (2^-8) times the conditioning
        # exceeds 1, so refinement cannot contract; the solver must say so, not claim success
        assert st.status == ba.BA_MAXITER and true >= 1e-6, st
        return
    assert st.status == ba.BA_OK, st
    assert true < 1e-6
    assert st.refinement_steps >= 1
    S, xs = dense(name, o)
    x, st = run(eps=1e-10, max_iter=20000, max_outer=60)
    ev = np.linalg.eigvalsh(S)
    u = 2.0 ** -24 if prec == "fp32" else 2.0 ** -8
    if ev[-1] / ev[0] * u >= 1.0:
        # refinement contracts only while kappa(S) times the operator's relative error is
        # below 1; past that (tiny: kappa = 3e9) reaching 1e-10 depends on rounding, and a
        # solver that stops must report its true residual
        true = np.linalg.norm(-bt - o.matvec(_h(x))) / np.linalg.norm(bt)
        assert abs(true - st.rel_res_true) <= 1e-9 + 1e-9 * true
        assert st.status == ba.BA_OK or (st.status == ba.BA_MAXITER and true < 1e-6), st
        if st.status == ba.BA_MAXITER:
            return
    assert st.status == ba.BA_OK, st
    assert energy_err(S, _h(x), xs) <= 1e-6


def test_fp32_history_copy_keeps_the_conjugation():
    """Mixed-precision MCG reading the FP32 copy of the history (block 0 copied, every later
    block's P and Q written in both precisions by the kernels that finish them) needs about
    as many iterations as with the FP64 history; a stale or missing column of the copy
    would drop its block from the reorthogonalisation and multiply them."""
    p = synth.walk_problem(n_cams=200, n_lms=20000, seed=7, name="walk200")
    g = ba.System.from_problem(p)
    for N in (1, 4, 16):
        _, s64 = g.mcg(N, 3.3, precision="fp32", history_fp32=False)
        _, s32 = g.mcg(N, 3.3, precision="fp32", history_fp32=True)
        assert s64.status == ba.BA_OK and s32.status == ba.BA_OK, (N, s64, s32)
        assert s32.rel_res_true < 1e-6
        assert abs(s32.iterations - s64.iterations) <= 0.05 * s64.iterations + 2, (N, s64, s32)


def test_mcg_history_on_matrix_cores_matches_the_oracle():
    """The matrix-core history products (ba_solve_opts.history_mfma, blocks wider than 16
    columns) give the same iterates as the oracle's Algorithm 2 within 1e-9."""
    p = synth.walk_problem(n_cams=120, n_lms=8000, seed=5, name="walk120")
    o = oracle.System(p)
    g = ba.System.from_problem(p)
    for N in (40, 64):
        x, st = g.mcg(N, 10.0, eps=0.0, max_iter=8, history_mfma=True)
        xo, so = o.mcg(N, 10.0, eps=0.0, imax=8)
        assert st.multi_steps == so.multi_steps and st.multi_steps > 0
        assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) < 1e-9, N
        x2, st2 = g.mcg(N, 10.0, eps=0.0, max_iter=8)
        assert np.linalg.norm(x2.cpu().numpy() - x.cpu().numpy()) / np.linalg.norm(xo) < 1e-11
    x, st = g.mcg(64, 10.0, history_mfma=True)
    assert st.status == ba.BA_OK and st.rel_res_true < 1.05e-6
    g.close()
