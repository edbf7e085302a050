"""Pins of the FP64 CPU oracle against what the paper and the mathematics fix.

None of these re-types the oracle's formulas: the reduced camera system is
checked against a dense J assembled observation by observation and a dense
Schur complement / dense solves done by NumPy; PCG against SciPy's textbook CG;
MCG against the Galerkin property of block conjugate-direction methods; the
pseudo-inverse against LU inverses and the Penrose conditions.
"""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------- dense helpers


def dense_system(p, lam=None):
    """Dense H = J^T J + lam diag(J^T J) and b = J^T r0 (eq. (6)-(12) with Marquardt D)."""
    lam = p.lam if lam is None else lam
    m, n, nl, dp = p.n_obs, p.n, p.n_lms, p.d_p
    J = np.zeros((2 * m, n + 3 * nl))
    for o in range(m):
        c, l = int(p.obs_cam[o]), int(p.obs_lm[o])
        J[2 * o:2 * o + 2, dp * c:dp * c + dp] = p.J_p[o]
        J[2 * o:2 * o + 2, n + 3 * l:n + 3 * l + 3] = p.J_l[o]
    JtJ = J.T @ J
    H = JtJ + lam * np.diag(np.diag(JtJ))
    b = J.T @ p.r.ravel()
    return H, b, n


def dense_schur(H, b, n):
    Hpp, Hpl, Hll = H[:n, :n], H[:n, n:], H[n:, n:]
    X = np.linalg.solve(Hll, np.concatenate([Hpl.T, b[n:, None]], axis=1))
    S = Hpp - Hpl @ X[:, :-1]
    bt = b[:n] - Hpl @ X[:, -1]
    return S, bt


TINY = [dict(n_cams=3, n_lms=12, seed=0), dict(n_cams=4, n_lms=30, seed=1),
        dict(n_cams=5, n_lms=40, seed=2, c_hi=5), dict(n_cams=6, n_lms=25, seed=7, c_hi=3)]


@pytest.fixture(params=[(i, dp) for dp in (9, 6) for i in range(len(TINY))],
                ids=lambda a: f"tiny{a[0]}_dp{a[1]}")
def tiny_case(request):
    i, dp = request.param
    kw = dict(TINY[i])
    shuffle = i % 2 == 1
    p = synth.tiny(shuffle=shuffle, **kw)
    if dp == 6:
        p = synth.extrinsics_only(p)
    H, b, n = dense_system(p)
    S, bt = dense_schur(H, b, n)
    return p, H, b, n, S, bt


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# ---------------------------------------------------------------- A1: build, S, b~


def test_schur_complement_matches_dense(tiny_case):
    p, H, b, n, S, bt = tiny_case
    o = oracle.System(p)
    assert rel(o.dense_S(), S) < 1e-12
    assert rel(o.rhs(), bt) < 1e-12


def test_normal_equation_blocks_match_dense(tiny_case):
    p, H, b, n, S, bt = tiny_case
    o = oracle.System(p)
    U = o.U_blocks()
    dp = p.d_p
    for c in range(p.n_cams):
        assert rel(U[c], H[dp * c:dp * c + dp, dp * c:dp * c + dp]) < 1e-13
    Vi = o.Vinv_blocks()
    for l in range(p.n_lms):
        blk = H[n + 3 * l:n + 3 * l + 3, n + 3 * l:n + 3 * l + 3]
        assert rel(Vi[l] @ blk, np.eye(3)) < 1e-10
    bp, bl = o.bp_bl()
    assert rel(bp, b[:n]) < 1e-13 and rel(bl, b[n:]) < 1e-13
    D = o.D_blocks()
    for c in range(p.n_cams):
        assert rel(D[c], S[dp * c:dp * c + dp, dp * c:dp * c + dp]) < 1e-12


def test_schur_symmetric_positive_definite(tiny_case):
    p, H, b, n, S, bt = tiny_case
    Sd = oracle.System(p).dense_S()
    assert rel(Sd, Sd.T) < 1e-12
    assert np.linalg.eigvalsh(0.5 * (Sd + Sd.T)).min() > 0
    np.linalg.cholesky(0.5 * (Sd + Sd.T))


def test_operator_symmetric_positive_on_dense_problem():
    p = synth.cap_problem(n_cams=60, n_lms=3000, seed=3)
    o = oracle.System(p)
    rng = np.random.default_rng(0)
    for _ in range(3):
        v, w = rng.standard_normal(o.n), rng.standard_normal(o.n)
        Sv, Sw = o.matvec(v), o.matvec(w)
        assert abs(w @ Sv - v @ Sw) <= 1e-12 * np.linalg.norm(Sv) * np.linalg.norm(w)
        assert v @ Sv > 0


def test_damping_scales_with_lambda():
    """U_lambda and V_lambda grow by lambda * diag (eq. (9)-(10)); S changes accordingly."""
    p = synth.tiny(n_cams=4, n_lms=20, seed=5)
    for lam in (0.0, 1e-4, 1e-1):
        H, b, n = dense_system(p, lam)
        S, bt = dense_schur(H, b, n)
        o = oracle.System(p, lam=lam)
        assert rel(o.dense_S(), S) < 1e-11
        assert rel(o.rhs(), bt) < 1e-11


# ---------------------------------------------------------------- x*, eq. (13), (16)


def test_solution_and_corrected_back_substitution(tiny_case):
    p, H, b, n, S, bt = tiny_case
    o = oracle.System(p)
    full = np.linalg.solve(H, -b)                      # eq. (7) solved densely
    dxp = np.linalg.solve(S, -bt)                      # eq. (13)
    assert rel(dxp, full[:n]) < 1e-8
    dxl = o.back_substitute(full[:n])
    assert rel(dxl, full[n:]) < 1e-8
    # the sign printed in eq. (16), -V^-1(-b_l + W^T dx_p), does not reproduce the solve
    Hpl, Hll = H[:n, n:], H[n:, n:]
    printed = -np.linalg.solve(Hll, -b[n:] + Hpl.T @ full[:n])
    assert rel(printed, full[n:]) > 1e-3


# ---------------------------------------------------------------- Algorithm 1


def _scipy_pcg_iterates(o, k):
    n = o.n
    A = spla.LinearOperator((n, n), matvec=o.matvec, dtype=np.float64)
    M = spla.LinearOperator((n, n), matvec=o.precond, dtype=np.float64)
    its = []
    spla.cg(A, -o.rhs(), x0=np.zeros(n), rtol=0.0, atol=0.0, maxiter=k, M=M,
            callback=lambda xk: its.append(np.array(xk)))
    return its


@pytest.mark.parametrize("k,dp", [(1, 9), (5, 9), (25, 9), (5, 6), (25, 6)])
def test_pcg_matches_textbook_cg(k, dp):
    p = synth.config0(seed=1)
    if dp == 6:
        p = synth.extrinsics_only(p)
    o = oracle.System(p)
    ref = _scipy_pcg_iterates(o, k)
    x, st = o.pcg(eps=0.0, imax=k)
    assert st.iterations == k and st.status == oracle.MAXITER
    assert np.linalg.norm(x - ref[-1]) <= 1e-10 * np.linalg.norm(ref[-1])


def test_pcg_energy_error_monotone():
    p = synth.tiny(n_cams=6, n_lms=80, seed=11, c_hi=5)
    o = oracle.System(p)
    S = o.dense_S()
    xs = np.linalg.solve(S, -o.rhs())
    errs = []
    for k in range(1, 30):
        x, _ = o.pcg(eps=0.0, imax=k)
        e = x - xs
        errs.append(e @ S @ e)
    errs = np.array(errs)
    assert np.all(np.diff(errs) <= 1e-10 * errs[0])


def test_pcg_converges_to_dense_solution():
    p = synth.config0(seed=2)
    o = oracle.System(p)
    S = o.dense_S()
    xs = np.linalg.solve(0.5 * (S + S.T), -o.rhs())
    x, st = o.pcg(eps=1e-12, imax=5000)
    assert st.status == oracle.OK
    assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)
    x6, st6 = o.pcg(eps=1e-6)
    assert st6.status == oracle.OK and st6.rel_res_recursive < 1e-6
    assert st6.rel_res_true < 1.01e-6


def test_pcg_zero_rhs_and_warm_start():
    p = synth.tiny(n_cams=4, n_lms=30, seed=1)
    p.r[:] = 0.0
    o = oracle.System(p)
    x, st = o.pcg()
    assert st.iterations == 0 and st.status == oracle.OK and not np.any(x)
    p2 = synth.tiny(n_cams=4, n_lms=30, seed=1)
    o2 = oracle.System(p2)
    xs = np.linalg.solve(o2.dense_S(), -o2.rhs())
    x2, st2 = o2.pcg(x0=xs, eps=1e-6)
    # the stop test is relative to |r_0| (Alg. 1), which is rounding noise here: the
    # iteration may run on, but the iterate stays at x*
    assert st2.rel_res_true < 1e-12
    assert np.linalg.norm(x2 - xs) <= 1e-9 * np.linalg.norm(xs)


# ---------------------------------------------------------------- Algorithm 2


@pytest.mark.parametrize("dp", [9, 6])
def test_mcg_single_subset_is_pcg(dp):
    p = synth.config0(seed=3)
    o = oracle.System(p if dp == 9 else synth.extrinsics_only(p))
    for k in (3, 20):
        xp, _ = o.pcg(eps=0.0, imax=k)
        xm, st = o.mcg(1, 10.0, eps=0.0, imax=k)
        assert st.multi_steps == 0
        assert np.linalg.norm(xm - xp) <= 1e-9 * np.linalg.norm(xp)
    xp, sp = o.pcg()
    xm, sm = o.mcg(1, 10.0)
    assert abs(sp.iterations - sm.iterations) <= 1


def test_mcg_tau_zero_is_pcg():
    o = oracle.System(synth.config0(seed=3))
    xp, _ = o.pcg(eps=0.0, imax=20)
    xm, st, tr = o.mcg(10, 0.0, eps=0.0, imax=20, trace=True)
    assert st.multi_steps == 0 and np.all(tr[:, 2] == 1)
    assert np.linalg.norm(xm - xp) <= 1e-9 * np.linalg.norm(xp)


@pytest.mark.parametrize("N,tau,dp", [(3, 10.0, 9), (6, 3.0, 9), (3, 10.0, 6)])
def test_mcg_galerkin_projection(N, tau, dp):
    """Block CG with full conjugation: x_m = x0 + P (P^T S P)^+ P^T r0 and P^T r_m = 0."""
    p = synth.tiny(n_cams=8, n_lms=120, seed=4, c_hi=5)
    if dp == 6:
        p = synth.extrinsics_only(p)
    o = oracle.System(p)
    S = o.dense_S()
    bt = o.rhs()
    for k in (2, 4):
        x, st, tr, P = o.mcg(N, tau, eps=0.0, imax=k, trace=True, history=True)
        P = P[:, :st.history_cols - (int(tr[-1, 2]) if k == st.iterations else 0)]
        r0 = -bt
        G = P.T @ S @ P
        xg = P @ np.linalg.lstsq(G, P.T @ r0, rcond=1e-13)[0]
        assert np.linalg.norm(S @ (x - xg)) <= 1e-7 * np.linalg.norm(bt)
        rm = -bt - S @ x
        assert np.abs(P.T @ rm).max() <= 1e-7 * np.abs(P).max() * np.linalg.norm(bt)


def test_mcg_blocks_are_S_conjugate():
    p = synth.tiny(n_cams=8, n_lms=120, seed=6, c_hi=5)
    o = oracle.System(p)
    S = o.dense_S()
    x, st, tr, P = o.mcg(4, 1e9, eps=0.0, imax=4, trace=True, history=True)
    ks = [1] + [int(v) for v in tr[:, 2]]
    offs = np.cumsum([0] + ks)
    blocks = [P[:, offs[i]:offs[i + 1]] for i in range(len(ks) - 1)]
    for i in range(len(blocks)):
        for j in range(i):
            Bi, Bj = blocks[i], blocks[j]
            num = np.abs(Bi.T @ S @ Bj).max()
            den = np.sqrt(np.abs(np.diag(Bi.T @ S @ Bi)).max() * np.abs(np.diag(Bj.T @ S @ Bj)).max())
            assert num <= 1e-8 * den


def test_mcg_tau_test_branch_rule():
    o = oracle.System(synth.config0(seed=4))
    x, st, tr = o.mcg(8, 3.0, trace=True)
    t, k = tr[:-1, 1], tr[:-1, 2]
    assert np.all((t < 3.0) == (k == 8))
    assert np.all(t >= 0)
    assert st.multi_steps == int((k == 8).sum())
    assert st.history_cols == 1 + int(k.sum())


def test_mcg_eq19_matches_direct_product():
    o = oracle.System(synth.config0(seed=5))
    xa, sa = o.mcg(10, 10.0, eps=0.0, imax=15, q_mode=0)
    xb, sb = o.mcg(10, 10.0, eps=0.0, imax=15, q_mode=1)
    assert sa.multi_steps > 0
    assert np.linalg.norm(xa - xb) <= 1e-8 * np.linalg.norm(xb)


def test_mcg_converges_to_dense_solution():
    p = synth.config0(seed=6)
    o = oracle.System(p)
    S = o.dense_S()
    xs = np.linalg.solve(0.5 * (S + S.T), -o.rhs())
    for N, tau in ((5, 10.0), (47, 10.0)):
        x, st = o.mcg(N, tau, eps=1e-12, imax=3000)
        assert st.status == oracle.OK
        assert np.linalg.norm(x - xs) <= 1e-6 * np.linalg.norm(xs)
        x6, st6 = o.mcg(N, tau)
        assert st6.status == oracle.OK and st6.rel_res_true < 1.01e-6
        assert st6.multi_steps > 0


def test_mcg_needs_fewer_iterations_than_pcg():
    """The point of the method (Sec. 3.2): an enlarged search space needs fewer iterations."""
    o = oracle.System(synth.config0(seed=7))
    _, sp = o.pcg()
    _, sm = o.mcg(10, 10.0)
    assert sm.iterations < sp.iterations


def test_mcg_rejects_bad_subset_count():
    o = oracle.System(synth.tiny(n_cams=4, n_lms=20, seed=0))
    for N in (0, 5):
        x, st = o.mcg(N, 1.0)
        assert st.status == oracle.ERR_INVALID


# ---------------------------------------------------------------- pseudo-inverse


def test_pinv_full_rank_is_inverse():
    rng = np.random.default_rng(1)
    for k in (1, 2, 5, 16, 47, 64):
        A = rng.standard_normal((k, k))
        A = A @ A.T + k * np.eye(k)
        Ap, rank, eig = oracle.pinv(A)
        assert rank == k
        assert rel(Ap, np.linalg.inv(A)) < 1e-11
        assert rel(np.sort(eig), np.linalg.eigvalsh(A)) < 1e-12


def test_pinv_rank_deficient_penrose():
    rng = np.random.default_rng(2)
    for k, r in ((4, 2), (16, 9), (47, 40), (64, 1)):
        Qm, _ = np.linalg.qr(rng.standard_normal((k, k)))
        lam = np.zeros(k)
        lam[:r] = rng.uniform(0.5, 3.0, r)
        A = (Qm * lam) @ Qm.T
        A = 0.5 * (A + A.T)
        Ap, rank, _ = oracle.pinv(A)
        assert rank == r
        tol = 1e-12 * max(1.0, np.abs(A).max()) * max(1.0, np.abs(Ap).max())
        assert np.abs(A @ Ap @ A - A).max() < tol * 10
        assert np.abs(Ap @ A @ Ap - Ap).max() < tol * 10
        assert np.abs((A @ Ap).T - A @ Ap).max() < 1e-11
        assert np.abs((Ap @ A).T - Ap @ A).max() < 1e-11
        assert rel(Ap, np.linalg.pinv(A, rcond=1e-10, hermitian=True)) < 1e-10


def test_pinv_zero_matrix():
    Ap, rank, _ = oracle.pinv(np.zeros((3, 3)))
    assert rank == 0 and not np.any(Ap)


# ---------------------------------------------------------------- partition (reading)


def _table1():
    rows = []
    with open(os.path.join(HERE, "golden", "table1_problems.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            name, poses, pts, proj, d, N, tau = line.split()
            rows.append((name, int(poses), int(N), float(tau)))
    return rows


def test_partition_invariants():
    for n_cams, N in [(10, 1), (10, 10), (10, 3), (50, 7), (1936, 64)] + \
            [(r[1], r[2]) for r in _table1()]:
        g = oracle.partition(n_cams, N)
        assert g.min() == 0 and g.max() == N - 1
        assert np.all(np.diff(g) >= 0) and np.all(np.diff(g) <= 1)       # contiguous, ordered
        sizes = np.bincount(g, minlength=N)
        assert np.all(sizes > 0)
        assert np.all(sizes[:-1] == sizes[0])                             # N-1 equal subsets
        assert sizes[-1] >= sizes[0] and sizes[-1] < 2 * sizes[0] + N     # the last holds the rest


def test_partition_rejects_bad_counts():
    assert np.all(oracle.partition(5, 0) == -1)
    assert np.all(oracle.partition(5, 6) == -1)


# ---------------------------------------------------------------- failure paths


def test_build_rejects_invalid_inputs():
    p = synth.tiny(n_cams=4, n_lms=20, seed=0)
    q = synth.tiny(n_cams=4, n_lms=20, seed=0)
    q.J_p[3, 1, 4] = np.nan
    with pytest.raises(oracle.OracleError) as e:
        oracle.System(q)
    assert e.value.status == oracle.ERR_NONFINITE
    q = synth.tiny(n_cams=4, n_lms=20, seed=0)
    q.obs_cam[1] = q.obs_cam[0]
    q.obs_lm[1] = q.obs_lm[0]
    with pytest.raises(oracle.OracleError) as e:
        oracle.System(q)
    assert e.value.status == oracle.ERR_INVALID
    q = synth.tiny(n_cams=4, n_lms=20, seed=0)
    q.obs_lm[2] = 20
    with pytest.raises(oracle.OracleError) as e:
        oracle.System(q)
    assert e.value.status == oracle.ERR_INVALID
    # a camera nobody observes gives a zero diagonal block: not SPD for any lambda
    q = synth.tiny(n_cams=4, n_lms=20, seed=0)
    q.n_cams = 5
    with pytest.raises(oracle.OracleError) as e:
        oracle.System(q)
    assert e.value.status == oracle.ERR_NOT_SPD
    assert oracle.System(p).n == 36
