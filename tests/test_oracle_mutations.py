"""Planted mistakes in a copy of the oracle must be caught by its pins.

Each case copies the oracle's C source, applies one textual edit that a
plausible slip would produce (a dropped term, a flipped sign, a wrong index, a
transposed operand, a missing reorthogonalisation term), compiles the copy in a
temporary directory and checks that at least one of the dense / textbook /
invariant checks below rejects it.  The real oracle passes the same checks.
"""
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import synth

SRC = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "oracle", "ba_oracle.c")


def _dense(p):
    m, n, nl = p.n_obs, p.n, p.n_lms
    J = np.zeros((2 * m, n + 3 * nl))
    for o in range(m):
        c, l = int(p.obs_cam[o]), int(p.obs_lm[o])
        J[2 * o:2 * o + 2, 9 * c:9 * c + 9] = p.J_p[o]
        J[2 * o:2 * o + 2, n + 3 * l:n + 3 * l + 3] = p.J_l[o]
    JtJ = J.T @ J
    H = JtJ + p.lam * np.diag(np.diag(JtJ))
    b = J.T @ p.r.ravel()
    Hpp, Hpl, Hll = H[:n, :n], H[:n, n:], H[n:, n:]
    S = Hpp - Hpl @ np.linalg.solve(Hll, Hpl.T)
    bt = b[:n] - Hpl @ np.linalg.solve(Hll, b[n:])
    return H, b, S, bt


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def run_pins(libobj):
    """Return the names of the checks that fail for the oracle as built (with any planted mistake)."""
    failed = []
    p = synth.tiny(n_cams=5, n_lms=40, seed=2, c_hi=5)
    p.lam = 1e-2
    H, b, S, bt = _dense(p)
    n = p.n
    try:
        o = oracle.System(p, libobj=libobj)
    except oracle.OracleError:
        return ["build"]
    Sd = np.empty((n, n))
    for j in range(n):
        e = np.zeros(n)
        e[j] = 1.0
        Sd[:, j] = o.matvec(e)
    if _rel(Sd, S) > 1e-10:
        failed.append("S")
    if _rel(o.rhs(), bt) > 1e-10:
        failed.append("rhs")
    D = o.D_blocks()
    if max(_rel(D[c], S[9 * c:9 * c + 9, 9 * c:9 * c + 9]) for c in range(p.n_cams)) > 1e-10:
        failed.append("D")
    full = np.linalg.solve(H, -b)
    if _rel(o.back_substitute(full[:n]), full[n:]) > 1e-8:
        failed.append("backsub")
    z = o.precond(bt)
    zr = np.concatenate([np.linalg.solve(S[9 * c:9 * c + 9, 9 * c:9 * c + 9], bt[9 * c:9 * c + 9])
                         for c in range(p.n_cams)])
    if _rel(z, zr) > 1e-8:
        failed.append("precond")
    # PCG against SciPy's textbook CG at a fixed iteration count
    A = spla.LinearOperator((n, n), matvec=lambda v: S @ v, dtype=np.float64)
    M = spla.LinearOperator((n, n), matvec=lambda v: zr_apply(S, v, p.n_cams), dtype=np.float64)
    its = []
    spla.cg(A, -bt, x0=np.zeros(n), rtol=0.0, atol=0.0, maxiter=8, M=M,
            callback=lambda xk: its.append(np.array(xk)))
    x, st = o.pcg(eps=0.0, imax=8)
    if np.linalg.norm(x - its[-1]) > 1e-8 * np.linalg.norm(its[-1]):
        failed.append("pcg")
    # MCG: Galerkin property with the returned direction history
    for N, tau in ((3, 1e9), (2, 1e9)):
        xm, sm, tr, P = o.mcg(N, tau, eps=0.0, imax=4, trace=True, history=True)
        P = P[:, :sm.history_cols - int(tr[-1, 2])]
        xg = P @ np.linalg.lstsq(P.T @ S @ P, P.T @ (-bt), rcond=1e-13)[0]
        if not np.all(np.isfinite(xm)) or np.linalg.norm(S @ (xm - xg)) > 1e-7 * np.linalg.norm(bt):
            failed.append(f"mcg-galerkin-{N}")
            break
    xs = np.linalg.solve(S, -bt)
    xm, sm = o.mcg(3, 10.0, eps=1e-12, imax=2000)
    if not np.all(np.isfinite(xm)) or np.linalg.norm(xm - xs) > 1e-6 * np.linalg.norm(xs):
        failed.append("mcg-converge")
    # pseudo-inverse
    rng = np.random.default_rng(3)
    Qm, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    lam = np.array([2.0, 1.0, 0.5, 3.0, 0.0, 0.0])
    Am = (Qm * lam) @ Qm.T
    Am = 0.5 * (Am + Am.T)
    Ap = np.empty((6, 6))
    eig = np.empty(6)
    import ctypes as C
    dp = C.POINTER(C.c_double)
    libobj.or_pinv(6, np.ascontiguousarray(Am).ctypes.data_as(dp), Ap.ctypes.data_as(dp),
                   eig.ctypes.data_as(dp))
    if _rel(Ap, np.linalg.pinv(Am, rcond=1e-10, hermitian=True)) > 1e-9:
        failed.append("pinv")
    return failed


def zr_apply(S, v, nc):
    return np.concatenate([np.linalg.solve(S[9 * c:9 * c + 9, 9 * c:9 * c + 9], v[9 * c:9 * c + 9])
                           for c in range(nc)])


MUTANTS = {
    "no_U_damping": ("for (int i = 0; i < dp; ++i) U[i * dp + i] += lambda * U[i * dp + i];", ""),
    "no_V_damping": ("for (int i = 0; i < 3; ++i) V[i * 3 + i] += lambda * V[i * 3 + i];", ""),
    "rhs_sign": ("bt[i] -= w[i * 3 + 0] * vb[0]", "bt[i] += w[i * 3 + 0] * vb[0]"),
    "matvec_transposed_W": ("g[j] += w[i * 3 + j] * vc[i];\n        }\n        const double *Vi = s->Vinv + (size_t)l * 9;\n        for (int i = 0; i < 3; ++i) h[",
                            "g[j] += w[(i % 3) * 3 + (j % 3)] * vc[i];\n        }\n        const double *Vi = s->Vinv + (size_t)l * 9;\n        for (int i = 0; i < 3; ++i) h["),
    "matvec_drop_U": ("for (int j = 0; j < dp; ++j) a += U[i * dp + j] * vc[j];", "(void)U;"),
    "matvec_Vinv_transposed_index": ("h[(size_t)l * 3 + i] = Vi[i * 3 + 0] * g[0] + Vi[i * 3 + 1] * g[1] + Vi[i * 3 + 2] * g[2];",
                                     "h[(size_t)l * 3 + i] = Vi[0 * 3 + i] * g[0] + Vi[0 * 3 + i] * g[1] + Vi[2 * 3 + i] * g[2];"),
    "pcg_beta_sign": ("for (int i = 0; i < n; ++i) P[i] = Z[i] - beta * P[i];",
                      "for (int i = 0; i < n; ++i) P[i] = Z[i] + beta * P[i];"),
    "pcg_alpha_uses_Q": ("double Delta = dot(Q, P, n), gamma = dot(P, r, n);",
                         "double Delta = dot(Q, P, n), gamma = dot(Q, r, n);"),
    "backsub_printed_sign": ("for (int j = 0; j < 3; ++j) g[j] = s->bl[(size_t)l * 3 + j];",
                             "for (int j = 0; j < 3; ++j) g[j] = -s->bl[(size_t)l * 3 + j];"),
    "mcg_no_full_reorth": ("for (int j = 0; j < nb; ++j) {\n            blk_t *Bj = &H[j];",
                           "for (int j = nb - 1; j < nb; ++j) {\n            blk_t *Bj = &H[j];"),
    "mcg_beta_without_pinv": ("for (int b = 0; b < kj; ++b) t += Bj->Dp[a * kj + b] * Phi[(size_t)b * kn + p];",
                              "t = Phi[(size_t)a * kn + p];"),
    "mcg_split_wrong_group": ("Z[(size_t)group[c] * n + (size_t)c * dp + q] = z[(size_t)c * dp + q];",
                              "Z[(size_t)((group[c] + 1) % kn) * n + (size_t)c * dp + q] = z[(size_t)c * dp + q];"),
    "pinv_rotation_sign": ("a[r * k + p] = c * arp - s * arq;", "a[r * k + p] = c * arp + s * arq;"),
    "pinv_keeps_null_space": ("if (!(fabs(l) > thr)) continue;", "if (l == 0.0) l = 1e-300;"),
    "precond_lower_only": ("for (int i = k - 1; i >= 0; --i) {\n        double s = x[i];",
                           "for (int i = -1; i >= 0; --i) {\n        double s = x[i];"),
    "D_missing_schur_term": ("D[i * dp + j] -= WV[i * 3 + 0] * w[j * 3 + 0]", "D[i * dp + j] -= 0.0 * WV[i * 3 + 0] * w[j * 3 + 0]"),
}


def test_real_oracle_passes_pins():
    assert run_pins(oracle.lib()) == []


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation anchor for {name} not found"
    mutated = src.replace(old, new, 1)
    cpath = tmp_path / "mut.c"
    cpath.write_text(mutated)
    so = tmp_path / "libmut.so"
    subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-w", "-o", str(so),
                           str(cpath), "-lm"])
    lib = oracle.load(str(so))
    failed = run_pins(lib)
    assert failed, f"planted mistake {name} went unnoticed"
