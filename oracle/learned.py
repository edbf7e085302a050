"""FP64 oracle of the learned low-rank correction of the block-Jacobi preconditioner.

TEST INFRASTRUCTURE (see oracle/__init__.py).  Plain NumPy, written from the
definitions below; shares nothing with the HIP kernels.

The paper's preconditioner is block Jacobi, D(S) (Sec. 3.2, before Alg. 1).  The
learned part adds a global rank-8 term:
    M^-1 = D^-1 + U U^T,   U = [U_1; ...; U_np] (n x 8),   U_c = L_c^-T Uh_c,
where D_c = L_c L_c^T is camera c's diagonal block of S and Uh_c (9 x 8) is the
output of a 2-layer MLP (47 -> 128 tanh -> 72) applied to 47 scale-free
features of camera c.  M^-1 is symmetric positive definite for any weights.

Features of camera c (47):
  36  correlations C_ij = D_ij / sqrt(D_ii D_jj), i < j, of the block D_c
   9  relative log scales log D_ii - mean_k log D_kk
   1  log(1 + number of other cameras sharing a landmark with c)
   1  log(max(lambda, 1e-12))

Training loss over probes w_k (n-vectors, scaled coordinates: Sh = L^-1 S L^-T,
s_k = Sh w_k precomputed):
    loss = 1/(P n) sum_k | w_k - s_k - Uh (Uh^T s_k) |^2
i.e. a Hutchinson estimate of |I - (I + Uh Uh^T) Sh|_F^2 / n, the scaled form of
|I - M^-1 S|.  MLP weights: W1 [128, 47], b1 [128], W2 [72, 128], b2 [72].
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

N_FEAT = 47
N_HID = 128
RANK = 8
N_OUT = 9 * RANK


@dataclass
class Weights:
    W1: np.ndarray
    b1: np.ndarray
    W2: np.ndarray
    b2: np.ndarray

    def flat(self) -> np.ndarray:
        return np.concatenate([self.W1.ravel(), self.b1, self.W2.ravel(), self.b2])

    @staticmethod
    def from_flat(v: np.ndarray) -> "Weights":
        a = 0
        W1 = v[a:a + N_HID * N_FEAT].reshape(N_HID, N_FEAT); a += N_HID * N_FEAT
        b1 = v[a:a + N_HID]; a += N_HID
        W2 = v[a:a + N_OUT * N_HID].reshape(N_OUT, N_HID); a += N_OUT * N_HID
        b2 = v[a:a + N_OUT]
        return Weights(W1.copy(), b1.copy(), W2.copy(), b2.copy())


def n_params() -> int:
    return N_HID * N_FEAT + N_HID + N_OUT * N_HID + N_OUT


def covisibility_degree(n_cams: int, obs_cam: np.ndarray, obs_lm: np.ndarray) -> np.ndarray:
    """Number of other cameras that share at least one landmark with each camera."""
    order = np.argsort(obs_lm, kind="stable")
    cam = obs_cam[order].astype(np.int64)
    lm = obs_lm[order]
    starts = np.flatnonzero(np.r_[True, lm[1:] != lm[:-1]])
    ends = np.r_[starts[1:], lm.shape[0]]
    pairs = set()
    for a, b in zip(starts, ends):
        cs = cam[a:b]
        for i in range(len(cs)):
            for j in range(len(cs)):
                if i != j:
                    pairs.add((int(cs[i]), int(cs[j])))
    deg = np.zeros(n_cams)
    for (i, _j) in pairs:
        deg[i] += 1
    return deg


def features(D: np.ndarray, degree: np.ndarray, lam: float) -> np.ndarray:
    """47 features per camera from its 9x9 diagonal block D[c] of S."""
    nc = D.shape[0]
    F = np.empty((nc, N_FEAT))
    iu = np.triu_indices(9, 1)
    for c in range(nc):
        d = np.diag(D[c])
        corr = D[c] / np.sqrt(np.outer(d, d))
        F[c, :36] = corr[iu]
        ld = np.log(d)
        F[c, 36:45] = ld - ld.mean()
        F[c, 45] = np.log1p(degree[c])
        F[c, 46] = np.log(max(lam, 1e-12))
    return F


def mlp_forward(w: Weights, F: np.ndarray):
    """Returns (pre-activation [nc,128], hidden [nc,128], out [nc,72])."""
    pre = F @ w.W1.T + w.b1
    hid = np.tanh(pre)
    out = hid @ w.W2.T + w.b2
    return pre, hid, out


def chol_blocks(D: np.ndarray) -> np.ndarray:
    return np.linalg.cholesky(D)


def U_from_out(out: np.ndarray, L: np.ndarray) -> np.ndarray:
    """U (n x 8): U_c = L_c^-T Uh_c with Uh_c = out[c] reshaped 9 x 8 (row-major)."""
    nc = out.shape[0]
    Uh = out.reshape(nc, 9, RANK)
    U = np.stack([np.linalg.solve(L[c].T, Uh[c]) for c in range(nc)])
    return U.reshape(nc * 9, RANK)


def apply_precond(D: np.ndarray, U: np.ndarray, r: np.ndarray) -> np.ndarray:
    """M^-1 r = D^-1 r + U (U^T r)."""
    nc = D.shape[0]
    z = np.concatenate([np.linalg.solve(D[c], r[9 * c:9 * c + 9]) for c in range(nc)])
    return z + U @ (U.T @ r)


def loss_and_grad_Uh(Uh: np.ndarray, W: np.ndarray, Sw: np.ndarray):
    """Loss of the probes (columns of W, scaled coordinates) and d loss / d Uh (n x 8)."""
    n, P = W.shape
    T = Uh.T @ Sw                      # 8 x P
    E = W - Sw - Uh @ T                # n x P
    loss = float((E * E).sum()) / (P * n)
    G = -2.0 * (E @ T.T + Sw @ (E.T @ Uh)) / (P * n)
    return loss, G


def loss_and_grad(w: Weights, F: np.ndarray, W: np.ndarray, Sw: np.ndarray):
    """Loss for one system and the analytic gradient of every weight (backpropagation)."""
    pre, hid, out = mlp_forward(w, F)
    nc = F.shape[0]
    Uh = out.reshape(nc * 9, RANK)
    loss, GU = loss_and_grad_Uh(Uh, W, Sw)
    g_out = GU.reshape(nc, N_OUT)
    gW2 = g_out.T @ hid
    gb2 = g_out.sum(0)
    g_hid = g_out @ w.W2
    g_pre = g_hid * (1.0 - hid * hid)
    gW1 = g_pre.T @ F
    gb1 = g_pre.sum(0)
    return loss, Weights(gW1, gb1, gW2, gb2)


def init_weights(seed: int, scale_out: float = 1e-2) -> Weights:
    """The seeded initial weights of the input generator (synth.mlp_init)."""
    import synth
    return Weights.from_flat(synth.mlp_init(seed, scale_out))


def adam_step(w: Weights, g: Weights, m: np.ndarray, v: np.ndarray, t: int, lr=1e-3, b1=0.9, b2=0.999,
              eps=1e-8) -> Weights:
    """One Adam update of the flattened weights (m, v updated in place); t counts from 1."""
    p = w.flat()
    gf = g.flat()
    m *= b1
    m += (1 - b1) * gf
    v *= b2
    v += (1 - b2) * gf * gf
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return Weights.from_flat(p - lr * mh / (np.sqrt(vh) + eps))
