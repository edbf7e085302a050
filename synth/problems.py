"""Seeded synthetic bundle-adjustment problems.

This module only sets up problems: camera geometry, the 9-parameter camera
model, analytic Jacobians and residuals evaluated at a perturbed state.  It
holds none of the solver's arithmetic (normal equations, Schur complement,
preconditioners, Krylov iterations); the CPU oracle and the HIP path both
consume its output and nothing else from each other.

Camera model (9 parameters per pose, the intrinsics-estimating case of the
paper's state vector, Sec. 3 before eq. (1)): axis-angle rotation w, translation
t, focal f, radial k1, k2.  A world point X maps to camera coordinates
P = R(w) X + t, normalised p = (P_x, P_y) / P_z with P_z > 0, and pixels
u = f (1 + k1 |p|^2 + k2 |p|^4) p (principal point at 0).  The residual of an
observation is u - u_obs.

Jacobians are taken with respect to a local 9-parameter update of each camera:
a left rigid-motion increment (R, t) <- (exp([dw]x) R, exp([dw]x) t + dt), which
rotates about the camera centre, additive increments of f, k1, k2; and additive
increments of the 3 landmark coordinates.  Each observation
contributes one 2x9 pose block and one 2x3 landmark block (the per-residual
split of J = (J_p J_l), eq. (2)-(5)).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

NOISE_PX = 1.0          # projection noise, pixels (sigma)
PERTURB_SIGMA = 1e-2    # perturbation of every camera parameter / coordinate
LAMBDA_DEFAULT = 1e-4   # LM damping at the first LM iteration (Sec. 4.1)


@dataclass
class Problem:
    """One linearised BA problem: per-observation Jacobian blocks and residuals."""
    name: str
    seed: int
    n_cams: int
    n_lms: int
    obs_cam: np.ndarray          # int32 [m]
    obs_lm: np.ndarray           # int32 [m]
    J_p: np.ndarray              # float64 [m, 2, 9]
    J_l: np.ndarray              # float64 [m, 2, 3]
    r: np.ndarray                # float64 [m, 2]
    lam: float = LAMBDA_DEFAULT
    # geometry at the linearisation point (for an outer LM loop)
    cams: Optional[Dict[str, np.ndarray]] = None   # R [np,3,3], t, f, k1, k2
    points: Optional[np.ndarray] = None            # [nl, 3]
    u_obs: Optional[np.ndarray] = None             # [m, 2]
    info: Dict[str, float] = field(default_factory=dict)

    @property
    def n_obs(self) -> int:
        return int(self.obs_cam.shape[0])

    @property
    def d_p(self) -> int:
        """Pose dimension: 9 (extrinsics and intrinsics) or 6 (extrinsics only)."""
        return int(self.J_p.shape[-1])

    @property
    def n(self) -> int:
        return self.d_p * self.n_cams


# ---------------------------------------------------------------------------
# camera model


def skew(a: np.ndarray) -> np.ndarray:
    """[a]x for a batch of 3-vectors, shape [..., 3] -> [..., 3, 3]."""
    z = np.zeros_like(a[..., 0])
    return np.stack([
        np.stack([z, -a[..., 2], a[..., 1]], -1),
        np.stack([a[..., 2], z, -a[..., 0]], -1),
        np.stack([-a[..., 1], a[..., 0], z], -1)], -2)


def so3_exp(w: np.ndarray) -> np.ndarray:
    """Rotation matrices exp([w]x) for a batch of axis-angle vectors (Rodrigues)."""
    w = np.asarray(w, dtype=np.float64)
    th = np.linalg.norm(w, axis=-1)[..., None, None]
    K = skew(w)
    small = th < 1e-8
    th_s = np.where(small, 1.0, th)
    a = np.where(small, 1.0 - th ** 2 / 6.0, np.sin(th_s) / th_s)
    b = np.where(small, 0.5 - th ** 2 / 24.0, (1.0 - np.cos(th_s)) / th_s ** 2)
    eye = np.broadcast_to(np.eye(3), K.shape)
    return eye + a * K + b * (K @ K)


def project(cams: Dict[str, np.ndarray], X: np.ndarray, cam: np.ndarray, lm: np.ndarray):
    """Pixel coordinates and the two Jacobian blocks of every observation.

    Returns (u [m,2], J_p [m,2,9], J_l [m,2,3], Pz [m]).
    """
    R = cams["R"][cam]                       # [m,3,3]
    RX = np.einsum("mij,mj->mi", R, X[lm])   # rotated point
    P = RX + cams["t"][cam]
    z = P[:, 2]
    iz = 1.0 / z
    p = P[:, :2] * iz[:, None]
    rho2 = np.einsum("mi,mi->m", p, p)
    f = cams["f"][cam]
    k1 = cams["k1"][cam]
    k2 = cams["k2"][cam]
    s = 1.0 + k1 * rho2 + k2 * rho2 * rho2
    u = (f * s)[:, None] * p
    # du/dp = f (s I + (2 k1 + 4 k2 rho2) p p^T)
    ds = 2.0 * k1 + 4.0 * k2 * rho2
    dudp = (f * ds)[:, None, None] * (p[:, :, None] * p[:, None, :])
    dudp[:, 0, 0] += f * s
    dudp[:, 1, 1] += f * s
    # dp/dP = [[1/z, 0, -x/z^2], [0, 1/z, -y/z^2]]
    dpdP = np.zeros((P.shape[0], 2, 3))
    dpdP[:, 0, 0] = iz
    dpdP[:, 1, 1] = iz
    dpdP[:, 0, 2] = -p[:, 0] * iz
    dpdP[:, 1, 2] = -p[:, 1] * iz
    A = np.einsum("mij,mjk->mik", dudp, dpdP)          # du/dP [m,2,3]
    J_p = np.empty((P.shape[0], 2, 9))
    J_p[:, :, 0:3] = -np.einsum("mij,mjk->mik", A, skew(P))    # left rigid-motion increment
    J_p[:, :, 3:6] = A
    J_p[:, :, 6] = s[:, None] * p
    J_p[:, :, 7] = (f * rho2)[:, None] * p
    J_p[:, :, 8] = (f * rho2 * rho2)[:, None] * p
    J_l = np.einsum("mij,mjk->mik", A, R)
    return u, J_p, J_l, z


def look_at(C: np.ndarray, target: np.ndarray, up=(0.0, 0.0, 1.0)) -> np.ndarray:
    """World-to-camera rotations whose optical (z) axis points from C to target."""
    zc = target - C
    zc /= np.linalg.norm(zc, axis=-1, keepdims=True)
    upv = np.broadcast_to(np.asarray(up, dtype=np.float64), zc.shape)
    xc = np.cross(zc, upv)
    xc /= np.linalg.norm(xc, axis=-1, keepdims=True)
    yc = np.cross(zc, xc)
    return np.stack([xc, yc, zc], axis=-2)


def _cams_from_Rc(R: np.ndarray, C: np.ndarray, rng: np.random.Generator) -> Dict[str, np.ndarray]:
    n = R.shape[0]
    t = -np.einsum("nij,nj->ni", R, C)
    return {"R": R, "t": t,
            "f": rng.uniform(400.0, 600.0, n),
            "k1": rng.normal(0.0, 1e-3, n),
            "k2": rng.normal(0.0, 1e-3, n)}


def _perturb(cams, X, rng):
    n = cams["R"].shape[0]
    dw = rng.normal(0.0, PERTURB_SIGMA, (n, 3))
    E = so3_exp(dw)
    est = {"R": np.einsum("nij,njk->nik", E, cams["R"]),
           "t": np.einsum("nij,nj->ni", E, cams["t"]) + rng.normal(0.0, PERTURB_SIGMA, (n, 3)),
           "f": cams["f"] + rng.normal(0.0, PERTURB_SIGMA, n),
           "k1": cams["k1"] + rng.normal(0.0, PERTURB_SIGMA, n),
           "k2": cams["k2"] + rng.normal(0.0, PERTURB_SIGMA, n)}
    Xe = X + rng.normal(0.0, PERTURB_SIGMA, X.shape)
    return est, Xe


def _finish(name, seed, rng, cams, X, cam, lm, lam, info, shuffle=False, noise_px=NOISE_PX) -> Problem:
    """Observe with noise at the true state, linearise at a perturbed state."""
    u_true, _, _, _ = project(cams, X, cam, lm)
    u_obs = u_true + rng.normal(0.0, noise_px, u_true.shape)
    est, Xe = _perturb(cams, X, rng)
    u, J_p, J_l, _ = project(est, Xe, cam, lm)
    r = u - u_obs
    cam = cam.astype(np.int32)
    lm = lm.astype(np.int32)
    if shuffle:
        perm = rng.permutation(cam.shape[0])
        cam, lm, J_p, J_l, r, u_obs = cam[perm], lm[perm], J_p[perm], J_l[perm], r[perm], u_obs[perm]
    info = dict(info)
    info["obs_per_landmark_mean"] = cam.shape[0] / max(1, X.shape[0])
    return Problem(name=name, seed=seed, n_cams=cams["R"].shape[0], n_lms=X.shape[0],
                   obs_cam=np.ascontiguousarray(cam), obs_lm=np.ascontiguousarray(lm),
                   J_p=np.ascontiguousarray(J_p), J_l=np.ascontiguousarray(J_l),
                   r=np.ascontiguousarray(r), lam=lam, cams=est, points=Xe, u_obs=u_obs,
                   info=info)


def _topc(keys: np.ndarray, c: np.ndarray) -> np.ndarray:
    """Column indices of the c[i] smallest keys of each row (ragged), row-major."""
    order = np.argsort(keys, axis=1, kind="stable")
    take = np.arange(keys.shape[1])[None, :] < c[:, None]
    return order, take


# ---------------------------------------------------------------------------
# problem families


def ring_problem(n_cams=50, n_lms=5000, c_lo=2, c_hi=8, radius=20.0, half=5.0, seed=0,
                 lam=LAMBDA_DEFAULT, name="ring", shuffle=False, noise_px=NOISE_PX) -> Problem:
    """Cameras on a ring in z=0 facing the origin, landmarks uniform in a cube.

    Every landmark is seen by c ~ U{c_lo..c_hi} cameras, the ones nearest to it in
    azimuth.  radius > sqrt(3)*half keeps every landmark in front of every camera.
    noise_px = 0 gives exact observations of the true state (same random stream).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    th = 2.0 * np.pi * np.arange(n_cams) / n_cams
    C = np.stack([radius * np.cos(th), radius * np.sin(th), np.zeros(n_cams)], -1)
    R = look_at(C, np.zeros_like(C))
    cams = _cams_from_Rc(R, C, rng)
    X = rng.uniform(-half, half, (n_lms, 3))
    c = rng.integers(c_lo, min(c_hi, n_cams) + 1, n_lms)
    phi = np.arctan2(X[:, 1], X[:, 0])
    lm = np.repeat(np.arange(n_lms), c)
    cam = _ring_nearest(phi, th, c, c_hi)
    return _finish(name, seed, rng, cams, X, cam, lm, lam, {"geometry": 0.0}, shuffle, noise_px)


def _ring_nearest(phi: np.ndarray, th: np.ndarray, c: np.ndarray, c_hi: int, full: bool = False) -> np.ndarray:
    """The c[i] cameras nearest in azimuth to each landmark, nearest first, flattened.

    The cameras are evenly spaced, so the nearest ones form an arc around the
    closest camera: only a window of 2 (c_hi + 2) + 1 candidates is ranked (the
    full ranking gives the same cameras in the same order; `full` forces it)."""
    n = th.shape[0]
    w = c_hi + 2
    if full or 2 * w + 1 >= n:
        cand = np.broadcast_to(np.arange(n)[None, :], (phi.shape[0], n))
    else:
        k0 = np.rint(phi / (2.0 * np.pi / n)).astype(np.int64)
        cand = (k0[:, None] + np.arange(-w, w + 1)[None, :]) % n
    d = np.abs(np.angle(np.exp(1j * (phi[:, None] - th[cand]))))
    order, take = _topc(d, c)
    return np.take_along_axis(cand, order, 1)[take]


def walk_problem(n_cams=1936, n_lms=650_000, c_max=60, geo_p=1.0 / 7.0, window=10,
                 seed=0, lam=LAMBDA_DEFAULT, name="walk", batch=65536) -> Problem:
    """Cameras along a path-like 3-D random walk, landmarks seen within a camera window.

    The walk takes 1 m steps whose horizontal heading itself random-walks
    (N(0, 0.1 rad) per step) plus N(0, 0.1 m) vertical jitter, so the camera index
    follows the path.  Each camera's optical axis is horizontal and perpendicular
    to the local heading (smoothed over +-15 cameras), all facing the same side.
    A landmark picks an anchor camera a, a depth U[5, 30] m along a's axis and a
    lateral offset inside a's field of view.  Its observer count is
    c = min(c_max, 2 + G), G geometric on {0, 1, ...} with success probability
    geo_p (mean 8 for 1/7).  The observers are the anchor and c-1 distinct cameras
    drawn uniformly among the cameras of [a - w, a + w], w = max(window,
    ceil((c-1)/2)), that see the point in front of them with |p| < 1.2 (c is
    capped by the number of such cameras).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    head_ang = np.cumsum(rng.normal(0.0, 0.1, n_cams))
    steps = np.stack([np.cos(head_ang), np.sin(head_ang), rng.normal(0.0, 0.1, n_cams)], -1)
    C = np.cumsum(steps, axis=0)
    C -= C.mean(axis=0)
    k = np.arange(n_cams)
    hw = 15
    lo = np.clip(k - hw, 0, n_cams - 1)
    hi = np.clip(k + hw, 0, n_cams - 1)
    head = C[hi] - C[lo]
    head[:, 2] = 0.0
    head /= np.linalg.norm(head, axis=1, keepdims=True)
    up = np.array([0.0, 0.0, 1.0])
    zc = np.cross(head, up)
    zc /= np.linalg.norm(zc, axis=1, keepdims=True)
    R = look_at(C, C + zc)
    cams = _cams_from_Rc(R, C, rng)

    Xs: List[np.ndarray] = []
    cams_l: List[np.ndarray] = []
    cnt_l: List[np.ndarray] = []
    have = 0
    W = 2 * max(window, c_max // 2) + 1
    off = np.arange(W) - W // 2
    while have < n_lms:
        nb = min(batch, n_lms - have)
        a = rng.integers(0, n_cams, nb)
        depth = rng.uniform(5.0, 30.0, nb)
        lat = rng.uniform(-0.4, 0.4, (nb, 2)) * depth[:, None]
        Ra = R[a]
        X = C[a] + depth[:, None] * Ra[:, 2, :] + lat[:, :1] * Ra[:, 0, :] + lat[:, 1:] * Ra[:, 1, :]
        c = np.minimum(c_max, 2 + rng.geometric(geo_p, nb) - 1)
        w = np.maximum(window, c // 2)
        cand = a[:, None] + off[None, :]
        inr = (np.abs(off)[None, :] <= w[:, None]) & (cand >= 0) & (cand < n_cams)
        cc = np.clip(cand, 0, n_cams - 1)
        P = np.einsum("nkij,nkj->nki", R[cc], X[:, None, :] - C[cc])
        vis = (P[..., 2] > 1.0) & (np.abs(P[..., 0]) < 1.2 * P[..., 2]) & \
              (np.abs(P[..., 1]) < 1.2 * P[..., 2])
        ok = inr & vis
        keys = rng.random((nb, W))
        keys[~ok] = 2.0
        keys[:, W // 2] = -1.0                                # the anchor always observes
        c = np.minimum(c, ok.sum(1))
        order, take = _topc(keys, c)
        cidx = np.take_along_axis(cand, order, 1)
        good = c >= 2
        Xs.append(X[good])
        cams_l.append(cidx[good][take[good]])
        cnt_l.append(c[good])
        have += int(good.sum())
    X = np.concatenate(Xs)[:n_lms]
    cnt = np.concatenate(cnt_l)[:n_lms]
    cam = np.concatenate(cams_l)[:int(cnt.sum())]
    lm = np.repeat(np.arange(n_lms), cnt)
    return _finish(name, seed, rng, cams, X, cam, lm, lam, {"geometry": 1.0})


def cap_problem(n_cams=571, n_lms=100_000, c_min=5, c_max=40, geo_p=0.2, zipf_s=1.2,
                radius=30.0, seed=0, lam=LAMBDA_DEFAULT, name="cap", batch=32768) -> Problem:
    """Cameras on a spherical cap looking at a central site, Zipf camera popularity.

    Cameras at distance `radius` with polar angle in [10, 60] degrees (uniform on
    the cap) look at a jittered point of the site; landmarks are uniform in a
    12 x 12 x 4 m box.  A landmark has c = min(c_max, c_min + G) observers (G
    geometric on {0, 1, ...}, success probability geo_p), drawn without
    replacement with probability proportional to rank^-zipf_s, where the ranks
    are a seeded permutation of the cameras.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    ct = rng.uniform(np.cos(np.radians(60.0)), np.cos(np.radians(10.0)), n_cams)
    st = np.sqrt(1.0 - ct ** 2)
    az = rng.uniform(0.0, 2.0 * np.pi, n_cams)
    C = radius * np.stack([st * np.cos(az), st * np.sin(az), ct], -1)
    target = rng.normal(0.0, 1.0, (n_cams, 3)) * np.array([1.0, 1.0, 0.3])
    R = look_at(C, target)
    cams = _cams_from_Rc(R, C, rng)
    X = rng.uniform(-1.0, 1.0, (n_lms, 3)) * np.array([6.0, 6.0, 2.0])
    rank = rng.permutation(n_cams) + 1
    logw = -zipf_s * np.log(rank.astype(np.float64))
    c = np.minimum(c_max, c_min + rng.geometric(geo_p, n_lms) - 1)
    c = np.minimum(c, n_cams)
    cam_parts = []
    for s0 in range(0, n_lms, batch):
        s1 = min(n_lms, s0 + batch)
        g = rng.gumbel(0.0, 1.0, (s1 - s0, n_cams))
        keys = -(logw[None, :] + g)                      # Gumbel top-k = sampling w/o replacement
        part = np.argpartition(keys, c_max - 1, axis=1)[:, :c_max] if c_max < n_cams else \
            np.tile(np.arange(n_cams), (s1 - s0, 1))
        pk = np.take_along_axis(keys, part, 1)
        o = np.argsort(pk, axis=1, kind="stable")
        part = np.take_along_axis(part, o, 1)
        take = np.arange(part.shape[1])[None, :] < c[s0:s1, None]
        cam_parts.append(part[take])
    cam = np.concatenate(cam_parts)
    lm = np.repeat(np.arange(n_lms), c)
    return _finish(name, seed, rng, cams, X, cam, lm, lam, {"geometry": 2.0})


# ---------------------------------------------------------------------------
# the named workloads


def config0(seed=0, **kw) -> Problem:
    """50 ring cameras, 5,000 landmarks, 2-8 observers each (~25k observations)."""
    return ring_problem(n_cams=50, n_lms=5000, c_lo=2, c_hi=8, seed=seed, name="ring50", **kw)


def config1(seed=0, **kw) -> Problem:
    """F-1936-shaped banded problem: 1,936 cameras, 650k landmarks, ~5.2M observations."""
    return walk_problem(n_cams=1936, n_lms=650_000, seed=seed, name="walk1936", **kw)


def config2(seed=0, **kw) -> Problem:
    """Alamo-shaped dense-Schur problem: 571 cameras, 100k landmarks, ~0.9M observations."""
    return cap_problem(n_cams=571, n_lms=100_000, seed=seed, name="cap571", **kw)


def config4_sizes(seed=0, count=64, lo=50, hi=800) -> np.ndarray:
    """Camera counts of the batch workload (config4) without generating it."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(lo, hi + 1, count)


def _config4_member(args) -> Problem:
    n, s, kw = args
    return ring_problem(n_cams=int(n), n_lms=200 * int(n), c_lo=2, c_hi=20, radius=20.0, seed=int(s),
                        name=f"ring{n}", **kw)


def config4(seed=0, count=64, lo=50, hi=800, workers: int = 1, **kw) -> List[Problem]:
    """Batch of uneven ring problems: cameras ~ U{lo..hi}, 200 landmarks per camera,
    2-20 observers per landmark.  Each problem has its own seed, so `workers`
    processes generate exactly the same problems."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.integers(lo, hi + 1, count)
    seeds = rng.integers(0, 2 ** 31 - 1, count)
    jobs = [(int(n), int(s), kw) for n, s in zip(sizes, seeds)]
    if workers <= 1:
        return [_config4_member(j) for j in jobs]
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_config4_member, jobs))


def tiny(n_cams=4, n_lms=30, seed=0, c_lo=2, c_hi=4, **kw) -> Problem:
    """A problem small enough to form every matrix densely."""
    return ring_problem(n_cams=n_cams, n_lms=n_lms, c_lo=c_lo, c_hi=c_hi, seed=seed,
                        name=f"tiny{n_cams}x{n_lms}", **kw)


def schur_block_density(p: Problem) -> float:
    """Fraction of nonzero 9x9 blocks of the reduced camera system (diagonal included):
    cameras j, k are coupled iff they observe a common landmark."""
    order = np.argsort(p.obs_lm, kind="stable")
    cam = p.obs_cam[order].astype(np.int64)
    lm = p.obs_lm[order]
    starts = np.flatnonzero(np.r_[True, lm[1:] != lm[:-1]])
    counts = np.diff(np.r_[starts, lm.shape[0]])
    pairs = set()
    n = p.n_cams
    pair_codes = []
    for L in np.unique(counts):
        sel = starts[counts == L]
        blk = cam[sel[:, None] + np.arange(L)[None, :]]          # [k, L]
        code = blk[:, :, None] * n + blk[:, None, :]
        pair_codes.append(np.unique(code.ravel()))
    if pair_codes:
        pairs = np.unique(np.concatenate(pair_codes))
        nnz = pairs.shape[0]
    else:
        nnz = 0
    return nnz / float(n * n)


# ---------------------------------------------------------------------------
# outer Levenberg-Marquardt loop support (Sec. 4.1): moving the state by a solved
# step and linearising again.  No solver arithmetic lives here; the step comes from
# whichever solver the caller runs.


def extrinsics_only(p: Problem) -> Problem:
    """The same problem with the intrinsics (f, k1, k2) held fixed: poses of dimension
    d_p = 6 (Sec. 3.1), i.e. the first six columns of every pose block."""
    return Problem(name=p.name + "_dp6", seed=p.seed, n_cams=p.n_cams, n_lms=p.n_lms, obs_cam=p.obs_cam,
                   obs_lm=p.obs_lm, J_p=np.ascontiguousarray(p.J_p[:, :, :6]), J_l=p.J_l, r=p.r, lam=p.lam,
                   cams=p.cams, points=p.points, u_obs=p.u_obs, info=dict(p.info, d_p=6))


def camera_array(cams: Dict[str, np.ndarray]) -> np.ndarray:
    """The cameras as rows of 15 numbers: R row-major (9), t (3), f, k1, k2."""
    n = cams["R"].shape[0]
    return np.ascontiguousarray(np.concatenate([cams["R"].reshape(n, 9), cams["t"], cams["f"][:, None],
                                                cams["k1"][:, None], cams["k2"][:, None]], axis=1))


def cost(p: Problem) -> float:
    """F(x) = |r(x)|^2 at the problem's linearisation point (eq. (1))."""
    return float(np.einsum("mi,mi->", p.r, p.r))


def relinearize(p: Problem, dx_p: np.ndarray, dx_l: np.ndarray, lam: Optional[float] = None) -> Problem:
    """The problem linearised at the state moved by the step (dx_p, dx_l).

    Camera c's 9 step entries follow J_p's parametrisation: a left rigid motion
    (rotation vector w, translation dt: R <- exp(w) R, t <- exp(w) t + dt), then f,
    k1, k2 added; points move by dx_l.  Observations and their pixels are kept.
    """
    if p.cams is None or p.points is None or p.u_obs is None:
        raise ValueError("the problem carries no linearisation state")
    d = np.asarray(dx_p, dtype=np.float64).reshape(p.n_cams, 9)
    E = so3_exp(d[:, 0:3])
    cams = {"R": np.einsum("nij,njk->nik", E, p.cams["R"]),
            "t": np.einsum("nij,nj->ni", E, p.cams["t"]) + d[:, 3:6],
            "f": p.cams["f"] + d[:, 6], "k1": p.cams["k1"] + d[:, 7], "k2": p.cams["k2"] + d[:, 8]}
    X = p.points + np.asarray(dx_l, dtype=np.float64).reshape(p.n_lms, 3)
    cam = p.obs_cam.astype(np.int64)
    lm = p.obs_lm.astype(np.int64)
    u, J_p, J_l, _ = project(cams, X, cam, lm)
    return Problem(name=p.name, seed=p.seed, n_cams=p.n_cams, n_lms=p.n_lms, obs_cam=p.obs_cam,
                   obs_lm=p.obs_lm, J_p=np.ascontiguousarray(J_p), J_l=np.ascontiguousarray(J_l),
                   r=np.ascontiguousarray(u - p.u_obs), lam=p.lam if lam is None else float(lam),
                   cams=cams, points=X, u_obs=p.u_obs, info=dict(p.info))


# ---------------------------------------------------------------------------
# seeded initial weights of the learned preconditioner's 47 -> 128 -> 72 MLP


def mlp_init(seed: int = 0, scale_out: float = 1e-2) -> np.ndarray:
    """Flat initial parameters W1 [128, 47], b1 [128], W2 [72, 128], b2 [72] (float64):
    W1 ~ N(0, 1/47), W2 ~ N(0, (scale_out)^2 / 128), biases 0."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.normal(0.0, 1.0 / np.sqrt(47), (128, 47))
    W2 = rng.normal(0.0, scale_out / np.sqrt(128), (72, 128))
    return np.concatenate([W1.ravel(), np.zeros(128), W2.ravel(), np.zeros(72)])
