"""Training and evaluation of the learned low-rank preconditioner M^-1 = D^-1 + U U^T.

The network (47 -> 128 tanh -> 72, FP32 weights) maps per-camera features of the
reduced camera system (its 9x9 diagonal block, covisibility degree and lambda) to
U_c = L_c^-T Uh_c, a global rank-8 correction of the block-Jacobi preconditioner
D(S) of Sec. 3.2.  It is trained on the reduced camera systems that the solver
itself produces along Levenberg-Marquardt runs (Sec. 4.1), with the probe loss
    1/(P n) sum_k |w_k - s_k - Uh (Uh^T s_k)|^2,   s_k = L^-1 S L^-T w_k,
a Hutchinson estimate of |I - (I + Uh Uh^T) L^-1 S L^-T|_F^2 / n.  Every step runs in
the library's kernels: features, S products, block scaling, forward, backward and Adam
on the device, BF16 matrix-core inference when the solver uses the network.
"""
from __future__ import annotations

import dataclasses
import time
from typing import Callable, Dict, List, Optional

import numpy as np

import synth
from . import System, mlp_forward, mlp_loss_grad, adam_step, MLP_PARAMS

N_PROBES = 8          # probes per system and gradient call


def _torch():
    import torch
    return torch


def training_problem(seed: int, n_cams: int = 250) -> synth.Problem:
    """A banded walk problem shaped like the 1,936-camera configuration (336 landmarks per
    camera, about 8 observers per landmark within a window of 20 cameras), scaled down."""
    return synth.walk_problem(n_cams=n_cams, n_lms=336 * n_cams, seed=seed, name=f"walk{n_cams}s{seed}")


def lm_run(p: synth.Problem, lm_iters: int = 5, visit: Optional[Callable] = None, eps: float = 1e-6):
    """Levenberg-Marquardt iterations on p (Sec. 4.1): solve the reduced camera system with
    block-Jacobi PCG, back-substitute, accept the step if F decreases (lambda / 10) or
    raise lambda (x 10).  visit(problem, system) sees every linear system on the way.
    Returns the final problem and the list of costs."""
    costs = [synth.cost(p)]
    for _ in range(lm_iters):
        g = System.from_problem(p)
        try:
            if visit is not None:
                visit(p, g)
            x, st = g.pcg(eps=eps, max_iter=2000)
            dxl = g.back_substitute(x)
            q = synth.relinearize(p, x.cpu().numpy(), dxl.cpu().numpy())
        finally:
            g.close()
        fq = synth.cost(q)
        if fq < costs[-1]:
            p = dataclasses.replace(q, lam=max(q.lam / 10.0, 1e-12))
            costs.append(fq)
        else:
            p = dataclasses.replace(p, lam=p.lam * 10.0)
            costs.append(costs[-1])
    return p, costs


def probe_pairs(g: System, n_probes: int = N_PROBES, seed: int = 0):
    """W (n x P, row-major) of N(0, 1) probes and Sw = L^-1 S L^-T W (scaled coordinates)."""
    torch = _torch()
    gen = torch.Generator(device=g.device).manual_seed(int(seed))
    W = torch.randn(g.n, n_probes, dtype=torch.float64, device=g.device, generator=gen)
    cols = []
    for k in range(n_probes):
        y = g.matvec(g.block_scale(W[:, k].contiguous(), transpose=True))
        cols.append(g.block_scale(y))
    return W.contiguous(), torch.stack(cols, 1).contiguous()


@dataclasses.dataclass
class Sample:
    F: object        # features [n_cams, 47] FP32 (device)
    W: object        # probes [n, P] FP64 (device)
    Sw: object       # scaled products [n, P] FP64 (device)


def collect(seeds, lm_iters: int = 5, n_cams: int = 250, n_probes: int = N_PROBES) -> List[Sample]:
    """Training samples: every system met along LM runs of the given seeds."""
    out: List[Sample] = []

    def visit(p, g):
        W, Sw = probe_pairs(g, n_probes, seed=int(p.seed) * 100 + len(out) if hasattr(p, "seed") else len(out))
        out.append(Sample(g.lowrank_features(), W, Sw))

    for s in seeds:
        lm_run(training_problem(int(s), n_cams), lm_iters, visit)
    return out


def _collect_worker(args):
    """Worker process: the samples of its seeds, saved as CPU tensors to path."""
    seeds, lm_iters, n_cams, path = args
    torch = _torch()
    torch.cuda.set_device(0)
    got = collect(seeds, lm_iters, n_cams)
    torch.save([(s.F.cpu(), s.W.cpu(), s.Sw.cpu()) for s in got], path)
    return len(got)


def _plain_learned_iters_worker(args):
    """Worker process: iterations to eps of plain and learned MCG on held-out seeds."""
    seeds, params_path, n_cams, N, tau = args
    torch = _torch()
    torch.cuda.set_device(0)
    params = torch.load(params_path, weights_only=True).to("cuda")
    rows = []
    for sd in seeds:
        g = System.from_problem(training_problem(int(sd), n_cams))
        try:
            x, st0 = g.mcg(N, tau, eps=1e-6)
            g.set_lowrank_from_mlp(mlp_forward(params, g.lowrank_features(), bf16=True))
            x, st1 = g.mcg(N, tau, eps=1e-6, precond="lowrank")
            rows.append({"seed": int(sd), "plain_iters": st0.iterations, "learned_iters": st1.iterations,
                         "plain_status": st0.status, "learned_status": st1.status,
                         "plain_res": st0.rel_res_true, "learned_res": st1.rel_res_true})
        finally:
            g.close()
    return rows


def _pool(workers: int):
    """Worker processes, started before this process touches the GPU."""
    import multiprocessing as mp
    return mp.get_context("spawn").Pool(workers)


def _split(seq, k):
    seq = list(seq)
    return [seq[i::k] for i in range(k) if seq[i::k]]


def mean_loss(params, samples: List[Sample]) -> float:
    return float(np.mean([mlp_loss_grad(params, s.F, s.W, s.Sw)[0] for s in samples]))


def train(samples: List[Sample], epochs: int = 20, lr: float = 1e-4, seed: int = 0, params=None,
          log: Optional[Callable[[str], None]] = None) -> Dict[str, object]:
    """Adam over the samples (one system per step, shuffled every epoch)."""
    torch = _torch()
    dev = samples[0].F.device
    if params is None:
        params = torch.from_numpy(synth.mlp_init(seed)).to(device=dev, dtype=torch.float32)
    m = torch.zeros(MLP_PARAMS, dtype=torch.float32, device=dev)
    v = torch.zeros_like(m)
    rng = np.random.default_rng(seed)
    hist = [mean_loss(params, samples)]
    t = 0
    t0 = time.perf_counter()
    for ep in range(epochs):
        for i in rng.permutation(len(samples)):
            s = samples[int(i)]
            _, grad = mlp_loss_grad(params, s.F, s.W, s.Sw)
            t += 1
            adam_step(params, grad, m, v, t, lr)
        hist.append(mean_loss(params, samples))
        if log:
            log(f"epoch {ep + 1}: mean probe loss {hist[-1]:.5f}")
    torch.cuda.synchronize()
    return {"params": params, "loss_history": hist, "steps": t, "train_s": time.perf_counter() - t0}


def solve_compare(p: synth.Problem, params, N: int = 16, tau: float = 3.3, eps: float = 1e-6,
                  reps: int = 2) -> Dict[str, float]:
    """Iterations and time to eps for block-Jacobi MCG and for MCG with the learned term
    (feature extraction, BF16 inference and U included in the learned time)."""
    torch = _torch()
    g = System.from_problem(p)
    try:
        def plain():
            return g.mcg(N, tau, eps=eps)

        def learned():
            g.set_lowrank_from_mlp(mlp_forward(params, g.lowrank_features(), bf16=True))
            return g.mcg(N, tau, eps=eps, precond="lowrank")

        res = {}
        for name, f in (("plain", plain), ("learned", learned)):
            f()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                x, st = f()
            torch.cuda.synchronize()
            res[f"{name}_ms"] = (time.perf_counter() - t0) / reps * 1e3
            res[f"{name}_iters"] = st.iterations
            res[f"{name}_status"] = st.status
            res[f"{name}_res"] = st.rel_res_true
        return res
    finally:
        g.close()


def evaluate(params, seeds, n_cams: int = 250, N: int = 16, tau: float = 3.3) -> Dict[str, object]:
    rows = [solve_compare(training_problem(int(s), n_cams), params, N, tau) for s in seeds]
    agg = {k: float(np.mean([r[k] for r in rows])) for k in rows[0] if not k.endswith("status")}
    agg["all_converged"] = all(r["plain_status"] == 0 and r["learned_status"] == 0 for r in rows)
    agg["systems"] = len(rows)
    agg["rows"] = rows
    return agg


def main(argv=None):
    import argparse
    import json
    import os
    import tempfile
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--train-seeds", type=int, default=40)
    ap.add_argument("--eval-seeds", type=int, default=20)
    ap.add_argument("--timed-seeds", type=int, default=20, help="held-out seeds also timed, one process alone")
    ap.add_argument("--lm-iters", type=int, default=5)
    ap.add_argument("--n-cams", type=int, default=250)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--lr", type=float, default=1e-4)
    ap.add_argument("--workers", type=int, default=8, help="processes generating systems (each uses the GPU)")
    ap.add_argument("--out", default=None, help="JSON summary")
    ap.add_argument("--params-out", default=None, help="trained weights (torch.save of an FP32 tensor)")
    a = ap.parse_args(argv)
    log = lambda s: print(f"[learned] {s}", flush=True)
    tmp = tempfile.mkdtemp(prefix="lowrank_")
    pool = _pool(a.workers) if a.workers > 1 else None
    t0 = time.perf_counter()
    parts = _split(range(a.train_seeds), a.workers)
    jobs = [(pt, a.lm_iters, a.n_cams, os.path.join(tmp, f"part{i}.pt")) for i, pt in enumerate(parts)]
    if pool:
        pool.map(_collect_worker, jobs)
    else:
        for j in jobs:
            _collect_worker(j)
    torch = _torch()
    samples = []
    for j in jobs:
        for F, W, Sw in torch.load(j[3], weights_only=True):
            samples.append(Sample(F.cuda(), W.cuda(), Sw.cuda()))
        os.remove(j[3])
    gen_s = time.perf_counter() - t0
    log(f"{len(samples)} training systems from {a.train_seeds} seeds in {gen_s:.1f} s")
    tr = train(samples, a.epochs, a.lr, log=log)
    params_path = a.params_out or os.path.join(tmp, "params.pt")
    torch.save(tr["params"].detach().cpu(), params_path)
    # held-out iterations in the worker processes (iteration counts do not depend on timing)
    held = list(range(10_000, 10_000 + a.eval_seeds))
    t1 = time.perf_counter()
    ejobs = [(pt, params_path, a.n_cams, 16, 3.3) for pt in _split(held, a.workers)]
    rows = [r for part in (pool.map(_plain_learned_iters_worker, ejobs) if pool else
                           [_plain_learned_iters_worker(j) for j in ejobs]) for r in part]
    if pool:
        pool.close()
        pool.join()
    rows.sort(key=lambda r: r["seed"])
    pi = np.array([r["plain_iters"] for r in rows], dtype=float)
    li = np.array([r["learned_iters"] for r in rows], dtype=float)
    held_out = {"systems": len(rows), "plain_iters_mean": float(pi.mean()), "learned_iters_mean": float(li.mean()),
                "iters_change": float(li.mean() / pi.mean() - 1.0),
                "learned_fewer_or_equal": int((li <= pi).sum()),
                "all_converged": all(r["plain_status"] == 0 and r["learned_status"] == 0 for r in rows),
                "eval_s": round(time.perf_counter() - t1, 1)}
    # time on a subset, this process alone on the GPU
    timed = evaluate(tr["params"], held[:a.timed_seeds], a.n_cams) if a.timed_seeds > 0 else None
    summary = {"n_cams": a.n_cams, "n_lms": 336 * a.n_cams, "train_seeds": a.train_seeds,
               "train_systems": len(samples), "generation_s": round(gen_s, 1), "epochs": a.epochs,
               "steps": tr["steps"], "train_s": round(tr["train_s"], 2), "loss_first": tr["loss_history"][0],
               "loss_last": tr["loss_history"][-1], "held_out": held_out,
               "timed": None if timed is None else {k: v for k, v in timed.items() if k != "rows"}}
    log(json.dumps(summary))
    if a.out:
        with open(a.out, "w") as f:
            json.dump({"summary": summary, "loss_history": tr["loss_history"], "held_out_rows": rows}, f, indent=1)


if __name__ == "__main__":
    main()
