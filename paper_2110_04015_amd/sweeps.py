"""Sensitivity of Algorithm 2 to tau, to N and to the density of S on synthetic problems
(the studies of Sec. 4.2: Figs. 3, 4 and 5).

As in Sec. 4.2, the runtime of a solver on a problem is the total time of all the
linear solves of one bundle adjustment run (the LM loop of Sec. 4.1, ba_lm_solve)
from the generator's perturbed state until the loop stops, and the quantity studied
is the ratio t_MCG / t_PCG.  The problems are a series of increasing density
d = (nonzero 9x9 blocks of S) / n_cams^2: cameras on a ring seeing their nearest
neighbours, a random-walk trajectory, and cameras on a spherical cap with Zipf
popularity of decreasing exponent.

Usage: python -m paper_2110_04015_amd.sweeps [--quick] [--implicit-only] > sweeps.jsonl
"""
from __future__ import annotations

import argparse
import json
import sys
import time
from typing import Dict, List, Sequence

import synth

from . import BAError, Scene

TAUS = (0.0, 0.5, 1.0, 2.0, 3.3, 5.0, 10.0, 30.0, 1e9)
NS = (2, 4, 8, 16, 32, 64)


def density_series(seed: int = 1, n_cams: int = 240) -> List[synth.Problem]:
    """Problems of increasing Schur density (about 5%, 16%, 33%, 55%, 95% and 100% at 240 cameras)."""
    c = n_cams
    return [synth.ring_problem(n_cams=c, n_lms=125 * c, c_lo=2, c_hi=6, seed=seed, name="ring"),
            synth.walk_problem(n_cams=c, n_lms=170 * c, c_max=12, seed=seed, name="walk_c12"),
            synth.walk_problem(n_cams=c, n_lms=170 * c, seed=seed, name="walk"),
            synth.cap_problem(n_cams=c, n_lms=125 * c, zipf_s=2.0, seed=seed, name="cap_zipf2"),
            synth.cap_problem(n_cams=c, n_lms=125 * c, zipf_s=1.2, seed=seed, name="cap_zipf1.2"),
            synth.cap_problem(n_cams=c, n_lms=125 * c, zipf_s=0.6, seed=seed, name="cap_zipf0.6")]


def _run(scene, cams, X, **kw) -> Dict[str, float]:
    _, _, st = scene.lm(cams, X, **kw)
    return {"t_solve_ms": st.t_solve_ms, "t_total_ms": st.t_total_ms, "lm_iterations": st.iterations,
            "solver_iterations": st.solver_iterations, "cost": st.cost, "status": st.status}


def sweep_problem(p, taus: Sequence[float] = TAUS, Ns: Sequence[int] = NS, tau_fixed: float = 3.3,
                  N_fixed: int = 16, explicit: bool = False, emit=print) -> None:
    """Emits one record per run: the PCG reference, then MCG over taus at N_fixed and
    over Ns at tau_fixed, each with its ratio to PCG."""
    sc, cams, X = Scene.from_problem(p)
    d = synth.schur_block_density(p)
    base = dict(problem=p.name, n_cams=p.n_cams, n_obs=p.n_obs, density=round(d, 4),
                representation="explicit" if explicit else "implicit")
    try:
        _run(sc, cams, X, solver="pcg", explicit_schur=explicit)           # warm-up (allocations, code)
        ref = _run(sc, cams, X, solver="pcg", explicit_schur=explicit)
    except BAError as e:
        emit(dict(base, error=str(e)))
        return
    emit(dict(base, solver="pcg", **ref))
    runs = [("tau", t, dict(N=min(N_fixed, p.n_cams), tau=t)) for t in taus]
    runs += [("N", n, dict(N=n, tau=tau_fixed)) for n in Ns if n <= p.n_cams]
    for kind, val, kw in runs:
        r = _run(sc, cams, X, solver="mcg", explicit_schur=explicit, **kw)
        emit(dict(base, solver="mcg", sweep=kind, value=val, N=kw["N"], tau=kw["tau"],
                  ratio=round(r["t_solve_ms"] / ref["t_solve_ms"], 4), **r))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--n-cams", type=int, default=240)
    ap.add_argument("--quick", action="store_true", help="three problems, fewer tau and N values")
    ap.add_argument("--implicit-only", action="store_true")
    ap.add_argument("--taus", default=None, help="comma-separated tau values ('' for none)")
    ap.add_argument("--ns", default=None, help="comma-separated N values ('' for none)")
    args = ap.parse_args(argv)
    t0 = time.time()
    probs = density_series(args.seed, args.n_cams)
    if args.quick:
        probs = [probs[0], probs[2], probs[4]]
    taus = (0.0, 1.0, 3.3, 10.0, 1e9) if args.quick else TAUS
    Ns = (4, 16, 64) if args.quick else NS
    if args.taus is not None:
        taus = tuple(float(t) for t in args.taus.split(",") if t.strip())
    if args.ns is not None:
        Ns = tuple(int(n) for n in args.ns.split(",") if n.strip())

    def emit(rec):
        print(json.dumps(rec), flush=True)

    emit({"generated_s": round(time.time() - t0, 2), "problems": [p.name for p in probs]})
    for p in probs:
        for explicit in ((False,) if args.implicit_only else (False, True)):
            sweep_problem(p, taus, Ns, explicit=explicit, emit=emit)
    return 0


if __name__ == "__main__":
    sys.exit(main())
