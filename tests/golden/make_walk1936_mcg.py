"""Writes walk1936_mcg.json: the oracle's MCG (N = 16, tau = 3.3) and PCG solves to a
1e-6 relative residual on the benchmark workload (walk1936, seed 0, FP64).

Calls only the seeded input generator and the oracle.  Takes a few minutes of host
time (OpenMP), so the GPU parity test reads the stored record instead of rerunning it.

    python tests/golden/make_walk1936_mcg.py
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle  # noqa: E402
import synth  # noqa: E402


def main():
    t = time.time()
    p = synth.config1(seed=0)
    o = oracle.System(p)
    out = {"problem": "walk1936 (synth.config1, seed 0)", "n_obs": p.n_obs, "eps": 1e-6}
    x, s, tr = o.mcg(16, 3.3, eps=1e-6, imax=1000, trace=True)
    out["mcg_N16_tau3.3"] = {"iterations": s.iterations, "multi_steps": s.multi_steps, "status": s.status,
                             "rel_res_true": s.rel_res_true, "trace_res": tr[:, 0].tolist(),
                             "trace_t": [None if not np.isfinite(v) else float(v) for v in tr[:, 1]],
                             "trace_k": tr[:, 2].astype(int).tolist()}
    x, s, tr = o.pcg(eps=1e-6, imax=1000, trace=True)
    out["pcg"] = {"iterations": s.iterations, "status": s.status, "rel_res_true": s.rel_res_true,
                  "trace_res": tr.tolist()}
    out["oracle_threads"] = oracle.num_threads()
    out["seconds"] = round(time.time() - t, 1)
    with open(os.path.join(HERE, "walk1936_mcg.json"), "w") as f:
        json.dump(out, f)
    print(f"wrote walk1936_mcg.json in {out['seconds']} s", flush=True)


if __name__ == "__main__":
    main()
