"""Benchmark: reduced-camera-system solves/s on the F-1936-shaped banded workload.

One step = one complete solve of S dx_p = -b~ from x0 = 0 to a 1e-6 relative
residual (all device kernels of the chosen solver; the system is built once,
outside the timed region, with its inputs resident in HBM).  Prints one JSON
line, with the dominant kernel's roofline (algorithmic bytes per launch over its
event-timed average duration) and the CPU oracle's rate on a bounded sample.

    python bench.py [--steps K] [--warmup W] [--solver mcg|pcg] [--N 16] [--tau 3.3]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0       # MI355X HBM3E, vendor figure
COUNTERS = os.path.join(ROOT, "profiles", "schur1_fp64_walk1936_counters.json")
PROFILE_EVERY = 4   # timed launches of the dominant kernel: one in four
KERNEL_SRC = os.path.join(ROOT, "paper_2110_04015_amd", "csrc", "k_schur.hip")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the chunk kernel from committed rocprofv3 counters, or None
    when the counters were taken on another version of the kernel source."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    if c.get("kernel_src_sha256_16") != kernel_hash():
        return None
    return c.get("bytes_per_launch")


def run_batch(probs, seed, log):
    """The batched-serving workload: 64 uneven problems solved in one batch (device-resident
    Algorithm 2 per problem, FP32 products under FP64 refinement, chunk shape from the
    autotuner) against the same problems solved one by one with the single-problem solver."""
    import numpy as np
    import torch
    import paper_2110_04015_amd as ba
    from paper_2110_04015_amd import tune
    N, tau, prec, max_inner = 16, 3.3, "fp32", 300
    t = time.time()
    sample = [probs[i] for i in np.argsort([p.n_cams for p in probs])[::8]]
    tn = tune.tune_chunks(sample, prec)
    log(f"batch: autotuned chunk shape {tn['max_slots']} slots x {tn['max_tiles']} tiles in {time.time() - t:.1f} s")
    t = time.time()
    b = ba.Batch(probs, max_slots=tn["max_slots"], max_tiles=tn["max_tiles"], store_fp32=True)
    torch.cuda.synchronize()
    build_s = time.time() - t
    out = {"workload": f"64 ring problems, cameras U[50,800], 200 landmarks per camera, 2-20 observers "
                       f"({sum(p.n_obs for p in probs)} observations), seed {seed}",
           "solver": f"mcg N={N} tau={tau}, {prec} products + fp64 refinement, eps 1e-6",
           "build_s": round(build_s, 2), "autotune": tn}
    for mode, win in (("eager", 0), ("graph8", 8)):
        b.mcg(N, tau, precision=prec, max_inner=max_inner, graph_window=win)      # warm-up
        runs = []
        for _ in range(3):
            x, st, ms, rc = b.mcg(N, tau, precision=prec, max_inner=max_inner, graph_window=win)
            runs.append((ms, st, rc))
        ms = float(np.median([r[0] for r in runs]))
        done = np.concatenate([[s.done_ms for s in r[1]] for r in runs])
        st = runs[-1][1]
        out[mode] = {"solves_per_s": round(len(probs) / (ms * 1e-3), 2), "makespan_ms": round(ms, 2),
                     "p50_ms": round(float(np.percentile(done, 50)), 2),
                     "p99_ms": round(float(np.percentile(done, 99)), 2),
                     "all_converged": all(r[2] == ba.BA_OK for r in runs),
                     "worst_rel_res_true": max(s.rel_res_true for s in st),
                     "iterations_mean": round(float(np.mean([s.iterations for s in st])), 1)}
        log(f"batch {mode}: {out[mode]}")
    b.close()
    times = []
    for p in probs:
        g = ba.System.from_problem(p, store_fp32=True)
        g.mcg(N, tau, precision=prec, max_inner=max_inner)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, s = g.mcg(N, tau, precision=prec, max_inner=max_inner)
        torch.cuda.synchronize()
        times.append((time.perf_counter() - t1) * 1e3)
        g.close()
    times = np.array(times)
    queued = np.cumsum(times)
    out["one_by_one"] = {"solves_per_s": round(len(probs) / (times.sum() * 1e-3), 2),
                         "makespan_ms": round(float(times.sum()), 2),
                         "p50_ms": round(float(np.percentile(queued, 50)), 2),
                         "p99_ms": round(float(np.percentile(queued, 99)), 2),
                         "service_p50_ms": round(float(np.percentile(times, 50)), 2),
                         "service_p99_ms": round(float(np.percentile(times, 99)), 2)}
    log(f"batch one-by-one: {out['one_by_one']}")
    return out


def run_learned(g, variants, args, log):
    """The learned low-rank correction of the block-Jacobi preconditioner on the headline
    system: a network trained here on the systems of short LM runs over 250-camera
    walk1936-shaped problems (the library's own features, probes, loss, backpropagation and
    Adam), then applied to walk1936 (features, BF16 inference, U: the setup of one
    linearisation) and timed with MCG in FP64 and with FP32 products under FP64
    refinement, and with PCG, against the plain block-Jacobi solves and FP64 PCG of the
    variants."""
    import torch
    from paper_2110_04015_amd import learned as L
    t = time.time()
    samples = L.collect(range(args.learned_seeds), lm_iters=5, n_cams=250)
    torch.cuda.synchronize()
    gen_s = time.time() - t
    tr = L.train(samples, epochs=20, lr=1e-4)
    out = {"train_systems": len(samples), "train_seeds": args.learned_seeds, "n_cams_train": 250,
           "generation_s": round(gen_s, 1), "train_s": round(tr["train_s"], 2),
           "loss_first": tr["loss_history"][0], "loss_last": tr["loss_history"][-1]}
    del samples

    def setup():
        g.set_lowrank_from_mlp(L.mlp_forward(tr["params"], g.lowrank_features(), bf16=True))

    setup()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(3):
        setup()
    torch.cuda.synchronize()
    out["setup_ms"] = round((time.perf_counter() - t1) / 3 * 1e3, 3)
    for name, kw in [("mcg_fp64_N16", dict(N=16, precision="fp64")),
                     ("mcg_fp32_refined_N16", dict(N=16, precision="fp32")),
                     ("mcg_fp32_refined_N4", dict(N=4, precision="fp32")),
                     ("pcg_fp64", dict(N=0, precision="fp64")),
                     ("pcg_fp32_refined", dict(N=0, precision="fp32"))]:
        if kw["N"]:
            f = lambda: g.mcg(kw["N"], args.tau, eps=1e-6, max_iter=1000, precision=kw["precision"],
                              precond="lowrank")
        else:
            f = lambda: g.pcg(eps=1e-6, max_iter=1000, precision=kw["precision"], precond="lowrank")
        f()
        ts = []
        for _ in range(3):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x, s2 = f()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        dt = sorted(ts)[1]   # median of 3
        log(f"learned {name}: solve times {[round(1e3 * t, 2) for t in ts]} ms")
        plain = variants.get(name)
        out[name] = {"solves_per_s": round(1.0 / dt, 3), "iterations": s2.iterations,
                     "multi_steps": s2.multi_steps, "refinement_steps": s2.refinement_steps,
                     "rel_res_true": s2.rel_res_true, "status": s2.status,
                     "plain_iterations": plain["iterations"] if plain else None,
                     "plain_solves_per_s": plain["solves_per_s"] if plain else None}
        log(f"learned {name}: {out[name]}")
    g.set_lowrank(None)
    base = variants["pcg_fp64"]["solves_per_s"]
    out["vs_pcg_fp64"] = {k: round(v["solves_per_s"] / base, 3) for k, v in out.items()
                          if isinstance(v, dict) and "solves_per_s" in v}
    return out


def run_dense(seed, log):
    """The dense-Schur workload: cap571, shaped like Table 1's Alamo row (571 poses, about
    0.9M projections, block density near 0.8), with that row's N = 47 and tau = 10.  FP64
    PCG and MCG, and MCG with FP32 products or BF16-stored Jacobians under FP64
    refinement, each timed to a 1e-6 relative residual.  Errors are against the GPU's
    own FP64 PCG solution at 1e-12 (whose parity with the oracle the tests establish),
    in the energy norm |x - x*|_S / |x*|_S and in the 2-norm."""
    import numpy as np
    import torch
    import paper_2110_04015_amd as ba
    import synth
    N, tau = 47, 10.0
    p = synth.config2(seed=seed)
    t = time.time()
    g = ba.System.from_problem(p, store_fp32=True, store_bf16=True)
    torch.cuda.synchronize()
    out = {"workload": f"cap571: Alamo-shaped dense-Schur synthetic BA ({p.n_cams} cameras, {p.n_lms} landmarks, "
                       f"{p.n_obs} observations, Schur block density {synth.schur_block_density(p):.3f}), seed {seed}",
           "N": N, "tau": tau, "build_s": round(time.time() - t, 3)}
    t = time.time()
    for prec in ("fp64", "fp32", "bf16"):
        g.prepare_mcg(N, prec)
    torch.cuda.synchronize()
    out["mcg_plan_s"] = round(time.time() - t, 3)
    xs, s0 = g.pcg(eps=1e-12, max_iter=5000)
    xs_S = float(torch.dot(xs, g.matvec(xs)))

    def errors(x):
        e = x - xs
        return (float(np.sqrt(max(float(torch.dot(e, g.matvec(e))), 0.0) / xs_S)),
                float(torch.linalg.norm(e) / torch.linalg.norm(xs)))

    legs = [("pcg_fp64", lambda: g.pcg(eps=1e-6, max_iter=1000)),
            ("mcg_fp64", lambda: g.mcg(N, tau, eps=1e-6, max_iter=1000)),
            ("mcg_fp32_refined", lambda: g.mcg(N, tau, eps=1e-6, max_iter=1000, precision="fp32")),
            ("mcg_bf16_refined", lambda: g.mcg(N, tau, eps=1e-6, max_iter=1000, precision="bf16"))]
    for name, f in legs:
        f()
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x, st = f()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        dt = float(np.median(ts))
        ee, e2 = errors(x)
        out[name] = {"solves_per_s": round(1.0 / dt, 2), "ms": round(dt * 1e3, 3), "iterations": st.iterations,
                     "multi_steps": st.multi_steps, "refinement_steps": st.refinement_steps,
                     "rel_res_true": st.rel_res_true, "status": st.status, "energy_err": ee, "rel_err": e2}
        log(f"dense {name}: {out[name]}")
    # S v: the FP64 chunk kernel (event-timed) over the algorithmic bytes of one product;
    # the 182 MB stream fits in the 256 MB Infinity Cache, so this is not an HBM figure
    v = torch.randn(g.n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(v)
    info = g.info()
    for prec in ("fp64", "fp32", "bf16"):
        g.matvec(v, precision=prec, out=y)
        g.profile(True)
        g.profile_read(reset=True)
        for _ in range(50):
            g.matvec(v, precision=prec, out=y)
        kms, nl = g.profile_read(reset=True)
        g.profile(False)
        esz = {"fp64": 8, "fp32": 4, "bf16": 2}[prec]
        by = p.n_obs * (24 * esz + 4) + p.n_lms * 6 * 8 + g.n * 8
        ms = kms / max(nl, 1)
        out[f"matvec_{prec}"] = {"bytes": int(by), "chunk_kernel_ms": round(ms, 5),
                                 "gbs": round(by / (ms * 1e-3) / 1e9, 1), "cache_resident": by < 256e6}
    out["matvec_fp64"]["bytes_reported_by_library"] = info["matvec_bytes_fp64"]
    out["ratio_mcg_fp64_vs_pcg_fp64"] = round(out["mcg_fp64"]["ms"] / out["pcg_fp64"]["ms"], 4)
    log(f"dense matvec: {out['matvec_fp64']}")
    # the paper's representation: S formed explicitly (rows of up to 571 blocks, assembled in pieces)
    t = time.time()
    ge = ba.System.from_problem(p, explicit_schur=True)
    torch.cuda.synchronize()
    ie = ge.explicit_schur_info()
    ex = {"build_s": round(time.time() - t, 3), "nnz_blocks": ie["nnz_blocks"], "bytes": ie["bytes"],
          "assembly_ms": round(ie["assembly_ms"], 3)}
    ms = ge.matvec_timed(v, reps=50, out=y)   # back-to-back launches, events around all 50
    ex["matvec_ms"] = round(ms, 5)
    ex["matvec_gbs"] = round((ie["bytes"] + ge.n * 8 * 2) / (ms * 1e-3) / 1e9, 1) if ms > 0 else None
    for name, f in [("pcg_fp64", lambda: ge.pcg(eps=1e-6, max_iter=1000)),
                    ("mcg_fp64", lambda: ge.mcg(N, tau, eps=1e-6, max_iter=1000))]:
        f()
        ts = []
        for _ in range(5):
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            x, st = f()
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t1)
        dt = float(np.median(ts))
        ee, e2 = errors(x)
        ex[name] = {"solves_per_s": round(1.0 / dt, 2), "ms": round(dt * 1e3, 3), "iterations": st.iterations,
                    "multi_steps": st.multi_steps, "rel_res_true": st.rel_res_true, "status": st.status,
                    "energy_err": ee}
    out["explicit_schur"] = ex
    log(f"dense explicit S: {ex}")
    ge.close()
    g.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--solver", choices=["mcg", "pcg"], default="mcg")
    ap.add_argument("--N", type=int, default=16)
    ap.add_argument("--tau", type=float, default=3.3)
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16"], default="fp64")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--history-mfma", action="store_true",
                    help="MCG history products of blocks wider than 16 columns on the FP64 matrix cores")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-problem batched-serving workload")
    ap.add_argument("--no-lm", action="store_true", help="skip the LM outer-loop runs")
    ap.add_argument("--no-dense", action="store_true", help="skip the dense-Schur (cap571) workload")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned low-rank correction")
    ap.add_argument("--learned-seeds", type=int, default=4,
                    help="250-camera problems whose 5 LM systems train the learned correction")
    ap.add_argument("--dense-only", action="store_true", help="profiling mode: only the dense-Schur workload")
    ap.add_argument("--matvec-only", type=int, default=0, metavar="K",
                    help="profiling mode: K S v products (at --precision) and one 1 GiB copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the solver runs on one GPU; --gpus must be 1",
                          "n_gpus": args.gpus}), flush=True)
        sys.exit(2)

    import numpy as np
    import synth

    batch_probs = None
    if not args.no_batch and not args.matvec_only and not args.dense_only:
        # generated before the GPU is touched: the worker processes are started here
        t = time.time()
        batch_probs = synth.config4(seed=args.seed, workers=16)
        log(f"generated the 64-problem batch ({sum(p.n_obs for p in batch_probs)} observations) "
            f"in {time.time() - t:.1f} s")

    import torch

    import paper_2110_04015_amd as ba

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}), flush=True)
        sys.exit(3)
    torch.cuda.set_device(0)
    if args.dense_only:
        print(json.dumps({"mode": "dense-only", "dense_schur": run_dense(args.seed, log)}), flush=True)
        return
    t = time.time()
    p = synth.config1(seed=args.seed)
    log(f"generated {p.name}: {p.n_cams} cameras, {p.n_lms} landmarks, {p.n_obs} observations "
        f"in {time.time() - t:.1f} s")
    t = time.time()
    g = ba.System.from_problem(p, store_fp32=args.matvec_only > 0 and args.precision == "fp32",
                               store_bf16=args.matvec_only > 0 and args.precision == "bf16")
    torch.cuda.synchronize()
    build_s = time.time() - t
    info = g.info()
    log(f"built system in {build_s:.2f} s: {info}")

    if args.matvec_only:
        v = torch.randn(g.n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(v)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(args.matvec_only):
            g.matvec(v, out=y, precision=args.precision)
        torch.cuda.synchronize()
        t_mv = (time.perf_counter() - t1) / args.matvec_only
        src = torch.empty(1 << 27, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dst.copy_(src)
        torch.cuda.synchronize()
        t_cp = time.perf_counter() - t1
        print(json.dumps({"mode": "matvec-only", "precision": args.precision, "matvecs": args.matvec_only,
                          "ms_per_matvec": 1e3 * t_mv,
                          "copy_bytes_read": src.numel() * 8, "copy_bytes_written": dst.numel() * 8,
                          "copy_ms": 1e3 * t_cp, "info": info}), flush=True)
        g.close()
        return

    # MCG's partition and multidirectional-product plan (host, once per N): timed apart
    plan_s = None
    if args.solver == "mcg":
        t = time.time()
        g.prepare_mcg(args.N, args.precision)
        torch.cuda.synchronize()
        plan_s = time.time() - t
        log(f"MCG plan for N = {args.N} in {plan_s:.3f} s")

    def step(precision=args.precision, solver=args.solver, N=args.N, tau=args.tau):
        if solver == "pcg":
            return g.pcg(eps=1e-6, max_iter=1000, precision=precision)
        return g.mcg(N, tau, eps=1e-6, max_iter=1000, precision=precision, history_mfma=args.history_mfma)

    for i in range(args.warmup):
        x, st = step()
        log(f"warmup {i}: {st.iterations} iterations, {st.multi_steps} multidirectional, "
            f"true rel. residual {st.rel_res_true:.3e}, {st.t_solve_ms:.1f} ms")
    # the events bracket every PROFILE_EVERY-th launch of the dominant kernel: an event
    # record between two kernels costs a few microseconds of idle device
    g.profile(True, every=PROFILE_EVERY)
    g.profile_read(reset=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        x, st = step()
        stats.append(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kms, launches = g.profile_read(reset=True)
    g.profile(False)
    st = stats[-1]
    log(f"timed {args.steps} solves in {wall:.3f} s; last: {st.iterations} iterations, "
        f"true rel. residual {st.rel_res_true:.3e}; chunk kernel {launches} launches, {kms:.1f} ms")
    if st.status != ba.BA_OK or st.rel_res_true > 1.05e-6:
        log(f"WARNING: solve did not reach 1e-6: status {st.status}, residual {st.rel_res_true:.3e}")

    # algorithmic bytes of one chunk-kernel launch: every observation's 2x9 + 2x3 FP64
    # Jacobian blocks and its camera index, every landmark's V^-1 (6 FP64), v once
    esz = {"fp64": 8, "fp32": 4, "bf16": 2}[args.precision]
    bytes_per_launch = p.n_obs * (24 * esz + 4) + p.n_lms * 6 * 8 + p.n * 8
    avg_ms = kms / max(launches, 1)
    achieved = bytes_per_launch / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    roofline = {"bound": "hbm", "kernel": f"k_schur1<{ {'fp64': 0, 'fp32': 1, 'bf16': 2}[args.precision] }, 9>",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "bytes_per_launch": int(bytes_per_launch), "avg_launch_ms": round(avg_ms, 5),
                "launches": int(launches), "timed_every": PROFILE_EVERY}
    # practical ceiling: a pure read of as many bytes in the same access pattern
    ceiling = ba.stream_read_gbs(bytes_per_launch, reps=10)
    roofline["stream_read_ceiling"] = round(ceiling, 1)
    roofline["frac_of_ceiling"] = round(achieved / ceiling, 4)
    log(f"stream-read ceiling {ceiling:.0f} GB/s; chunk kernel at {achieved / ceiling:.3f} of it")

    variants = {}
    mixed_vs_pcg = None
    if not args.no_variants:
        for name, kw in [("pcg_fp64", dict(solver="pcg", precision="fp64")),
                         ("mcg_fp64_N4", dict(solver="mcg", N=4, precision="fp64")),
                         ("mcg_fp64_N16", dict(solver="mcg", N=16, precision="fp64")),
                         ("mcg_fp64_N64", dict(solver="mcg", N=64, precision="fp64")),
                         ("pcg_fp32_refined", dict(solver="pcg", precision="fp32")),
                         ("pcg_bf16_refined", dict(solver="pcg", precision="bf16")),
                         ("mcg_fp32_refined_N16", dict(solver="mcg", N=16, precision="fp32")),
                         ("mcg_fp32_refined_N4", dict(solver="mcg", N=4, precision="fp32")),
                         ("mcg_bf16_refined_N16", dict(solver="mcg", N=16, precision="bf16")),
                         ("mcg_bf16_refined_N4", dict(solver="mcg", N=4, precision="bf16"))]:
            step(**kw)                         # first call: plan, history and precision buffers
            reps = 3
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(reps):
                x, s2 = step(**kw)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t1) / reps
            variants[name] = {"solves_per_s": round(1.0 / dt, 3), "iterations": s2.iterations,
                              "multi_steps": s2.multi_steps, "refinement_steps": s2.refinement_steps,
                              "rel_res_true": s2.rel_res_true, "status": s2.status}
            log(f"variant {name}: {1.0 / dt:.2f} solves/s, {s2.iterations} iterations, "
                f"residual {s2.rel_res_true:.2e}")
        # mixed-precision MCG against plain FP64 PCG on the same GPU (solves/s ratio)
        base = variants["pcg_fp64"]["solves_per_s"]
        mixed_vs_pcg = {k: round(v["solves_per_s"] / base, 3) for k, v in variants.items()
                        if k.startswith("mcg_") and "refined" in k}

    learned = None
    if not args.no_variants and not args.no_learned:
        learned = run_learned(g, variants, args, log)

    extrinsics = None
    if not args.no_variants:
        # poses of dimension 6 (intrinsics fixed): the same observations, 2 x 6 pose blocks
        gx = ba.System.from_problem(synth.extrinsics_only(p))
        v = torch.randn(gx.n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(v)
        gx.matvec(v, out=y)
        torch.cuda.synchronize()
        gx.profile(True)
        gx.profile_read(reset=True)
        for _ in range(20):
            gx.matvec(v, out=y)
        kx, nx = gx.profile_read(reset=True)
        gx.profile(False)
        bx = p.n_obs * (18 * 8 + 4) + p.n_lms * 6 * 8 + gx.n * 8
        ax = bx / (kx / max(nx, 1) * 1e-3) / 1e9
        extrinsics = {"d_p": 6, "chunk_kernel_ms": round(kx / max(nx, 1), 5), "bytes_per_launch": int(bx),
                      "achieved_gbs": round(ax, 1), "frac": round(ax / HBM_PEAK_GBS, 4)}
        for name, f in [("pcg_fp64", lambda: gx.pcg(eps=1e-6, max_iter=1000)),
                        ("mcg_fp64_N16", lambda: gx.mcg(16, args.tau, eps=1e-6, max_iter=1000))]:
            f()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(3):
                x, s2 = f()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t1) / 3
            extrinsics[name] = {"solves_per_s": round(1.0 / dt, 3), "iterations": s2.iterations,
                                "multi_steps": s2.multi_steps, "rel_res_true": s2.rel_res_true, "status": s2.status}
        log(f"extrinsics only: {extrinsics}")
        gx.close()

    explicit = None
    if not args.no_variants:
        # the paper's representation: S formed once in 9x9 block-sparse rows (assembly
        # timed separately), then read by every FP64 product
        t = time.time()
        ge = ba.System.from_problem(p, explicit_schur=True)
        torch.cuda.synchronize()
        info_e = ge.explicit_schur_info()
        explicit = {"build_s": round(time.time() - t, 3), "nnz_blocks": info_e["nnz_blocks"],
                    "bytes": info_e["bytes"], "assembly_ms": round(info_e["assembly_ms"], 3)}
        v = torch.randn(ge.n, dtype=torch.float64, device="cuda")
        y = torch.empty_like(v)
        mv_ms = ge.matvec_timed(v, reps=50, out=y)   # back-to-back launches, events around all 50
        explicit["matvec_ms"] = round(mv_ms, 4)
        explicit["matvec_gbs"] = round((info_e["bytes"] + ge.n * 8 * 2) / (mv_ms * 1e-3) / 1e9, 1)
        for name, f in [("pcg_fp64", lambda: ge.pcg(eps=1e-6, max_iter=1000)),
                        ("mcg_fp64_N16", lambda: ge.mcg(16, args.tau, eps=1e-6, max_iter=1000)),
                        ("mcg_fp64_N4", lambda: ge.mcg(4, args.tau, eps=1e-6, max_iter=1000))]:
            f()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for _ in range(3):
                x, s2 = f()
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t1) / 3
            explicit[name] = {"solves_per_s": round(1.0 / dt, 3), "iterations": s2.iterations,
                              "multi_steps": s2.multi_steps, "rel_res_true": s2.rel_res_true, "status": s2.status}
        log(f"explicit S: {explicit}")
        ge.close()

    lm = None
    if not args.no_lm and not args.no_variants:
        # the LM outer loop of Sec. 4.1 from the generator's perturbed state, PCG against MCG
        # (the analogue of the paper's global runtime ratio), implicit and explicit S
        sc, cams0, X0 = ba.Scene.from_problem(p)
        lm = {}
        for name, kw in [("pcg", dict(solver="pcg")), ("mcg_N16", dict(solver="mcg", N=16, tau=args.tau)),
                         ("pcg_explicit", dict(solver="pcg", explicit_schur=True)),
                         ("mcg_N4_explicit", dict(solver="mcg", N=4, tau=args.tau, explicit_schur=True))]:
            c1, X1, ls = sc.lm(cams0, X0, **kw)
            lm[name] = {"iterations": ls.iterations, "accepted": ls.accepted, "status": ls.status,
                        "cost0": ls.cost0, "cost": ls.cost, "solver_iterations": ls.solver_iterations,
                        "t_total_ms": round(ls.t_total_ms, 2), "t_solve_ms": round(ls.t_solve_ms, 2),
                        "t_linearize_ms": round(ls.t_linearize_ms, 2)}
            log(f"LM {name}: {lm[name]}")
            del c1, X1
        for a, b in [("mcg_N16", "pcg"), ("mcg_N4_explicit", "pcg_explicit")]:
            lm[f"ratio_{a}_vs_{b}"] = {"total": round(lm[a]["t_total_ms"] / lm[b]["t_total_ms"], 4),
                                       "solve": round(lm[a]["t_solve_ms"] / lm[b]["t_solve_ms"], 4)}
        del sc, cams0, X0

    dense = None
    if not args.no_dense and not args.no_variants:
        dense = run_dense(args.seed, log)

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        t = time.time()
        o = oracle.System(p)
        ob = time.time() - t
        # bounded sample: a few iterations of the same solver and path, scaled to a
        # full solve of the GPU's iteration count
        def run(k):
            t2 = time.perf_counter()
            if args.solver == "pcg":
                o.pcg(eps=0.0, imax=k)
            else:
                o.mcg(args.N, args.tau, eps=0.0, imax=k)
            return time.perf_counter() - t2
        probe = 2
        tp = run(probe)
        k = max(probe, min(st.iterations, int(10.0 / max(tp / probe, 1e-6))))
        tk = run(k) if k > probe else tp
        per_it = tk / k
        est_solve = per_it * st.iterations
        cpu = {"value": round(1.0 / est_solve, 5), "unit": "solves/s", "cores": oracle.num_threads(),
               "kind": "oracle",
               "sample": f"oracle {args.solver.upper()} (FP64 C, OpenMP) on the same problem: {k} of the "
                         f"{st.iterations} iterations timed ({tk:.1f} s), scaled to the full solve; "
                         f"oracle build {ob:.1f} s not included"}
        log(f"cpu baseline: {cpu}")

    batch = None
    if batch_probs is not None:
        g.close()
        batch = run_batch(batch_probs, args.seed, log)

    value = args.steps / wall
    out = {
        "metric": "RCS solves/s to 1e-6 rel residual (MCG vs PCG, FP64 vs mixed); Schur matvec HBM GB/s",
        "value": round(value, 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32 products, f64 solver", "bf16": "bf16 storage, f32 products"}[args.precision],
        "data": "synthetic",
        "config": {"workload": "walk1936: F-1936-shaped banded synthetic BA (1,936 cameras, 650k landmarks, "
                               f"{p.n_obs} observations), seed {args.seed}",
                   "solver": args.solver, "N": args.N if args.solver == "mcg" else None,
                   "tau": args.tau if args.solver == "mcg" else None, "eps": 1e-6,
                   "iterations": st.iterations, "multi_steps": st.multi_steps,
                   "rel_res_true": st.rel_res_true, "build_s": round(build_s, 3),
                   "mcg_plan_s": None if plan_s is None else round(plan_s, 3),
                   "history_products": "fp64 matrix cores" if args.history_mfma else "vector FMA"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "variants": variants,
        "mixed_mcg_vs_pcg_fp64": mixed_vs_pcg,
        "learned": learned,
        "explicit_schur": explicit,
        "extrinsics_only": extrinsics,
        "batch": batch,
        "lm": lm,
        "dense_schur": dense,
    }
    print(json.dumps(out), flush=True)
    if batch is None:
        g.close()


if __name__ == "__main__":
    main()
