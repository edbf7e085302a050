"""Autotuner of the chunk shape of the S products.

A chunk is the unit of one wavefront of the chunk kernel: consecutive 64-slot tiles
(at most max_tiles) touching at most max_slots cameras, whose camera rows are staged
in LDS.  Fewer tiles per chunk mean more partial rows for the camera reduction and
more v gathers; more tiles mean fewer, longer wavefronts and a worse tail on 256 CUs.
The best shape depends on the problem mix, so it is measured: every candidate layout
is built for a sample of the workload and its S product timed with device events.
"""
from __future__ import annotations

from typing import Dict, List, Sequence, Tuple

from . import Batch, System

CANDIDATES: Tuple[Tuple[int, int], ...] = ((128, 4), (128, 8), (128, 16), (128, 32), (128, 64), (256, 16), (64, 16))


def _time_products(system: System, precision: str, reps: int) -> float:
    import torch
    gen = torch.Generator(device=system.device).manual_seed(0)
    v = torch.randn(system.n, dtype=torch.float64, device=system.device, generator=gen)
    y = torch.empty_like(v)
    system.matvec(v, precision=precision, out=y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        system.matvec(v, precision=precision, out=y)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune_chunks(problems: Sequence, precision: str = "fp32", candidates: Sequence[Tuple[int, int]] = CANDIDATES,
                reps: int = 20) -> Dict[str, object]:
    """Times the S product of a batch of `problems` for every (max_slots, max_tiles)
    candidate; returns the fastest and the whole table (ms per product)."""
    table: List[Dict[str, object]] = []
    for slots, tiles in candidates:
        b = Batch(list(problems), max_slots=slots, max_tiles=tiles, store_fp32=precision == "fp32",
                  store_bf16=precision == "bf16")
        try:
            ms = _time_products(b.system, precision, reps)
            info = b.system.info()
        finally:
            b.close()
        table.append({"max_slots": slots, "max_tiles": tiles, "ms": ms, "chunks": info["n_chunks"]})
    best = min(table, key=lambda r: r["ms"])
    return {"max_slots": best["max_slots"], "max_tiles": best["max_tiles"], "ms": best["ms"], "table": table}
