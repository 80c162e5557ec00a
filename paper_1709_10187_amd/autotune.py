"""Launch-schedule autotuner for rddmc_transport.

Candidates are (threads per block, resident blocks per CU, steps between refills).  Each
candidate transports the same packet sample of the batch with a per-packet step cap (a
throughput trial: the cap fixes the work per packet, so the trial measures steps/s of the
schedule, not a result), timed with device events on its own tally and work buffers.  The
fastest schedule is returned and remembered per batch signature for the process.
"""
from __future__ import annotations

import itertools
from typing import Dict, Iterable, Optional, Tuple

from . import rddmc

_CACHE: Dict[tuple, dict] = {}


def signature(batch: rddmc.Batch) -> tuple:
    meds = batch.meds
    return (meds[0].geometry, len(meds), any(m.vel is not None for m in meds),
            sum(int(m.n_packets) for m in meds) // 4096,
            max(m.n_cells_total * m.n_bins for m in meds) // 65536)


def default_candidates(n_cu: int) -> Iterable[Tuple[int, int, int]]:
    for block, per_cu, chunk in itertools.product((64, 128, 256), (2, 4, 8), (32, 128)):
        yield block, per_cu * n_cu * (256 // block), chunk


def tune(problem: "rddmc.Problem", sample_packets: int = 1 << 18, trial_steps: int = 20000,
         candidates: Optional[Iterable[Tuple[int, int, int]]] = None, seed: int = 0,
         use_cache: bool = True) -> dict:
    import torch
    b = problem.batch
    key = signature(b)
    if use_cache and key in _CACHE:
        return _CACHE[key]
    n_cu = torch.cuda.get_device_properties(torch.cuda.current_device()).multi_processor_count
    total = sum(int(m.n_packets) for m in b.meds)
    count = min(total, int(sample_packets))
    tally = torch.zeros_like(problem.tallies)
    work = torch.zeros_like(problem.work)
    stream = torch.cuda.current_stream()
    results = []
    for block, grid, chunk in (candidates or default_candidates(n_cu)):
        rddmc.tally_reset(b, tally)
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        rddmc.transport(b, problem.tables, tally, work, seed=seed, first=0, count=count,
                        max_steps=trial_steps, block=block, grid=grid, chunk=chunk)
        stop.record(stream)
        torch.cuda.synchronize()
        ms = start.elapsed_time(stop)
        steps = sum(r.steps_total for r in rddmc.tally(b, tally))
        results.append({"block": block, "grid": grid, "chunk": chunk, "ms": ms,
                        "steps_per_s": steps / (ms / 1e3)})
    best = max(results, key=lambda r: r["steps_per_s"])
    out = {"block": best["block"], "grid": best["grid"], "chunk": best["chunk"],
           "steps_per_s": best["steps_per_s"], "trials": results}
    _CACHE[key] = out
    return out


def schedule(tuned: dict) -> dict:
    """Run keyword arguments for ``Problem.run`` / ``transport`` from a tuning result."""
    return {"block": tuned["block"], "grid": tuned["grid"], "chunk": tuned["chunk"]}
