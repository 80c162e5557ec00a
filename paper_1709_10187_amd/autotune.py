"""Launch-schedule autotuner for rddmc_transport, and the longest-first order of a batch.

Two phases:
  * bulk: candidates (threads per block, resident blocks per CU, steps between refills) each
    transport the same packet sample of the batch with a per-packet step cap (the cap fixes
    the work per packet, so the trial measures the schedule's steps/s), timed with device
    events on their own tally and work buffers;
  * tail: with the fastest bulk schedule, each candidate hand-over threshold of the cooperative
    tail walk (``tail_lanes``) walks a per-cloud sample of the batch WHOLE (every packet to
    escape, or to a generous step cap) in one launch; the shortest launch wins.  A launch of
    a tail-bound workload ends with its slowest packets, which the bulk phase cannot see.
The result is remembered per batch signature for the process.

``pilot_costs`` / ``longest_first``: a short pilot walk of every cloud gives its mean steps per
packet; queueing the clouds most expensive first lets their packets start first, so the
launch does not end on them.
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
         use_cache: bool = True, tail_candidates: Iterable[int] = (16, -1, 8, 32),
         tail_packets_per_cloud: int = 64, tail_max_steps: int = 1 << 26) -> dict:
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
           "steps_per_s": best["steps_per_s"], "trials": results, "tail_lanes": 0, "tail_trials": []}
    tails = list(tail_candidates or ())
    if len(tails) > 1:
        # a per-cloud sample of the batch, walked whole: tables of the same clouds with fewer packets
        meds = [m.with_packets(min(int(m.n_packets), int(tail_packets_per_cloud))) for m in b.meds]
        sample = rddmc.Problem(meds, streams=list(b.streams))
        for tl in tails:
            sample.reset()
            start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            start.record(stream)
            sample.run(seed=seed, max_steps=tail_max_steps, tail_lanes=tl, block=best["block"],
                       grid=best["grid"], chunk=best["chunk"])
            stop.record(stream)
            torch.cuda.synchronize()
            out["tail_trials"].append({"tail_lanes": tl, "ms": start.elapsed_time(stop)})
        out["tail_lanes"] = min(out["tail_trials"], key=lambda r: r["ms"])["tail_lanes"]
        del sample
    _CACHE[key] = out
    return out


def pilot_costs(meds, streams=None, packets: int = 64, seed: int = 987654321, max_steps: int = 1 << 20,
                surrogate_fn=None) -> list:
    """Mean steps per packet of every cloud from a pilot walk of ``packets`` packets each (capped
    at ``max_steps``); ``surrogate_fn(problem)`` may return a surrogate / exit-kernel buffer to
    walk the pilot with."""
    pilot = rddmc.Problem([m.with_packets(packets) for m in meds], streams=streams)
    kw = {}
    if surrogate_fn is not None:
        kw["surrogate"] = surrogate_fn(pilot)
    pilot.run(seed=seed, max_steps=max_steps, **kw)
    return [r.steps_mean for r in pilot.results()]


def longest_first(costs) -> list:
    """Cloud order, most expensive first (ties keep the given order)."""
    return sorted(range(len(costs)), key=lambda i: -costs[i])


def schedule(tuned: dict) -> dict:
    """Run keyword arguments for ``Problem.run`` / ``transport`` from a tuning result."""
    return {"block": tuned["block"], "grid": tuned["grid"], "chunk": tuned["chunk"],
            "tail_lanes": tuned.get("tail_lanes", 0)}
