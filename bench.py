"""Benchmark: rDDMC packets/s and packet-steps/s on one MI355X.

Workload: the static uniform sphere -- tau0 = 1e7, T = 1e4 K, 256 radial shells x 512
frequency bins over |x| <= 6 (a tau0)^(1/3), central point source at x = 0, 2^22 packets,
FP32 walk with FP64 tables and clock, int64 tallies.  One benchmark step transports one
contiguous block of that job's packet ids (block k = ids [k B, (k+1) B)) through the
whole hot path: every leakage step, re-binning, escape and tally of those packets runs
inside the timed rddmc_transport launch; the tables are built (untimed) once before.

Prints one JSON line.  ``--gpus`` must be 1 (the path runs on one GPU).
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "packets/s & packet-steps/s at 1 GPU; surrogate vs plain speedup at ≤1% spectrum L1"

# Algorithmic VALU work of one DDMC step (the minimal instruction stream of a step, every
# VALU instruction issuing at one wave-instruction per 4 cycles per SIMD on gfx950, the
# 32x32->64 multiply included, as SQ_INSTS_VALU / time confirms): half a Philox4x32-10
# block (10 rounds x (2 multiplies + 2 three-input xors) / 2 = 20), the path length
# (u32->f32, scale, log2, multiply, f32->f64, f64 add = 6), the event (3 compares, select,
# add = 5) and the record address (1): 32 lane-ops.
OPS_PER_STEP = 32.0
# VALU lane-op issue rate of the chip: 256 CUs x 4 SIMDs x 64 lanes per 4 cycles x 2.4 GHz.
PEAK_OPS = 256 * 4 * 16 * 2.4e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=0,
                    help="untimed blocks before the timed ones (module load happens at the table build)")
    ap.add_argument("--block-packets", type=int, default=1 << 16,
                    help="packets of the 2^22-packet job per benchmark step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-packets", type=int, default=12)
    ap.add_argument("--cpu-threads", type=int, default=0)
    return ap.parse_args()


def cpu_baseline(m, n_packets, threads):
    """The oracle's literal FP64 walker (O1) timed on the host's cores on a bounded sample."""
    from oracle import tables as otb
    from oracle import walk as owalk
    t = otb.build(m)
    t0 = time.perf_counter()
    w = owalk.run(m, n_packets=n_packets, seed=0, n_threads=threads, tabs=t)
    dt = time.perf_counter() - t0
    return {"value": w.n_packets / dt, "unit": "packets/s", "cores": threads, "kind": "oracle",
            "sample": f"packets 0..{n_packets - 1} of the same sphere job (own xoshiro256** streams), "
                      f"{w.steps_sum:.3e} steps in {dt:.1f} s = {w.steps_sum / dt:.3e} steps/s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this path runs on one GPU; --gpus must be 1 (multi-GPU sharding is "
                                   "described in DESIGN.md, not built)"}))
        sys.exit(2)
    import torch
    from paper_1709_10187_amd import media, rddmc
    assert torch.cuda.is_available()
    torch.cuda.set_device(0)
    m = media.config_sphere()
    B = int(args.block_packets)
    n_blocks = m.n_packets // B
    if args.warmup + args.steps > n_blocks:
        raise SystemExit("not enough packet blocks in the job for warmup + steps")
    print(f"[bench] building tables for {m.name}", file=sys.stderr, flush=True)
    prob = rddmc.Problem(m)
    stream = torch.cuda.current_stream()
    # warmup blocks are taken from the end of the job's id range
    for w in range(args.warmup):
        first = (n_blocks - 1 - w) * B
        print(f"[bench] warmup block {w} (ids {first}..{first + B - 1})", file=sys.stderr, flush=True)
        prob.run(seed=0, first=first, count=B)
        torch.cuda.synchronize()
    prob.reset()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for k in range(args.steps):
        prob.run(seed=0, first=k * B, count=B)
    stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop)
    res = prob.results()[0]
    sec = ms / 1e3
    pk_s = res.launched / sec
    st_s = res.steps_total / sec
    per_launch_s = sec / args.steps
    achieved = (res.steps_total / args.steps) * OPS_PER_STEP / per_launch_s
    out = {
        "metric": METRIC,
        "value": pk_s,
        "unit": "packets/s",
        "packet_steps_per_s": st_s,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "static uniform sphere tau0=1e7 T=1e4K, 256 shells x 512 bins, "
                               "|x|<=6(a tau0)^(1/3), central source x=0, job of 2^22 packets; "
                               f"timed: {args.steps} block(s) of {B} consecutive packet ids",
                   "packets_timed": int(res.launched), "escaped": int(res.escaped),
                   "steps_mean": res.steps_mean, "steps_max": int(res.steps_max),
                   "t_mean_light_crossings": res.t_mean, "wall_s": wall,
                   "precision": "f32 walk, f64 tables and clock, i64 tallies, Philox4x32-10"},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_OPS / 1e12,
                     "unit": "T VALU lane-ops/s", "frac": achieved / PEAK_OPS,
                     "traffic": None},
    }
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        print(f"[bench] cpu baseline: oracle walker, {args.cpu_packets} packets, {threads} threads",
              file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(m, args.cpu_packets, threads)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
