"""Benchmark: rDDMC packets/s and packet-steps/s on one MI355X.

Workload: the static uniform sphere -- tau0 = 1e7, T = 1e4 K, 256 radial shells x 512
frequency bins over |x| <= 6 (a tau0)^(1/3), central point source at x = 0, 2^22 packets,
FP32 walk with FP64 tables and clock, int64 tallies.  One benchmark step transports one
contiguous block of that job's packet ids (block k = ids [k B, (k+1) B)) through the
whole hot path: every leakage step, re-binning, escape and tally of those packets runs
inside the timed rddmc_transport launch; the tables are built (untimed) once before.

Other workloads (``--workload``):
  cube       the 128^3 lognormal cube (256 bins of 25 km/s, hybrid DDMC / MC at tau = 10,
             2^24 packets from the 64 densest cells): one block of packet ids;
  surrogate  the learned escape surrogate: sub-walk data and training on the GPU (timed
             apart), then the sweep clouds inside the trained domain as one batch, with
             the surrogate and plain, same packet ids, packets/s of each.

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
# HBM bytes of one launch on the default block (2^16 packets of the sphere), from the
# FETCH_SIZE and WRITE_SIZE counters scaled by a plain copy of known size
# (profiles/walk1d_sphere_tau1e7_block65536_pmc.md), taken on the kernel as it is now;
# None for any other block, and None while the kernel has changed since the counters ran.
TRAFFIC_DEFAULT_BLOCK = 5.27e7


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
    ap.add_argument("--workload", choices=["sphere", "cube", "surrogate", "sweep"], default="sphere")
    ap.add_argument("--sweep-packets", type=int, default=128, help="packets per cloud, sweep workload")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy this many MiB device to device (a plain copy of known size that "
                         "calibrates hardware byte counters read in the same run)")
    ap.add_argument("--tail-lanes", type=int, default=0,
                    help="hand a wave's packets to the cooperative walk at <= this many (0 = library default)")
    ap.add_argument("--surrogate-packets", type=int, default=2048, help="packets per cloud, surrogate run")
    ap.add_argument("--plain-packets", type=int, default=64, help="packets per cloud, plain run")
    return ap.parse_args()


def _timed(prob, **kw):
    import torch
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    prob.run(**kw)
    stop.record(stream)
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / 1e3


def bench_cube(args):
    """128^3 hybrid cube: one block of packet ids (the hot path is walk3d)."""
    from paper_1709_10187_amd import media, rddmc
    m = media.cube()
    B = int(args.block_packets)
    print(f"[bench] building tables for the 128^3 x 256 cube", file=sys.stderr, flush=True)
    prob = rddmc.Problem(m)
    sec = 0.0
    for k in range(args.steps):
        sec += _timed(prob, seed=0, first=k * B, count=B)
    res = prob.results()[0]
    ddmc = res.steps_total - res.mc_steps
    return {
        "metric": METRIC, "value": res.launched / sec, "unit": "packets/s",
        "packet_steps_per_s": res.steps_total / sec, "n_gpus": 1, "steps": args.steps, "warmup": 0,
        "ms_per_step": 1e3 * sec / args.steps, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "3D cube 128^3 lognormal (sigma_ln 1, mean tau_cell 1e3), T=1e4K, 20 km/s "
                               "Gaussian velocities, 256 bins of 25 km/s, hybrid at tau_th=10, 64 densest-cell "
                               f"sources, job of 2^24 packets; timed: {args.steps} block(s) of {B} ids",
                   "packets_timed": int(res.launched), "steps_mean": res.steps_mean,
                   "ddmc_steps": int(ddmc), "mc_events": int(res.mc_steps), "to_mc": int(res.to_mc),
                   "to_ddmc": int(res.to_ddmc), "reflected": int(res.reflected), "t_mean": res.t_mean,
                   "table_gib": prob.tables.numel() / 2 ** 30},
        "roofline": None,
    }


# Sweep clouds (media.sweep_parameters(), 256 clouds) whose plain rDDMC walk takes <= 1e7
# expected steps per packet (exact-chain values, 158 clouds): the rest, up to 8e8 steps
# per packet, are the surrogate's ground; with them one launch would wait minutes on its
# slowest packets.
SWEEP_CLOUDS = [0, 1, 2, 6, 7, 10, 11, 12, 13, 15, 16, 17, 19, 20, 21, 23, 25, 26, 27, 28, 29, 30, 32, 33, 34, 35,
                36, 37, 39, 40, 43, 44, 45, 46, 48, 49, 53, 55, 56, 59, 60, 62, 64, 65, 66, 67, 69,
                71, 73, 75, 77, 80, 81, 83, 84, 85, 86, 87, 88, 92, 93, 94, 96, 98, 99, 101, 103,
                104, 105, 106, 107, 109, 110, 112, 113, 116, 117, 118, 120, 122, 123, 124, 126, 130,
                132, 133, 134, 135, 139, 142, 143, 144, 145, 147, 150, 152, 155, 156, 157, 158, 159,
                160, 161, 165, 166, 168, 170, 172, 173, 174, 176, 177, 178, 179, 180, 183, 185, 186,
                188, 189, 190, 191, 193, 196, 198, 199, 200, 201, 202, 203, 204, 206, 207, 209, 213,
                219, 221, 222, 224, 225, 226, 227, 229, 230, 231, 233, 236, 240, 241, 242, 246, 247,
                248, 249, 250, 253, 254, 255]

# Sweep clouds with cells in the surrogate's trained domain whose plain rDDMC walk takes
# <= 5e7 expected steps per packet (exact-chain values; the 10 costlier in-domain clouds, up
# to 5e8 steps per packet, would make the plain leg's slowest packets run for minutes).
SURROGATE_CLOUDS = [9, 18, 48, 58, 68, 74, 75, 96, 101, 103, 125, 131, 144, 149, 151, 155, 156, 176, 181, 184,
                    188, 195, 199, 203, 205, 226, 235, 250]


def bench_sweep(args):
    """The batched sweep: many clouds of uneven grid size in one hipGraph-captured
    rddmc_transport launch with an autotuned schedule."""
    import torch
    from paper_1709_10187_amd import autotune, media, rddmc
    clouds = [media.sweep_cloud_medium(c) for c in media.sweep_parameters()]
    ids = SWEEP_CLOUDS
    meds = [clouds[i].with_packets(args.sweep_packets) for i in ids]
    print(f"[bench] sweep: building tables for {len(ids)} clouds", file=sys.stderr, flush=True)
    prob = rddmc.Problem(meds, streams=ids)
    t0 = time.perf_counter()
    tuned = autotune.tune(prob, sample_packets=1 << 16, trial_steps=20000, use_cache=False)
    t_tune = time.perf_counter() - t0
    sched = autotune.schedule(tuned)
    print(f"[bench] sweep: schedule {sched} ({t_tune:.1f} s of trials)", file=sys.stderr, flush=True)
    graph = prob.capture(seed=1, **sched)
    prob.reset()
    stream = torch.cuda.current_stream()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    start.record(stream)
    graph.replay()
    stop.record(stream)
    torch.cuda.synchronize()
    sec = start.elapsed_time(stop) / 1e3
    res = prob.results()
    n = sum(r.launched for r in res)
    steps = sum(r.steps_total for r in res)
    return {
        "metric": METRIC, "value": n / sec, "unit": "packets/s", "packet_steps_per_s": steps / sec, "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": 1e3 * sec, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"batched sweep: {len(ids)} of the 256 sweep clouds (those with <= 1e7 expected "
                               f"steps per packet), {args.sweep_packets} packets each, one hipGraph replay of "
                               "one rddmc_transport launch with the autotuned schedule",
                   "clouds": ids, "packets": int(n), "escaped": int(sum(r.escaped for r in res)),
                   "shells": [int(m.n_cells[0]) for m in meds], "bins": [int(m.n_bins) for m in meds],
                   "schedule": sched, "tune_s": t_tune,
                   "tune_trials": [{k: v for k, v in t.items()} for t in tuned["trials"]]},
        "roofline": None,
    }


def bench_surrogate(args):
    """Learned escape surrogate against plain rDDMC on the in-domain sweep clouds."""
    import torch
    from paper_1709_10187_amd import media, rddmc
    from paper_1709_10187_amd import surrogate as sg
    dom = sg.Domain(tau_min=1.0e5, tau_max=1.0e6, dx_min=0.5, dx_max=4.5)
    t0 = time.perf_counter()
    probes = sg.sample_probes(2048, dom, seed=11)
    print("[bench] surrogate: 2048 x 128 sub-walks", file=sys.stderr, flush=True)
    data = sg.generate(probes, 128, dom, seed=12, max_steps=1 << 30)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    net = rddmc.Mdn(max_batch=4096, seed=0)
    t1 = time.perf_counter()
    print(f"[bench] surrogate: training on {data.n} samples", file=sys.stderr, flush=True)
    hist = sg.train(net, data, epochs=60, lr=2e-3, lr_final=1e-4)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    clouds = [media.sweep_cloud_medium(c) for c in media.sweep_parameters()]
    ids = [i for i in SURROGATE_CLOUDS if sg.window(clouds[i], dom)[1] >= sg.window(clouds[i], dom)[0]]
    surr = rddmc.Problem([clouds[i].with_packets(args.surrogate_packets) for i in ids], streams=ids)
    att = sg.Attached(surr, net, dom)
    print(f"[bench] surrogate: {len(ids)} clouds, {att.n_states} window states", file=sys.stderr, flush=True)
    ts = _timed(surr, seed=1, surrogate=att.buffer)
    rs = surr.results()
    plain = rddmc.Problem([clouds[i].with_packets(args.plain_packets) for i in ids], streams=ids)
    print("[bench] plain rDDMC on the same clouds", file=sys.stderr, flush=True)
    tp = _timed(plain, seed=1)
    rp = plain.results()
    ns, npl = sum(r.launched for r in rs), sum(r.launched for r in rp)
    v_s, v_p = ns / ts, npl / tp
    return {
        "metric": METRIC, "value": v_s, "unit": "packets/s", "plain_packets_per_s": v_p, "speedup": v_s / v_p,
        "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": 1e3 * ts, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16 network (f32 accumulate), f32 walk",
        "data": "synthetic",
        "config": {"workload": f"{len(ids)} sweep clouds with cells in the trained domain and <= 5e7 plain steps/packet "
                               f"(tau_c {dom.tau_min:g}-{dom.tau_max:g}, dx {dom.dx_min}-{dom.dx_max}), one batch; "
                               f"{args.surrogate_packets} packets per cloud with the surrogate, "
                               f"{args.plain_packets} plain",
                   "clouds": ids, "window_states": int(att.n_states),
                   "surrogate_calls_per_packet": sum(r.surrogate_calls for r in rs) / ns,
                   "steps_per_packet_surrogate": sum(r.steps_total for r in rs) / ns,
                   "steps_per_packet_plain": sum(r.steps_total for r in rp) / npl,
                   "data_s": t_data, "train_s": t_train, "train_samples": data.n, "final_nll": hist[-1],
                   "accuracy": "spectrum vs the exact chain in tests/test_gpu_surrogate.py"},
        "roofline": None,
    }


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
    if args.workload != "sphere":
        out = {"cube": bench_cube, "surrogate": bench_surrogate, "sweep": bench_sweep}[args.workload](args)
        print(json.dumps(out))
        return
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy probe: {args.copy_probe_mib} MiB read, {args.copy_probe_mib} MiB written",
              file=sys.stderr, flush=True)
        del src, dst
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
        prob.run(seed=0, first=first, count=B, tail_lanes=args.tail_lanes)
        torch.cuda.synchronize()
    prob.reset()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(stream)
    for k in range(args.steps):
        prob.run(seed=0, first=k * B, count=B, tail_lanes=args.tail_lanes)
        if args.steps > 1:   # the block has finished: report it (the next block starts at once)
            torch.cuda.synchronize()
            print(f"[bench] block {k} done ({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
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
                     "traffic": TRAFFIC_DEFAULT_BLOCK if (B == 1 << 16 and args.steps == 1) else None},
    }
    if not args.no_cpu_baseline:
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        print(f"[bench] cpu baseline: oracle walker, {args.cpu_packets} packets, {threads} threads",
              file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(m, args.cpu_packets, threads)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
