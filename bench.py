"""Benchmark: rDDMC packets/s and packet-steps/s on one MI355X.

Default workload: the 3D Cartesian lognormal cube -- 128^3 unit cells, ln k0 ~ N(ln 1e3 - 1/2, 1)
(mean cell optical depth 1e3), T = 1e4 K, Gaussian bulk velocities of 20 km/s per component,
256 frequency bins of 25 km/s, hybrid DDMC / continuous MC switched at a cell optical depth of
10, 2^24 packets from the 64 densest cells.  One benchmark step is the WHOLE job: all 2^24
packets walked to escape (every DDMC leak, MC flight, conversion, re-binning, escape and int64
tally) in one rddmc_transport launch; the 30.5 GiB of tables are built once, untimed, and are
resident in HBM.  Each step uses its own Philox seed (step k: seed k), so every step is a fresh
walk of the same workload.

Other workloads (``--workload``):
  sphere     the static uniform sphere tau0 = 1e7, 256 shells x 512 bins, 2^22 packets: one
             step is the whole job (about 7 minutes), or ``--block-packets`` consecutive ids;
  sphere-efficient
             the same sphere on the paper's efficient frequency grid (79 bins: a central bin
             of 2 x_cw, unit-width wings to 2.5 (a tau0)^(1/3)), the whole job per step;
  sweep      batched sweep clouds in one hipGraph-captured launch with the autotuned schedule;
  sweep-full all 256 sweep clouds at their stated packet counts (2^14..2^18 each) in one launch
             with the exact per-cell exit kernel, clouds ordered longest first by a pilot walk;
  surrogate  the learned escape surrogate against plain rDDMC on the same clouds and packets;
  methods    static uniform slabs (tau0 = 1e3 .. 1e6, 64 cells x 128 bins over |x| <= 6 (a tau0)^(1/3),
             T = 1e4 K, central source at x = 0), each walked whole on the same packet ids by
             rDDMC, rDDMC on the efficient frequency grid, frequency-group Monte Carlo (Sec. 5.3,
             eq. 42), continuous-frequency Monte Carlo (the scattering-by-scattering reference) and
             the latter with core-skipping (x_crit = 3, the kind of MCRT the paper compares with);
             the value is rDDMC's packets/s on the tau0 = 1e5 slab;
  census     the time-dependent estimators' cost: the tau0 = 1e5 slab (64 x 128, 2^16 packets)
             walked whole by the pure 1D walk, by the hybrid 1D walk without estimators, and by
             the hybrid walk with 16 census intervals (eq. 17's bin and path estimators and
             eq. 18's sums), on the same packet ids.

Prints one JSON line.  ``--gpus`` must be 1 (the path runs on one GPU).
"""
import argparse
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "packets/s & packet-steps/s at 1 GPU; surrogate vs plain speedup at ≤1% spectrum L1"
CSRC = os.path.join(ROOT, "paper_1709_10187_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")

# Algorithmic bytes of the 3D walk (per unit, the gathers a step cannot avoid): a DDMC step
# reads its state's record, 36 B (16 B hot record + the 20 B face-split CDF of the full 3D
# table); a continuous-MC event reads the cell's 32 B record; an escape adds 32 B of integer
# tally atomics.  Bound: HBM (the 30.5 GiB table does not fit any cache), peak 8 TB/s.
BYTES_DDMC_STEP = 36.0
BYTES_MC_EVENT = 32.0
BYTES_ESCAPE = 32.0
HBM_PEAK = 8.0e12

# The 1D walk is bound by instruction issue (its 2 MB table stays in L2): one DDMC step's
# minimal VALU stream is 32 lane-ops (half a Philox4x32-10 block = 20, path length 6, event 5,
# address 1) against 256 CUs x 4 SIMDs x 16 lanes per cycle x 2.4 GHz.
OPS_PER_STEP = 32.0
PEAK_OPS = 256 * 4 * 16 * 2.4e9

# Sources of each walk kernel: HBM traffic recorded in a profile counts only while they are
# unchanged since the counters were taken.
KERNEL_SOURCES = {
    "walk3d": ["transport3d.hip", "mc_dev.h", "philox.h", "rddmc_internal.h"],
    "walk1d": ["transport.hip", "philox.h", "rddmc_internal.h", "surrogate_dev.h", "linemath_dev.h"],
}
TRAFFIC_RE = re.compile(r"traffic_bytes_per_launch = ([0-9.eE+]+) \(sources sha256 ([0-9a-f]{64})\)")


def sources_sha256(kernel):
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def profiled_traffic(profile, kernel):
    """HBM bytes per launch from a committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary, or None
    when the summary is missing or the kernel's sources changed since it was taken."""
    path = os.path.join(PROFILES, profile)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        m = TRAFFIC_RE.search(f.read())
    if not m or m.group(2) != sources_sha256(kernel):
        return None
    return float(m.group(1))


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", choices=["cube", "sphere", "sphere-efficient", "surrogate", "sweep", "sweep-full",
                                           "methods", "census"], default="cube")
    ap.add_argument("--block-packets", type=int, default=0,
                    help="sphere: packets per step (0 = the whole 2^22-packet job)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-packets", type=int, default=0, help="oracle sample size (0 = workload default)")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--sweep-packets", type=int, default=128, help="packets per cloud, sweep workload")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first copy this many MiB device to device (a plain copy of known size that "
                         "calibrates hardware byte counters read in the same run)")
    ap.add_argument("--tail-lanes", type=int, default=0,
                    help="1D: hand a wave's packets to the cooperative walk at <= this many (0 = default)")
    ap.add_argument("--surrogate-packets", type=int, default=2048, help="packets per cloud, surrogate workload")
    ap.add_argument("--train-per-probe", type=int, default=0,
                    help="surrogate: training samples per probe medium (0 = the library's recipe)")
    ap.add_argument("--train-epochs", type=int, default=0, help="surrogate: training epochs (0 = the recipe)")
    ap.add_argument("--train-step-budget", type=float, default=0.0,
                    help="surrogate: longest expected sub-walk run as a walk; longer ones draw from the exact "
                         "in-cell law (0 = the recipe)")
    ap.add_argument("--exit-kernel", action="store_true",
                    help="sphere workloads: walk with the exact per-cell exit kernel (built untimed)")
    ap.add_argument("--ek-min-steps", type=float, default=64.0, help="exit-kernel window: shortest expected sub-walk")
    ap.add_argument("--sweep-scale", type=float, default=1.0, help="sweep-full: fraction of the stated packet counts")
    ap.add_argument("--census-packets", type=int, default=0,
                    help="census: packets per leg (0 = the slab's 2^16)")
    ap.add_argument("--methods-tau0", type=float, nargs="*", default=[1e3, 1e4, 1e5, 1e6],
                    help="methods: the slabs' line-centre depths")
    ap.add_argument("--methods-legs", nargs="*", default=["rddmc", "rddmc_efficient", "groups", "mcrt", "mcrt_cs"],
                    help="methods: which methods walk each slab")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def copy_probe(mib):
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy probe: {mib} MiB read, {mib} MiB written")
    del src, dst


def timed_steps(prob, steps, warmup, **kw):
    """W untimed then K timed rddmc_transport launches on torch's current stream (the stream
    the library launches on), step k with Philox seed k.  Returns (total seconds between the
    synchronised brackets, per-launch seconds from event pairs around each launch)."""
    import torch
    stream = torch.cuda.current_stream()
    for w in range(warmup):
        prob.run(seed=1000 + w, **kw)
        torch.cuda.synchronize()
        log(f"warmup step {w} done")
    prob.reset()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    outer = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outer[0].record(stream)
    for k in range(steps):
        ev[k][0].record(stream)
        prob.run(seed=k, **kw)
        ev[k][1].record(stream)
        if steps > 1:
            torch.cuda.synchronize()
            log(f"step {k} done ({time.perf_counter() - t0:.1f} s)")
    outer[1].record(stream)
    torch.cuda.synchronize()
    total = outer[0].elapsed_time(outer[1]) / 1e3
    per = [a.elapsed_time(b) / 1e3 for a, b in ev]
    return total, per


def watched_step(prob, seed, **kw):
    """One step as ONE rddmc_transport launch (a single tail for the whole job) on a side
    stream.  While it runs, the tallies are read on another stream every 2 s and a line is
    logged whenever the number of finished packets has grown (nothing is printed while no
    packet finishes).  Returns (seconds between events bracketing the launch, [same])."""
    import torch
    from paper_1709_10187_amd import rddmc
    cur = torch.cuda.current_stream()
    run_s, poll_s = torch.cuda.Stream(), torch.cuda.Stream()
    prob.reset()
    torch.cuda.synchronize()
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    run_s.wait_stream(cur)
    start.record(run_s)
    rddmc.transport(prob.batch, prob.tables, prob.tallies, prob.work, seed=seed, stream=run_s, **kw)
    stop.record(run_s)
    t0 = time.perf_counter()
    total = prob.total_packets
    done_last = 0
    while not stop.query():
        time.sleep(2.0)
        done = sum(r.escaped + r.capped + r.absorbed for r in rddmc.tally(prob.batch, prob.tallies, stream=poll_s))
        if done > done_last:
            log(f"{done} of {total} packets finished ({time.perf_counter() - t0:.0f} s)")
            done_last = done
    torch.cuda.synchronize()
    sec = start.elapsed_time(stop) / 1e3
    return sec, [sec]


def base_line(args, value, sec, dtype, config, **extra):
    out = {"metric": METRIC, "value": value, "unit": "packets/s"}
    out.update(extra)
    out.update({"n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": 1e3 * sec / args.steps,
                "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": dtype,
                "data": "synthetic", "config": config})
    return out


def bench_cube(args):
    """The whole 2^24-packet cube job per step; the hot kernel is walk3d."""
    from paper_1709_10187_amd import media, rddmc
    if args.copy_probe_mib > 0:
        copy_probe(args.copy_probe_mib)
    m = media.cube()
    log("building tables for the 128^3 x 256 cube")
    prob = rddmc.Problem(m)
    sec, per = timed_steps(prob, args.steps, args.warmup)
    res = prob.results()[0]
    K = args.steps
    ddmc = res.steps_total - res.mc_steps
    bytes_launch = (BYTES_DDMC_STEP * ddmc + BYTES_MC_EVENT * res.mc_steps + BYTES_ESCAPE * res.escaped) / K
    launch_s = sum(per) / K
    achieved = bytes_launch / launch_s
    out = base_line(
        args, res.launched / sec, sec, "f32",
        {"workload": "3D cube 128^3 lognormal (sigma_ln 1, mean tau_cell 1e3), T=1e4K, 20 km/s Gaussian "
                     "velocities, 256 bins of 25 km/s, hybrid DDMC/MC at tau_th=10, 64 densest-cell sources, "
                     "2^24 packets; one step = the whole job (seed = step index)",
         "packets_per_step": int(m.n_packets), "escaped": int(res.escaped), "capped": int(res.capped),
         "steps_mean": res.steps_mean, "steps_max": int(res.steps_max), "ddmc_steps": int(ddmc),
         "mc_events": int(res.mc_steps), "to_mc": int(res.to_mc), "to_ddmc": int(res.to_ddmc),
         "reflected": int(res.reflected), "t_mean_cell_crossings": res.t_mean,
         "launch_ms": [1e3 * p for p in per], "table_gib": prob.tables.numel() / 2 ** 30,
         "precision": "f32 walk, f64 tables and clock, i64 tallies, Philox4x32-10"},
        packet_steps_per_s=res.steps_total / sec)
    out["roofline"] = {
        "bound": "hbm", "achieved": achieved / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s",
        "frac": achieved / HBM_PEAK,
        "traffic": profiled_traffic("walk3d_cube128_job_pmc.md", "walk3d"),
        "kernel": "walk3d", "algorithmic_bytes_per_launch": bytes_launch,
        "alu_frac": (res.steps_total / K) * OPS_PER_STEP / launch_s / PEAK_OPS}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_cube(args)
    return out


def bench_sphere(args, efficient=False):
    """The tau0 = 1e7 sphere; one step = the whole 2^22-packet job or a block of its ids.  With
    `efficient`, on the paper's efficient frequency grid instead of 512 uniform bins."""
    from paper_1709_10187_amd import media, rddmc
    if args.copy_probe_mib > 0:
        copy_probe(args.copy_probe_mib)
    m = media.config_sphere()
    grid = "256 shells x 512 bins, |x|<=6(a tau0)^(1/3)"
    if efficient:
        m = m.replace(bin_edges=media.efficient_edges(4.702e-4, 1.0e7, 1.0 / 256), name="sphere_tau1e7_efficient")
        grid = (f"256 shells x {m.n_bins} bins of the efficient grid (central bin 2 x_cw = "
                f"{m.bin_edges[m.n_bins // 2 + 1] - m.bin_edges[m.n_bins // 2]:.3f}, unit wings, |x|<=2.5(a tau0)^(1/3))")
    B = int(args.block_packets) or int(m.n_packets)
    log(f"building tables for {m.name}")
    prob = rddmc.Problem(m)
    extra, ek_info = {}, {}
    if args.exit_kernel:
        t0 = time.perf_counter()
        ek = rddmc.ExitKernel(prob, min_steps=args.ek_min_steps)
        ek_info = {"exit_kernel": {"window": list(ek.windows[0]), "states": ek.n_states,
                                   "mib": ek.buffer.numel() / 2 ** 20, "build_s": time.perf_counter() - t0,
                                   "min_steps": args.ek_min_steps}}
        extra["surrogate"] = ek.buffer
        log(f"exit kernel: {ek.n_states} window states, {ek_info['exit_kernel']['mib']:.1f} MiB")
    sec, per = timed_steps(prob, args.steps, args.warmup, first=0, count=B, tail_lanes=args.tail_lanes, **extra)
    res = prob.results()[0]
    K = args.steps
    launch_s = sum(per) / K
    achieved = (res.steps_total / K) * OPS_PER_STEP / launch_s
    out = base_line(
        args, res.launched / sec, sec, "f32",
        {"workload": f"static uniform sphere tau0=1e7 T=1e4K, {grid}, "
                     f"central source x=0, job of 2^22 packets; one step = packet ids 0..{B - 1}",
         "packets_per_step": B, "escaped": int(res.escaped), "steps_mean": res.steps_mean,
         "steps_max": int(res.steps_max), "t_mean_light_crossings": res.t_mean,
         "launch_ms": [1e3 * p for p in per],
         "precision": "f32 walk, f64 tables and clock, i64 tallies, Philox4x32-10", **ek_info},
        packet_steps_per_s=res.steps_total / sec)
    if args.exit_kernel:
        out["config"]["exit_kernel"]["exits_per_packet"] = res.surrogate_calls / res.launched
        out["config"]["workload"] += ("; cell sub-walks drawn from the exact per-cell exit kernel (spectrum exact in "
                                      "law, escape-time mean and variance exact)")
    out["roofline"] = {
        "bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_OPS / 1e12, "unit": "T VALU lane-ops/s",
        "frac": achieved / PEAK_OPS,
        "traffic": (profiled_traffic("walk1d_sphere_tau1e7_job_pmc.md", "walk1d")
                    if B == m.n_packets and not efficient else None),
        "kernel": "walk1d"}
    if args.exit_kernel:
        out["roofline"] = None   # exits are table gathers and solves' draws, not DDMC steps
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_1d(m, args.cpu_packets or (16384 if efficient else 12), args)
    return out


# Sweep clouds (media.sweep_parameters(), 256 clouds) whose plain rDDMC walk takes <= 1e7
# expected steps per packet (exact-chain values, 158 clouds).
SWEEP_CLOUDS = [0, 1, 2, 6, 7, 10, 11, 12, 13, 15, 16, 17, 19, 20, 21, 23, 25, 26, 27, 28, 29, 30, 32, 33, 34, 35,
                36, 37, 39, 40, 43, 44, 45, 46, 48, 49, 53, 55, 56, 59, 60, 62, 64, 65, 66, 67, 69,
                71, 73, 75, 77, 80, 81, 83, 84, 85, 86, 87, 88, 92, 93, 94, 96, 98, 99, 101, 103,
                104, 105, 106, 107, 109, 110, 112, 113, 116, 117, 118, 120, 122, 123, 124, 126, 130,
                132, 133, 134, 135, 139, 142, 143, 144, 145, 147, 150, 152, 155, 156, 157, 158, 159,
                160, 161, 165, 166, 168, 170, 172, 173, 174, 176, 177, 178, 179, 180, 183, 185, 186,
                188, 189, 190, 191, 193, 196, 198, 199, 200, 201, 202, 203, 204, 206, 207, 209, 213,
                219, 221, 222, 224, 225, 226, 227, 229, 230, 231, 233, 236, 240, 241, 242, 246, 247,
                248, 249, 250, 253, 254, 255]

# Sweep clouds with cells in the surrogate's trained domain and <= 5e7 expected plain steps
# per packet (exact-chain values).
SURROGATE_CLOUDS = [9, 18, 48, 58, 68, 74, 75, 96, 101, 103, 125, 131, 144, 149, 151, 155, 156, 176, 181, 184,
                    188, 195, 199, 203, 205, 226, 235, 250]


def bench_sweep(args):
    """Batched sweep clouds in one hipGraph-captured rddmc_transport launch, autotuned."""
    import torch
    from paper_1709_10187_amd import autotune, media, rddmc
    clouds = [media.sweep_cloud_medium(c) for c in media.sweep_parameters()]
    ids = SWEEP_CLOUDS
    meds = [clouds[i].with_packets(args.sweep_packets) for i in ids]
    log(f"sweep: building tables for {len(ids)} clouds")
    prob = rddmc.Problem(meds, streams=ids)
    t0 = time.perf_counter()
    tuned = autotune.tune(prob, sample_packets=1 << 16, trial_steps=20000, use_cache=False)
    t_tune = time.perf_counter() - t0
    sched = autotune.schedule(tuned)
    log(f"sweep: schedule {sched} ({t_tune:.1f} s of trials)")
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
    args.steps, args.warmup = 1, 0
    out = base_line(
        args, n / sec, sec, "f32",
        {"workload": f"batched sweep: {len(ids)} of the 256 sweep clouds (those with <= 1e7 expected steps "
                     f"per packet), {args.sweep_packets} packets each, one hipGraph replay of one "
                     "rddmc_transport launch with the autotuned schedule",
         "clouds": ids, "packets": int(n), "escaped": int(sum(r.escaped for r in res)),
         "schedule": sched, "tune_s": t_tune},
        packet_steps_per_s=steps / sec)
    out["roofline"] = None
    return out


def bench_sweep_full(args):
    """All 256 sweep clouds at their stated packet counts in one rddmc_transport launch with the
    exact per-cell exit kernel.  The clouds are queued longest first: a pilot walk of 64 packets
    per cloud (capped at 2^20 steps, untimed) estimates each cloud's steps per packet, so the
    clouds whose packets take longest start first and the launch does not end on them."""
    import torch
    from paper_1709_10187_amd import autotune, media, rddmc
    meds = media.config_sweep(packet_scale=args.sweep_scale)
    n_cl = len(meds)
    t0 = time.perf_counter()
    log(f"sweep-full: pilot of 64 packets per cloud over {n_cl} clouds")
    cost = autotune.pilot_costs(meds, streams=list(range(n_cl)),
                                surrogate_fn=lambda q: rddmc.ExitKernel(q, min_steps=args.ek_min_steps).buffer)
    torch.cuda.empty_cache()
    order = autotune.longest_first(cost)
    t_pilot = time.perf_counter() - t0
    log(f"sweep-full: building tables and exit kernels ({t_pilot:.1f} s of pilot)")
    prob = rddmc.Problem([meds[i] for i in order], streams=order)
    t1 = time.perf_counter()
    ek = rddmc.ExitKernel(prob, min_steps=args.ek_min_steps)
    torch.cuda.synchronize()
    t_ek = time.perf_counter() - t1
    args.steps, args.warmup = 1, 0
    sec, per = watched_step(prob, seed=0, surrogate=ek.buffer)
    res = prob.results()
    n = sum(r.launched for r in res)
    steps = sum(r.steps_total for r in res)
    exits = sum(r.surrogate_calls for r in res)
    out = base_line(
        args, n / sec, sec, "f32",
        {"workload": f"all {n_cl} sweep clouds (PCG64(3): tau0 10^U(4,9), T 10^U(2,5) K, 32..512 shells, "
                     f"256..1024 bins, 0..200 km/s outflow) at {args.sweep_scale:g} x their stated 2^U(14,18) "
                     "packets, cell sub-walks drawn from the exact per-cell exit kernel, clouds queued longest first "
                     "by a pilot, one launch",
         "packets": int(n), "escaped": int(sum(r.escaped for r in res)), "capped": int(sum(r.capped for r in res)),
         "exits_per_packet": exits / n, "exit_kernel_states": ek.n_states,
         "exit_kernel_mib": ek.buffer.numel() / 2 ** 20, "exit_kernel_build_s": t_ek, "pilot_s": t_pilot,
         "order_first": order[:8], "launch_ms": [1e3 * p for p in per]},
        packet_steps_per_s=steps / sec)
    out["roofline"] = None
    return out


def spectrum_agreement(ra, rb, n_groups=40):
    """Two escape spectra of the same cloud (surrogate and plain legs) on at most n_groups
    groups of adjacent bins: their L1 distance and the L1 that Monte Carlo noise alone gives
    two independent samples of these sizes (half-normal mean of each group's difference)."""
    import numpy as np
    a = np.asarray(ra.spectrum, dtype=np.float64).sum(axis=0)
    b = np.asarray(rb.spectrum, dtype=np.float64).sum(axis=0)
    k = max(1, a.size // n_groups)
    a = np.add.reduceat(a, np.arange(0, a.size, k))
    b = np.add.reduceat(b, np.arange(0, b.size, k))
    na, nb = a.sum(), b.sum()
    p = (a + b) / (na + nb)
    l1 = float(np.abs(a / na - b / nb).sum())
    noise = float((np.sqrt(2.0 / np.pi) * np.sqrt(p * (1.0 - p) * (1.0 / na + 1.0 / nb))).sum())
    return l1, noise


def bench_surrogate(args):
    """Learned escape surrogate against plain rDDMC: the same clouds, the same packet ids."""
    import torch
    from paper_1709_10187_amd import media, rddmc
    from paper_1709_10187_amd import surrogate as sg
    dom, use = sg.train_domain(), sg.use_domain()
    per_probe = args.train_per_probe or sg.TRAIN_PER_PROBE
    epochs = args.train_epochs or sg.TRAIN_EPOCHS
    budget = args.train_step_budget or sg.TRAIN_STEP_BUDGET
    t0 = time.perf_counter()
    probes = sg.sample_probes(sg.TRAIN_PROBES, dom, seed=11)
    log(f"surrogate: {sg.TRAIN_PROBES} x {per_probe} samples (sub-walks up to {budget:g} expected steps, "
        f"the exact in-cell law above)")
    data = sg.generate_mixed(probes, per_probe, dom, seed=12, step_budget=budget)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    n_walked = int((data.steps > 0).sum())
    log(f"surrogate: {data.n} samples in {t_data:.1f} s ({n_walked} walked)")
    held = sg.generate_mixed(sg.sample_probes(512, dom, seed=13), 128, dom, seed=14, step_budget=budget)
    net = rddmc.Mdn(max_batch=4096, seed=0)
    t1 = time.perf_counter()
    log(f"surrogate: training on {data.n} samples, {epochs} epochs")
    hist = sg.train(net, data, epochs=epochs, lr=2e-3, lr_final=1e-4,
                    log=log if data.n * epochs > (1 << 26) else None)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    nll_held = sg.mean_nll(net, held)
    log(f"surrogate: trained in {t_train:.1f} s; final training NLL {hist[-1]:.4f}, held-out NLL {nll_held:.4f} "
        f"({held.n} samples of 512 other probe media)")
    clouds = [media.sweep_cloud_medium(c) for c in media.sweep_parameters()]
    ids = [i for i in SURROGATE_CLOUDS if sg.window(clouds[i], use)[1] >= sg.window(clouds[i], use)[0]]
    meds = [clouds[i].with_packets(args.surrogate_packets) for i in ids]
    surr = rddmc.Problem(meds, streams=ids)
    att = sg.Attached(surr, net, use)
    log(f"surrogate: {len(ids)} clouds, {att.n_states} window states")
    args.steps, args.warmup = 1, 0
    ts, _ = timed_steps(surr, 1, 0, surrogate=att.buffer)
    rs = surr.results()
    plain = rddmc.Problem(meds, streams=ids)
    log("plain rDDMC on the same clouds and packet ids")
    tp, _ = timed_steps(plain, 1, 0)
    rp = plain.results()
    ns, npl = sum(r.launched for r in rs), sum(r.launched for r in rp)
    v_s, v_p = ns / ts, npl / tp
    agree = [spectrum_agreement(a, b) for a, b in zip(rs, rp)]
    l1s = [a for a, _ in agree]
    noise = [b for _, b in agree]
    log(f"surrogate vs plain spectra (40 groups): mean L1 {sum(l1s) / len(l1s):.4f}, noise {sum(noise) / len(noise):.4f}")
    out = base_line(
        args, v_s, ts, "bf16 network (f32 accumulate), f32 walk",
        {"workload": f"{len(ids)} sweep clouds with cells in the surrogate's domain (used at tau_c {use.tau_min:g}-"
                     f"{use.tau_max:g}, trained at {dom.tau_min:g}-{dom.tau_max:g}, dx {dom.dx_min}-{dom.dx_max}), "
                     f"one batch, {args.surrogate_packets} "
                     "packets per cloud, surrogate and plain on the same packet ids",
         "clouds": ids, "window_states": int(att.n_states),
         "surrogate_calls_per_packet": sum(r.surrogate_calls for r in rs) / ns,
         "steps_per_packet_surrogate": sum(r.steps_total for r in rs) / ns,
         "steps_per_packet_plain": sum(r.steps_total for r in rp) / npl,
         "data_s": t_data, "train_s": t_train, "train_samples": data.n, "walked_samples": n_walked,
         "train_epochs": epochs, "step_budget": budget, "final_nll": hist[-1], "heldout_nll": nll_held,
         "spectrum_l1_vs_plain_40_groups": {"mean": sum(l1s) / len(l1s), "max": max(l1s),
                                            "noise_mean": sum(noise) / len(noise),
                                            "max_ratio_to_noise": max(a / b for a, b in agree)}},
        plain_packets_per_s=v_p, speedup=v_s / v_p)
    out["roofline"] = None
    return out


def bench_methods(args):
    """rDDMC against frequency-group and continuous-frequency Monte Carlo on static slabs: each
    method walks the same 2^16 packet ids of each slab whole in one launch (tables built
    untimed).  Events are DDMC leaks for rDDMC, scatterings and cell-face crossings for the
    Monte Carlo methods."""
    import numpy as np
    import torch
    from paper_1709_10187_amd import media, rddmc
    n = 1 << 16
    rows, headline = [], None
    for tau0 in args.methods_tau0:
        base = media.slab(tau0, 1e4, 64, 128, n_packets=n, name=f"slab_tau{tau0:.0e}")
        legs = {"rddmc": base}
        try:   # the efficient grid needs the spectrum to reach beyond the core (a tau0 >~ 2.5)
            eff = media.efficient_edges(media._a_of_T(1e4), tau0, 1.0 / 32)
            legs["rddmc_efficient"] = base.replace(bin_edges=eff)
        except ValueError:
            eff = None
        legs["groups"] = base.replace(tau_threshold=media.ALL_THIN, flags=media.GROUP_MC)
        legs["mcrt"] = base.replace(tau_threshold=media.ALL_THIN)
        # continuous MC with core-skipping (the kind of MCRT the paper compares with): a photon
        # scattered at |x| < 3 takes the atom's perpendicular speed from the Maxwellian above 3
        legs["mcrt_cs"] = base.replace(tau_threshold=media.ALL_THIN, x_crit=3.0)
        legs = {k: v for k, v in legs.items() if k in args.methods_legs}
        row = {"tau0": tau0, "dx": float(base.bin_edges[1] - base.bin_edges[0])}
        spectra = {}
        for leg, m in legs.items():
            prob = rddmc.Problem(m)
            torch.cuda.synchronize()
            start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            start.record()
            prob.run(seed=0)
            stop.record()
            torch.cuda.synchronize()
            sec = start.elapsed_time(stop) / 1e3
            r = prob.results()[0]
            events = r.steps_total
            spectra[leg] = r.spectrum.sum(axis=0)[1:-1].astype(np.float64) / max(r.escaped, 1)
            row[leg] = {"packets_per_s": n / sec, "events_per_packet": events / n, "events_per_s": events / sec,
                        "seconds": sec, "t_mean": r.t_mean}
            log(f"tau0 {tau0:.0e} {leg}: {sec:.3f} s, {n / sec:.4g} packets/s, {events / n:.4g} events/packet")
            del prob
        if eff is not None:
            row["efficient_bins"] = len(eff) - 1
        if "mcrt" in row:
            for leg in ("rddmc", "rddmc_efficient", "groups", "mcrt_cs"):
                if leg in row:
                    row[f"speedup_{leg}_vs_mcrt"] = row[leg]["packets_per_s"] / row["mcrt"]["packets_per_s"]
                    if leg != "rddmc_efficient":
                        row[f"L1_{leg}_vs_mcrt"] = float(np.abs(spectra[leg] - spectra["mcrt"]).sum())
        if "mcrt_cs" in row:
            for leg in ("rddmc", "rddmc_efficient", "groups"):
                if leg in row:
                    row[f"speedup_{leg}_vs_mcrt_cs"] = row[leg]["packets_per_s"] / row["mcrt_cs"]["packets_per_s"]
        rows.append(row)
        if headline is None or tau0 == 1e5:
            headline = row
    lead = next(leg for leg in ("rddmc", "rddmc_efficient", "groups", "mcrt", "mcrt_cs") if leg in headline)
    out = base_line(
        args, headline[lead]["packets_per_s"], n / headline[lead]["packets_per_s"], "f32",
        {"workload": "static uniform slabs tau0 = 1e3..1e6, T = 1e4 K, 64 cells x 128 bins over "
                     "|x| <= 6 (a tau0)^(1/3), central source x = 0, 2^16 packets each, walked whole by rDDMC, "
                     "rDDMC on the efficient frequency grid (central bin 2 x_cw, unit wings), frequency-group "
                     "Monte Carlo (eq. 42), continuous-frequency Monte Carlo, and the latter with core-skipping "
                     "(x_crit = 3) on the same packet ids; "
                     "value = rDDMC on the tau0 = 1e5 slab (or the first method and slab asked for)",
         "methods": rows,
         "precision": "f32 walk, f64 tables (eq. 42 tables in f64), f64 clock, i64 tallies, Philox4x32-10"},
        packet_steps_per_s=headline[lead]["events_per_s"])
    out["roofline"] = None   # a comparison of methods; the kernels' own rooflines are the other workloads'
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_1d(media.config_slab(), args.cpu_packets or 4096, args)
        out["config"]["cpu_mcrt"] = cpu_mcrt_slabs(args)
    return out


def bench_census(args):
    """The cost of the census estimators (eq. 17 bin and path, eq. 18) on the config slab: the
    same packet ids (2^16 unless --census-packets) walked whole by the pure walk, by the hybrid walk (forced by a zero
    emission window, which is the same flash) without estimators, and by the hybrid walk with
    16 census intervals spanning 0..3 mean escape times.  The two hybrid legs draw the same
    random words, so their escape tallies are identical."""
    import numpy as np
    import torch
    from paper_1709_10187_amd import media, rddmc
    m = media.config_slab()
    if args.census_packets:
        m = m.with_packets(args.census_packets)
    n = int(m.n_packets)
    legs, tmean = {}, None
    for leg in ("pure", "hybrid", "census"):
        mm = m
        if leg != "pure":
            mm = m.replace(src_t=np.array([[0.0, 0.0]]))
        if leg == "census":
            mm = mm.replace(census=np.linspace(0.0, 3.0 * tmean, 17))
        prob = rddmc.Problem(mm)
        torch.cuda.synchronize()
        start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record()
        prob.run(seed=0)
        stop.record()
        torch.cuda.synchronize()
        sec = start.elapsed_time(stop) / 1e3
        r = prob.results()[0]
        tmean = tmean or r.t_mean
        legs[leg] = {"seconds": sec, "packets_per_s": n / sec, "steps_per_s": r.steps_total / sec,
                     "steps_per_packet": r.steps_mean, "steps_max": int(r.steps_max), "spectrum": r.spectrum.copy()}
        log(f"census workload, {leg}: {sec:.3f} s, {n / sec:.4g} packets/s, {r.steps_total / sec:.4g} steps/s")
        del prob
    same = np.array_equal(legs["census"]["spectrum"], legs["hybrid"]["spectrum"])
    for v in legs.values():
        del v["spectrum"]
    out = base_line(
        args, legs["census"]["packets_per_s"], legs["census"]["seconds"], "f32",
        {"workload": f"static slab tau0 = 1e5, T = 1e4 K, 64 cells x 128 bins, {n} packets, walked whole by the "
                     "pure 1D walk, the hybrid 1D walk without estimators and the hybrid walk with 16 census "
                     "intervals over 0..3 mean escape times (eq. 17 bin and path, eq. 18); value = the census leg",
         "legs": legs, "hybrid_spectra_identical": bool(same),
         "census_cost": legs["hybrid"]["packets_per_s"] / legs["census"]["packets_per_s"]},
        packet_steps_per_s=legs["census"]["steps_per_s"])
    out["roofline"] = None   # the estimators' cost against the same walk without them
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_1d(media.config_slab(), args.cpu_packets or 4096, args)
    return out


def cpu_mcrt_slabs(args):
    """The oracle's continuous-frequency Monte Carlo (the 1D hybrid walker with every state thin)
    on the host's cores: 4096 packets of the tau0 = 1e3 slab and 1024 of the 1e4 slab of the
    methods workload."""
    from paper_1709_10187_amd import media
    from oracle import walk1dh as ow1h
    threads = _threads(args)
    out = []
    for tau0, n in ((1e3, 4096), (1e4, 1024)):
        m = media.slab(tau0, 1e4, 64, 128, tau_threshold=media.ALL_THIN)
        t0 = time.perf_counter()
        w = ow1h.run(m, n_packets=n, seed=0, n_threads=threads)
        dt = time.perf_counter() - t0
        out.append({"tau0": tau0, "packets": n, "packets_per_s": n / dt, "events_per_packet": w.mc_steps_sum / n,
                    "cores": threads})
        log(f"cpu mcrt tau0 {tau0:.0e}: {n / dt:.4g} packets/s")
    return out


def _threads(args):
    return args.cpu_threads or min(16, os.cpu_count() or 1)


def cpu_baseline_cube(args):
    """The oracle's literal FP64 hybrid walker (O1-3D) on the host's cores.  Its FP64 tables
    for the 128^3 cube (5.4e8 states, ~60 GB, ~10 min of numpy) do not fit a bench run, so it
    walks a packet sample of the same-recipe 32^3 cube; the comparable rate is packet-steps/s."""
    from paper_1709_10187_amd import media
    from oracle import tables as otb
    from oracle import walk3d as ow3
    threads = _threads(args)
    n = args.cpu_packets or (1 << 20)
    m = media.cube(n=32)
    log(f"cpu baseline: oracle 3D walker, {n} packets of the 32^3 cube, {threads} threads")
    t = otb.build(m)
    t0 = time.perf_counter()
    w = ow3.run(m, n_packets=n, seed=0, n_threads=threads, tabs=t)
    dt = time.perf_counter() - t0
    return {"value": w.steps_sum / dt, "unit": "packet-steps/s", "cores": threads, "kind": "oracle",
            "packets_per_s": n / dt,
            "sample": f"packets 0..{n - 1} of the same-recipe 32^3 cube (PCG64(4), 64 densest-cell sources, "
                      f"256 bins of 25 km/s, tau_th 10; own xoshiro256** streams): {w.steps_sum:.3e} steps "
                      f"({w.mc_steps_sum:.3e} MC) in {dt:.1f} s"}


def cpu_baseline_1d(m, n_packets, args):
    """The oracle's literal FP64 1D walker (O1) on the host's cores on a bounded sample."""
    from oracle import tables as otb
    from oracle import walk as owalk
    threads = _threads(args)
    log(f"cpu baseline: oracle walker, {n_packets} packets, {threads} threads")
    t = otb.build(m)
    t0 = time.perf_counter()
    w = owalk.run(m, n_packets=n_packets, seed=0, n_threads=threads, tabs=t)
    dt = time.perf_counter() - t0
    return {"value": w.n_packets / dt, "unit": "packets/s", "cores": threads, "kind": "oracle",
            "packet_steps_per_s": w.steps_sum / dt,
            "sample": f"packets 0..{n_packets - 1} of the same job (own xoshiro256** streams), "
                      f"{w.steps_sum:.3e} steps in {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this path runs on one GPU; --gpus must be 1 (sharding over GPUs is a "
                                   "design, not built)"}))
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    fn = {"cube": bench_cube, "sphere": bench_sphere, "sphere-efficient": lambda a: bench_sphere(a, efficient=True),
          "surrogate": bench_surrogate, "sweep": bench_sweep, "sweep-full": bench_sweep_full,
          "methods": bench_methods, "census": bench_census}
    print(json.dumps(fn[args.workload](args)), flush=True)


if __name__ == "__main__":
    main()
