"""Test statistics for Monte Carlo spectra (per-bin z within 3 sigma, chi^2, L1).

Rules: spectra are compared as escape fractions over the lab slots; bins whose
expected count is below 10 are merged into their neighbours; the per-bin sigma
against an exact expectation is sqrt(p (1 - p) / N), against another Monte
Carlo sample sqrt(s1^2 + s2^2).  Pass:
  * "within 3 sigma per bin": the number of bins with |z| > 3 is no larger than a
    Binomial(n_bins, 0.0027) count exceeds with probability 1e-3 (for many bins this is
    the ">= 99 % of bins" rule; for ~100 bins it allows the 0-3 chance excursions a
    correct sampler produces), and no bin has |z| > 5;
  * chi^2 p-value >= 1e-3;
  * L1 <= the stated bound.
"""
import numpy as np
from scipy import stats


def _merge(expected_counts, *arrays, min_count=10.0):
    """Greedy left-to-right merge of consecutive bins until each group expects >= min_count."""
    groups, cur, acc = [], [], 0.0
    for i, e in enumerate(expected_counts):
        cur.append(i)
        acc += e
        if acc >= min_count:
            groups.append(cur)
            cur, acc = [], 0.0
    if cur:
        if groups:
            groups[-1].extend(cur)
        else:
            groups.append(cur)
    return [np.array([a[g].sum() for g in groups]) for a in arrays]


def compare_exact(counts, p, n=None):
    """counts: observed integer counts per slot; p: exact probabilities per slot."""
    counts = np.asarray(counts, dtype=np.float64).ravel()
    p = np.maximum(np.asarray(p, dtype=np.float64).ravel(), 0.0)   # exact zeros may round to -1e-17
    N = counts.sum() if n is None else n
    c, q = _merge(p * N, counts, p)
    f = c / N
    sig = np.sqrt(np.maximum(q * (1 - q), 1e-300) / N)
    z = (f - q) / sig
    chi2 = float(np.sum((c - q * N) ** 2 / np.maximum(q * N, 1e-300)))
    dof = max(len(c) - 1, 1)
    return {"z": z, "frac_within_3sigma": float(np.mean(np.abs(z) <= 3)), "max_abs_z": float(np.abs(z).max()),
            "chi2": chi2, "dof": dof, "p_value": float(stats.chi2.sf(chi2, dof)),
            "L1": float(np.abs(counts / N - p).sum()),
            "expected_noise_L1": float(np.sum(np.sqrt(2 / np.pi * p * (1 - p) / N)))}


def compare_two_samples(c1, c2):
    c1 = np.asarray(c1, dtype=np.float64).ravel()
    c2 = np.asarray(c2, dtype=np.float64).ravel()
    n1, n2 = c1.sum(), c2.sum()
    pooled = (c1 + c2) / (n1 + n2)
    a, b, q = _merge(pooled * min(n1, n2), c1, c2, pooled)
    f1, f2 = a / n1, b / n2
    sig = np.sqrt(q * (1 - q) * (1 / n1 + 1 / n2))
    z = (f1 - f2) / np.maximum(sig, 1e-300)
    chi2 = float(np.sum(z ** 2))
    dof = max(len(a) - 1, 1)
    return {"z": z, "frac_within_3sigma": float(np.mean(np.abs(z) <= 3)), "max_abs_z": float(np.abs(z).max()),
            "chi2": chi2, "dof": dof, "p_value": float(stats.chi2.sf(chi2, dof)),
            "L1": float(np.abs(c1 / n1 - c2 / n2).sum())}


def compare_weighted_exact(w, w2, n, p):
    """Weighted escapes (continuous dust weights) against an exact expectation: w, w2 the escaped
    weight and squared weight per slot over n packets, p the exact escape probability per slot
    (the expected weight).  Bins expecting < 10 packets' weight are merged; the per-bin sigma is
    the sample's own, sqrt((w2 / n - (w / n)^2) / n)."""
    w = np.asarray(w, dtype=np.float64).ravel()
    w2 = np.asarray(w2, dtype=np.float64).ravel()
    p = np.maximum(np.asarray(p, dtype=np.float64).ravel(), 0.0)
    a, b, q = _merge(p * n, w, w2, p)
    var = np.maximum(b / n - (a / n) ** 2, 1e-300) / n
    z = (a / n - q) / np.sqrt(var)
    chi2 = float(np.sum(z ** 2))
    dof = max(len(a), 1)
    return {"z": z, "frac_within_3sigma": float(np.mean(np.abs(z) <= 3)), "max_abs_z": float(np.abs(z).max()),
            "chi2": chi2, "dof": dof, "p_value": float(stats.chi2.sf(chi2, dof)),
            "L1": float(np.abs(w / n - p).sum())}


def compare_weighted_two(w_a, w2_a, n_a, w_b, w2_b, n_b):
    """Two samples of weighted escapes (either may be unweighted: then w2 = w, the counts):
    per-bin differences of the mean weight per packet over their joint sigma."""
    wa, w2a, wb, w2b = (np.asarray(v, dtype=np.float64).ravel() for v in (w_a, w2_a, w_b, w2_b))
    pooled = (wa + wb) / (n_a + n_b)
    a1, a2, b1, b2 = _merge(pooled * min(n_a, n_b), wa, w2a, wb, w2b)
    va = np.maximum(a2 / n_a - (a1 / n_a) ** 2, 0.0) / n_a
    vb = np.maximum(b2 / n_b - (b1 / n_b) ** 2, 0.0) / n_b
    z = (a1 / n_a - b1 / n_b) / np.sqrt(np.maximum(va + vb, 1e-300))
    chi2 = float(np.sum(z ** 2))
    dof = max(len(a1), 1)
    return {"z": z, "frac_within_3sigma": float(np.mean(np.abs(z) <= 3)), "max_abs_z": float(np.abs(z).max()),
            "chi2": chi2, "dof": dof, "p_value": float(stats.chi2.sf(chi2, dof)),
            "L1": float(np.abs(wa / n_a - wb / n_b).sum())}


def allowed_3sigma_exceedances(n_bins, p_fail=1e-3):
    k = 0
    while stats.binom.sf(k, n_bins, 0.0027) >= p_fail:
        k += 1
    return k


def assert_spectrum_matches(res, l1_max=None):
    z = np.abs(res["z"])
    assert int(np.sum(z > 3)) <= allowed_3sigma_exceedances(len(z)), res
    assert z.max() <= 5.0, res
    assert res["p_value"] >= 1e-3, res
    if l1_max is not None:
        assert res["L1"] <= l1_max, res


def run_watched(prob, seed, poll_s=10.0, label="", **kw):
    """One transport launch of ``prob`` on a side stream (a single tail for the whole run),
    with the tallies read on another stream every ``poll_s`` seconds and a line printed
    whenever more packets have finished: long GPU steps report their own progress."""
    import time
    import torch
    from paper_1709_10187_amd import rddmc
    cur = torch.cuda.current_stream()
    run_s, poll_st = torch.cuda.Stream(), torch.cuda.Stream()
    stop = torch.cuda.Event()
    run_s.wait_stream(cur)
    rddmc.transport(prob.batch, prob.tables, prob.tallies, prob.work, seed=seed, stream=run_s, **kw)
    stop.record(run_s)
    t0, last = time.perf_counter(), 0
    while not stop.query():
        time.sleep(poll_s)
        done = sum(r.escaped + r.capped + r.absorbed for r in rddmc.tally(prob.batch, prob.tallies, stream=poll_st))
        if done > last:
            print(f"    {label}{done} packets finished ({time.perf_counter() - t0:.0f} s)", flush=True)
            last = done
    torch.cuda.synchronize()
