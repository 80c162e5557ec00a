"""Host-side parts of bench.py: the one-GPU guard, the HBM traffic taken from the committed
counter summary while the kernel's sources are unchanged, and the two-sample spectrum
agreement the surrogate workload reports."""
import importlib.util
import json
import os
import subprocess
import sys
import types

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_cube_traffic_comes_from_the_committed_counters_of_the_current_sources():
    b = _bench()
    t = b.profiled_traffic("walk3d_cube128_job_pmc.md", "walk3d")
    assert t is not None, "walk3d's sources changed since its FETCH_SIZE / WRITE_SIZE counters were taken"
    with open(os.path.join(ROOT, "profiles", "walk3d_cube128_job_pmc.md")) as f:
        m = b.TRAFFIC_RE.search(f.read())
    assert t == float(m.group(1))
    assert b.profiled_traffic("no_such_profile.md", "walk3d") is None


def _res(counts):
    return types.SimpleNamespace(spectrum=np.asarray(counts)[None, :])


def test_spectrum_agreement_noise_level_and_a_shifted_sample():
    """Under the null (two samples of one law) the mean L1 equals the reported noise level;
    a law shifted by a few bins gives an L1 far above it."""
    b = _bench()
    rng = np.random.default_rng(5)
    p = rng.dirichlet(np.full(300, 2.0))
    runs = [b.spectrum_agreement(_res(rng.multinomial(4096, p)), _res(rng.multinomial(4096, p)))
            for _ in range(300)]
    l1 = np.mean([a for a, _ in runs])
    noise = np.mean([c for _, c in runs])
    assert abs(l1 / noise - 1.0) < 0.05
    x = np.arange(300)
    q = np.exp(-0.5 * ((x - 150) / 20.0) ** 2)
    q2 = np.roll(q, 12)
    a, n = b.spectrum_agreement(_res(rng.multinomial(4096, q / q.sum())), _res(rng.multinomial(4096, q2 / q2.sum())))
    assert a > 5 * n
