"""Writes tests/golden/chain_regression.json: the exact chain's (oracle O2) expected steps,
escape time and total escape probability for the 64 x 128 slab (tau0 = 1e5, T = 1e4 K) and
the 256 x 512 sphere (tau0 = 1e7).  Regression values only: they guard the oracle against
unintended changes of its arithmetic and pin nothing by themselves (the chain is pinned by
the closed forms and brute-force checks in tests/test_oracle_chain.py).

    python tests/golden/make_chain_regression.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import chain  # noqa: E402
from paper_1709_10187_amd import media  # noqa: E402


def main():
    out = {"_what": "exact-chain regression values (oracle O2), written by make_chain_regression.py"}
    for name, m in (("slab_tau1e5_64x128", media.config_slab()), ("sphere_tau1e7_256x512", media.config_sphere())):
        r = chain.solve(m)
        out[name] = {"steps": r.steps, "steps2": r.steps2, "t_mean": r.t_mean, "t2": r.t2, "total": r.total}
    with open(os.path.join(HERE, "chain_regression.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
