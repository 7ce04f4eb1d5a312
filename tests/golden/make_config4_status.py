"""Writes config4_status.txt: the oracle's set-up status (geometry and
collocation, steps S0 + S1) of every problem of the seeded batch of 512
random stars (N in {64, 128, 256, 512}, r = 0.4 + sum_k a_k cos(k t + p_k),
a_k ~ U(0, 0.04)).  Calls the oracle only.

    python tests/golden/make_config4_status.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import geometry, kfbi  # noqa: E402
from paper_2309_05965_amd import workloads as W  # noqa: E402


def main():
    lines = ["# problem N status (oracle set-up of the 512-star batch, seed %d)" % W.SEED_BATCH]
    for i, (prob, _) in enumerate(W.config4_batch()):
        try:
            kfbi.Plan(prob)
            st = "ok"
        except geometry.GeometryError as e:
            st = e.status
        lines.append("%d %d %s" % (i, prob["N"], st))
    with open(os.path.join(HERE, "config4_status.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
