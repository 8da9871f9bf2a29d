"""Write the stored expected values under tests/golden/.

Every value here is produced by the CPU oracle only (``oracle/``): the Ising
transfer matrix for log Z, and the oracle's planner for canonical plan text.
Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import network as nw  # noqa: E402
from oracle import plan as P      # noqa: E402

ISING = [(4, 4, 0.4), (10, 10, 0.2), (10, 10, 0.44), (10, 10, 0.6),
         (12, 12, 0.44), (13, 13, 0.44), (8, 8, 0.1), (8, 8, 0.8)]

PLANS = [(4, 4, 2, P.COLSWEEP), (4, 4, 2, P.QUADRANT), (3, 5, 3, P.HEURISTIC),
         (2, 1, 2, P.COLSWEEP), (1, 1, 2, P.COLSWEEP)]


def main():
    with open(os.path.join(HERE, "ising_logz.txt"), "w") as f:
        f.write("# rows cols betaJ logZ  (open-boundary Ising, h=0; row transfer matrix)\n")
        for r, c, K in ISING:
            f.write(f"{r} {c} {K!r} {nw.transfer_log_z(r, c, K)!r}\n")
    for r, c, D, o in PLANS:
        name = f"plan_{r}x{c}_D{D}_{P.ORDER_NAMES[o].lower()}.txt"
        with open(os.path.join(HERE, name), "w") as f:
            f.write(P.plan_text(P.plan_grid(r, c, D, order=o)))


if __name__ == "__main__":
    main()
