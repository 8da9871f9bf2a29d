"""The oracle still reproduces its stored values (tests/golden, written by
tests/golden/make_golden.py from the oracle alone)."""
import os

import pytest

from oracle import network as nw
from oracle import plan as P

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def ising_rows():
    with open(os.path.join(GOLD, "ising_logz.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                r, c, K, v = line.split()
                yield int(r), int(c), float(K), float(v)


@pytest.mark.parametrize("r,c,K,v", list(ising_rows()))
def test_ising_golden(r, c, K, v):
    assert abs(nw.transfer_log_z(r, c, K) - v) <= 1e-13 * abs(v)


@pytest.mark.parametrize("name", sorted(n for n in os.listdir(GOLD) if n.startswith("plan_")))
def test_plan_golden(name):
    stem = name[len("plan_"):-len(".txt")]
    shape, d, order = stem.split("_")
    r, c = (int(x) for x in shape.split("x"))
    o = {"colsweep": P.COLSWEEP, "quadrant": P.QUADRANT, "heuristic": P.HEURISTIC}[order]
    with open(os.path.join(GOLD, name)) as f:
        assert P.plan_text(P.plan_grid(r, c, int(d[1:]), order=o)) == f.read()
