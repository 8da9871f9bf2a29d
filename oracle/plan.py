"""Contraction orders for the planar network, written from the paper's §4.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper contracts the network by pairwise, sequential contractions and
tracks the number of elements of every intermediate (its "dimension"); the
largest intermediate is the bottleneck that sets memory and operation count
(§4, the dimension rule and the "bottleneck contraction" paragraph).  Two
orders are described (§4, Fig. 2): contracting along rows from one edge to
the other (a chain of chi^L-element tensors), and contracting each of four
quadrants from its outer edges towards the middle, leaving a ring of four
tensors.  The heuristic picks the order with the smallest bottleneck (§4,
last paragraph).

Readings taken where the text is silent or garbled:

* Dimension rule: §4 prints d(B) = d(A1) d(A2) / d(x); the shared legs sit on
  both operands, so the rule applied here (by literally tracking legs) is
  d(B) = d(A1) d(A2) / d(x)^2.
* The row scheme is realised sequentially as a column sweep: one boundary
  tensor absorbs the sites column by column, top to bottom (or, transposed,
  row by row).  The absorbed site's shared legs are replaced in place by its
  remaining legs (right leg, then down leg, in the sweep's own frame).
* Quadrants: rows [0,h) / [h,R), columns [0,w) / [w,C); defaults h = ceil(R/2),
  w = ceil(C/2).  Each quadrant is swept in a frame whose origin is its outer
  lattice corner; legs that leave the quadrant stay on its tensor.
* Bottleneck = the largest intermediate entry count.  The heuristic orders
  candidates by (bottleneck, total flops, enumeration index) with the
  enumeration column sweep, transposed column sweep, then every quadrant
  split (h, w) in lexicographic order.
* An exact power-of-two rescale follows the last site of every column of a
  sweep, except the final column of a column sweep, which ends in the scalar.

Frames map a local site (i, j) of a sweep to a lattice site and the local
legs (L, U, R, Dn) to canonical legs (left=0, up=1, right=2, down=3).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

LEFT, UP, RIGHT, DOWN = 0, 1, 2, 3
INT64_MAX = (1 << 63) - 1

COLSWEEP, QUADRANT, HEURISTIC, SWEEP_AUTO = 0, 1, 2, 3
ORDER_NAMES = {COLSWEEP: "COLSWEEP", QUADRANT: "QUADRANT", HEURISTIC: "HEURISTIC",
               SWEEP_AUTO: "SWEEP_AUTO"}

# frame name -> (local L, U, R, Dn as canonical legs)
FRAME_LEGS = {
    "ID": (LEFT, UP, RIGHT, DOWN),
    "T": (UP, LEFT, DOWN, RIGHT),
    "MH": (RIGHT, UP, LEFT, DOWN),
    "MHV": (RIGHT, DOWN, LEFT, UP),
    "MV": (LEFT, DOWN, RIGHT, UP),
}


class PlanOverflow(Exception):
    pass


def _mul(a: int, b: int) -> int:
    r = a * b
    if r > INT64_MAX:
        raise PlanOverflow()
    return r


def _add(a: int, b: int) -> int:
    r = a + b
    if r > INT64_MAX:
        raise PlanOverflow()
    return r


def frame_site(frame: str, rows: int, cols: int, i: int, j: int) -> Tuple[int, int]:
    if frame == "ID":
        return i, j
    if frame == "T":
        return j, i
    if frame == "MH":
        return i, cols - 1 - j
    if frame == "MHV":
        return rows - 1 - i, cols - 1 - j
    if frame == "MV":
        return rows - 1 - i, j
    raise ValueError(frame)


def canonical_legs(rows: int, cols: int, r: int, c: int) -> List[int]:
    legs = []
    if c > 0:
        legs.append(LEFT)
    if r > 0:
        legs.append(UP)
    if c < cols - 1:
        legs.append(RIGHT)
    if r < rows - 1:
        legs.append(DOWN)
    return legs


def leg_bond(r: int, c: int, leg: int) -> Tuple[str, int, int]:
    if leg == LEFT:
        return ("h", r, c - 1)
    if leg == UP:
        return ("v", r - 1, c)
    if leg == RIGHT:
        return ("h", r, c)
    return ("v", r, c)


@dataclass
class Step:
    unit: int
    site: Tuple[int, int]
    kind: str                 # "INIT" or "ABSORB"
    pre: int
    K: int
    N: int
    post: int
    perm: Tuple[int, ...]     # canonical axes of the site, in [K legs][N legs] order
    out: int
    flops: int
    rescale: int = -1         # exponent slot written after this step, or -1


@dataclass
class Unit:
    frame: str
    rows: int                 # local rows
    cols: int                 # local columns
    result: int = 0           # entries of the unit's final tensor
    legs: List = field(default_factory=list)   # bond ids of the final tensor


@dataclass
class Ring:
    xa: int
    xb: int
    ya: int
    yb: int
    m: int
    n: int
    kx: int
    ky: int
    flops: int


@dataclass
class Plan:
    rows: int
    cols: int
    hdim: np.ndarray
    vdim: np.ndarray
    requested: int
    order: int
    transpose: int
    quad: Tuple[int, int]
    units: List[Unit]
    steps: List[Step]
    ring: Optional[Ring]
    slots: int
    peak: int
    flops: int
    moved: int


def _bond_dim(b, hdim, vdim) -> int:
    kind, r, c = b
    return int(hdim[r][c]) if kind == "h" else int(vdim[r][c])


def _sweep(rows, cols, hdim, vdim, unit_id, frame, nh, nw,
           rescale_last: bool, slot0: int):
    """Sweep one region: local rows [0,nh), columns [0,nw) of ``frame``.
    Returns (steps, final legs, next free slot)."""
    fl = FRAME_LEGS[frame]
    steps: List[Step] = []
    boundary: List[Tuple[str, int, int]] = []
    slot = slot0
    for j in range(nw):
        for i in range(nh):
            r, c = frame_site(frame, rows, cols, i, j)
            canon = canonical_legs(rows, cols, r, c)
            axis_of = {leg: a for a, leg in enumerate(canon)}
            present = {loc: fl[loc] for loc in range(4) if fl[loc] in axis_of}
            # local L (0) and U (1) are shared with the boundary; R (2), Dn (3) are new
            shared = [leg_bond(r, c, present[loc]) for loc in (1, 0) if loc in present]
            new_locs = [loc for loc in (2, 3) if loc in present]
            new = [leg_bond(r, c, present[loc]) for loc in new_locs]
            if i == 0 and j == 0:
                assert not shared
                perm = tuple(axis_of[present[loc]] for loc in new_locs)
                n_entries = 1
                for b in new:
                    n_entries = _mul(n_entries, _bond_dim(b, hdim, vdim))
                boundary = list(new)
                steps.append(Step(unit_id, (r, c), "INIT", 1, 1, n_entries, 1,
                                  perm, n_entries, 0))
                continue
            pos = [boundary.index(b) for b in shared]
            k_start = min(pos)
            k_legs = boundary[k_start:k_start + len(shared)]
            assert sorted(k_legs) == sorted(shared), "shared legs are not adjacent"
            # map each boundary K leg back to the site axis carrying that bond
            kperm = []
            for b in k_legs:
                for loc in (0, 1):
                    if loc in present and leg_bond(r, c, present[loc]) == b:
                        kperm.append(axis_of[present[loc]])
            perm = tuple(kperm + [axis_of[present[loc]] for loc in new_locs])
            pre = 1
            for b in boundary[:k_start]:
                pre = _mul(pre, _bond_dim(b, hdim, vdim))
            post = 1
            for b in boundary[k_start + len(shared):]:
                post = _mul(post, _bond_dim(b, hdim, vdim))
            K = 1
            for b in k_legs:
                K = _mul(K, _bond_dim(b, hdim, vdim))
            N = 1
            for b in new:
                N = _mul(N, _bond_dim(b, hdim, vdim))
            out = _mul(_mul(pre, N), post)
            flops = _mul(_mul(out, K), 2)
            boundary = boundary[:k_start] + new + boundary[k_start + len(shared):]
            steps.append(Step(unit_id, (r, c), "ABSORB", pre, K, N, post,
                              perm, out, flops))
        if j < nw - 1 or rescale_last:
            steps[-1].rescale = slot
            slot += 1
    return steps, boundary, slot


def _finish(p_rows, p_cols, hdim, vdim, requested, order, transpose, quad,
            units, steps, ring, slots) -> Plan:
    peak = 0
    flops = 0
    moved = 0
    for s in steps:
        peak = max(peak, s.out)
        flops = _add(flops, s.flops)
        if s.kind == "ABSORB":
            moved = _add(moved, _add(_mul(_mul(s.pre, s.K), s.post), s.out))
    if ring is not None:
        peak = max(peak, _mul(ring.m, ring.n))
        flops = _add(flops, ring.flops)
        for u in units:
            moved = _add(moved, u.result)
        moved = _add(moved, _mul(_mul(ring.m, ring.n), 2))
    return Plan(p_rows, p_cols, hdim, vdim, requested, order, transpose, quad,
                units, steps, ring, slots, peak, flops, moved)


def plan_colsweep(rows, cols, hdim, vdim, transpose=0, requested=COLSWEEP) -> Plan:
    frame = "T" if transpose else "ID"
    nh, nw = (cols, rows) if transpose else (rows, cols)
    steps, legs, slots = _sweep(rows, cols, hdim, vdim, 0, frame, nh, nw,
                                False, 0)
    assert not legs
    u = Unit(frame, nh, nw, 1, [])
    return _finish(rows, cols, hdim, vdim, requested, COLSWEEP, transpose,
                   (0, 0), [u], steps, None, slots)


def plan_quadrant(rows, cols, hdim, vdim, h=0, w=0, requested=QUADRANT) -> Plan:
    if rows < 2 or cols < 2:
        raise ValueError("the quadrant order needs at least 2 rows and 2 columns")
    if h == 0:
        h = (rows + 1) // 2
    if w == 0:
        w = (cols + 1) // 2
    if not (1 <= h <= rows - 1 and 1 <= w <= cols - 1):
        raise ValueError("quadrant split out of range")
    regions = [("ID", h, w), ("MH", h, cols - w), ("MHV", rows - h, cols - w),
               ("MV", rows - h, w)]
    units: List[Unit] = []
    steps: List[Step] = []
    slot = 0
    for uid, (frame, nh, nw) in enumerate(regions):
        st, legs, slot = _sweep(rows, cols, hdim, vdim, uid, frame, nh, nw,
                                True, slot)
        res = 1
        for b in legs:
            res = _mul(res, _bond_dim(b, hdim, vdim))
        units.append(Unit(frame, nh, nw, res, legs))
        steps += st
    # TL = [b][a_tl], TR = [b][a_tr], BR = [d][a_tr], BL = [d][a_tl]
    kx = 1
    for r in range(h):
        kx = _mul(kx, int(hdim[r][w - 1]))
    ky = 1
    for r in range(h, rows):
        ky = _mul(ky, int(hdim[r][w - 1]))
    m = 1
    for c in range(w):
        m = _mul(m, int(vdim[h - 1][c]))
    n = 1
    for c in range(w, cols):
        n = _mul(n, int(vdim[h - 1][c]))
    # leg bookkeeping check: the four tensors carry exactly these legs
    b_legs = [("h", r, w - 1) for r in range(h)]
    d_legs = [("h", r, w - 1) for r in range(rows - 1, h - 1, -1)]
    a_tl = [("v", h - 1, c) for c in range(w - 1, -1, -1)]
    a_tr = [("v", h - 1, c) for c in range(w, cols)]
    assert units[0].legs == b_legs + a_tl
    assert units[1].legs == b_legs + a_tr
    assert units[2].legs == d_legs + a_tr
    assert units[3].legs == d_legs + a_tl
    mn = _mul(m, n)
    rflops = _add(_add(_mul(_mul(mn, kx), 2), _mul(_mul(mn, ky), 2)), _mul(mn, 2))
    ring = Ring(0, 1, 3, 2, m, n, kx, ky, rflops)
    return _finish(rows, cols, hdim, vdim, requested, QUADRANT, 0, (h, w),
                   units, steps, ring, slot)


def plan_grid(rows: int, cols: int, D: int = 2, hdim=None, vdim=None,
              order: int = COLSWEEP, quad_h: int = 0, quad_w: int = 0) -> Plan:
    """Build a plan; raises PlanOverflow if any integer exceeds int64."""
    if rows < 1 or cols < 1:
        raise ValueError("rows and cols must be >= 1")
    if hdim is None:
        hdim = np.full((rows, max(cols - 1, 0)), D, dtype=np.int64)
    if vdim is None:
        vdim = np.full((max(rows - 1, 0), cols), D, dtype=np.int64)
    hdim = np.asarray(hdim, dtype=np.int64).reshape(rows, max(cols - 1, 0))
    vdim = np.asarray(vdim, dtype=np.int64).reshape(max(rows - 1, 0), cols)
    if order == COLSWEEP:
        return plan_colsweep(rows, cols, hdim, vdim, 0)
    if order == QUADRANT:
        return plan_quadrant(rows, cols, hdim, vdim, quad_h, quad_w)
    if order == SWEEP_AUTO:
        # the sweep orientation with the smaller bottleneck (then fewer flops,
        # then untransposed): the boundary runs along the shorter side
        cands = []
        for t in (0, 1):
            try:
                cands.append(plan_colsweep(rows, cols, hdim, vdim, t, SWEEP_AUTO))
            except PlanOverflow:
                pass
        if not cands:
            raise PlanOverflow()
        best = min(range(len(cands)), key=lambda k: (cands[k].peak, cands[k].flops, k))
        return cands[best]
    if order == HEURISTIC:
        cands = []
        for t in (0, 1):
            try:
                cands.append(plan_colsweep(rows, cols, hdim, vdim, t, HEURISTIC))
            except PlanOverflow:
                pass
        if rows >= 2 and cols >= 2:
            for h in range(1, rows):
                for w in range(1, cols):
                    try:
                        cands.append(plan_quadrant(rows, cols, hdim, vdim, h, w,
                                                   HEURISTIC))
                    except PlanOverflow:
                        pass
        if not cands:
            raise PlanOverflow()
        best = min(range(len(cands)), key=lambda k: (cands[k].peak, cands[k].flops, k))
        return cands[best]
    raise ValueError("unknown order")


def _ints(a) -> str:
    flat = [str(int(x)) for x in np.asarray(a).reshape(-1)]
    return ",".join(flat) if flat else "-"


def plan_text(p: Plan) -> str:
    """Canonical text of a plan: one line per item, integers in decimal."""
    lines = [f"tnplan v1 rows={p.rows} cols={p.cols} requested={ORDER_NAMES[p.requested]}"
             f" order={ORDER_NAMES[p.order]} transpose={p.transpose}"
             f" quad={p.quad[0]},{p.quad[1]}",
             f"hdim {_ints(p.hdim)}",
             f"vdim {_ints(p.vdim)}"]
    for k, u in enumerate(p.units):
        lines.append(f"unit {k} frame={u.frame} rows={u.rows} cols={u.cols}"
                     f" result={u.result}")
    for k, s in enumerate(p.steps):
        perm = ".".join(str(a) for a in s.perm) if s.perm else "-"
        resc = str(s.rescale) if s.rescale >= 0 else "-"
        lines.append(f"step {k} unit={s.unit} site={s.site[0]},{s.site[1]} kind={s.kind}"
                     f" pre={s.pre} K={s.K} N={s.N} post={s.post} perm={perm}"
                     f" out={s.out} flops={s.flops} rescale={resc}")
    if p.ring is not None:
        g = p.ring
        lines.append(f"ring xa={g.xa} xb={g.xb} ya={g.ya} yb={g.yb} m={g.m} n={g.n}"
                     f" kx={g.kx} ky={g.ky} flops={g.flops}")
    lines.append(f"totals steps={len(p.steps)} slots={p.slots} peak={p.peak}"
                 f" flops={p.flops} moved={p.moved}")
    return "\n".join(lines) + "\n"
