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

COLSWEEP, QUADRANT, HEURISTIC, SWEEP_AUTO, ROWS, ROWS_T = 0, 1, 2, 3, 4, 5
ORDER_NAMES = {COLSWEEP: "COLSWEEP", QUADRANT: "QUADRANT", HEURISTIC: "HEURISTIC",
               SWEEP_AUTO: "SWEEP_AUTO", ROWS: "ROWS", ROWS_T: "ROWS_T"}

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
class Link:
    """One link of the row chain: v <- v . R (side 0, R = unit's tensor as
    [K][N]) or v <- R . v (side 1, R as [N][K]); K = the row's up legs."""
    unit: int
    side: int
    K: int
    N: int
    flops: int
    rescale: int = -1


class PlanTooLarge(Exception):
    """No candidate order fits the intermediate-storage budget."""


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
    chain: List[Link] = field(default_factory=list)
    buffers: int = 0          # intermediate storage, entries (see _buffers)


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


def _buffers(units, steps, ring, chain) -> int:
    """Entries of intermediate storage a plan keeps at once when every unit
    holds two buffers (input and output of its current step) of its largest
    intermediate until the end, plus the stored ring product, or two chain
    vectors of the largest link output.  (§4: the bottleneck tensor sets the
    memory; this counts everything live alongside it.)"""
    total = 0
    for u in range(len(units)):
        big = max((s.out for s in steps if s.unit == u), default=1)
        total = _add(total, _mul(big, 2))
    if ring is not None:
        total = _add(total, _mul(ring.m, ring.n))
    if chain:
        total = _add(total, _mul(max(lk.N for lk in chain), 2))
    return total


def _finish(p_rows, p_cols, hdim, vdim, requested, order, transpose, quad,
            units, steps, ring, slots, chain=None) -> Plan:
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
    for lk in chain or []:
        peak = max(peak, lk.N)
        flops = _add(flops, lk.flops)
        moved = _add(moved, _add(_mul(lk.K, lk.N), _add(lk.K, lk.N)))
    return Plan(p_rows, p_cols, hdim, vdim, requested, order, transpose, quad,
                units, steps, ring, slots, peak, flops, moved, list(chain or []),
                _buffers(units, steps, ring, chain))


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


def _row_unit(rows, cols, hdim, vdim, frame, i, nw, uid, up_first, slot, rescale_last):
    """Contract local row i of ``frame`` into one tensor, left to right (§4,
    the row scheme).  Each site is joined by its local left leg; its other
    legs are new and go in place of the joined one, in the order up, right,
    down (``up_first``) or down, right, up.  The row tensor then holds its up
    legs left to right followed by its down legs right to left, or its down
    legs left to right followed by its up legs right to left.  Rescale after
    every step (except, with ``rescale_last`` false, the last)."""
    fl = FRAME_LEGS[frame]
    order = (1, 2, 3) if up_first else (3, 2, 1)
    steps: List[Step] = []
    boundary: List[Tuple[str, int, int]] = []
    for j in range(nw):
        r, c = frame_site(frame, rows, cols, i, j)
        canon = canonical_legs(rows, cols, r, c)
        axis_of = {leg: a for a, leg in enumerate(canon)}
        present = {loc: fl[loc] for loc in range(4) if fl[loc] in axis_of}
        new_locs = [loc for loc in order if loc in present]
        new = [leg_bond(r, c, present[loc]) for loc in new_locs]
        N = 1
        for b in new:
            N = _mul(N, _bond_dim(b, hdim, vdim))
        if j == 0:
            perm = tuple(axis_of[present[loc]] for loc in new_locs)
            boundary = list(new)
            steps.append(Step(uid, (r, c), "INIT", 1, 1, N, 1, perm, N, 0))
        else:
            joined = leg_bond(r, c, present[0])
            k = boundary.index(joined)
            pre = 1
            for b in boundary[:k]:
                pre = _mul(pre, _bond_dim(b, hdim, vdim))
            post = 1
            for b in boundary[k + 1:]:
                post = _mul(post, _bond_dim(b, hdim, vdim))
            K = _bond_dim(joined, hdim, vdim)
            perm = tuple([axis_of[present[0]]] + [axis_of[present[loc]] for loc in new_locs])
            out = _mul(_mul(pre, N), post)
            steps.append(Step(uid, (r, c), "ABSORB", pre, K, N, post, perm, out,
                              _mul(_mul(out, K), 2)))
            boundary = boundary[:k] + new + boundary[k + 1:]
        if j < nw - 1 or rescale_last:
            steps[-1].rescale = slot
            slot += 1
    return steps, boundary, slot


def plan_rows(rows, cols, hdim, vdim, transpose=0, requested=ROWS) -> Plan:
    """The paper's row scheme (§4, Fig. 2a): every lattice row (every column
    when transposed) is contracted into one tensor with all its vertical legs
    open, leaving a chain of row tensors, which is then contracted as an MPS
    from the first row down by matrix-vector products.  Even rows keep their
    up legs first, odd rows their down legs first, so the legs a link sums
    over sit in the same order on the chain vector and on the row tensor."""
    frame = "T" if transpose else "ID"
    nh, nw = (cols, rows) if transpose else (rows, cols)
    fl = FRAME_LEGS[frame]
    units: List[Unit] = []
    steps: List[Step] = []
    slot = 0
    for i in range(nh):
        st, legs, slot = _row_unit(rows, cols, hdim, vdim, frame, i, nw, i, i % 2 == 0,
                                   slot, nh > 1)
        res = 1
        for b in legs:
            res = _mul(res, _bond_dim(b, hdim, vdim))
        units.append(Unit(frame, 1, nw, res, legs))
        steps += st
    chain: List[Link] = []
    v = list(units[0].legs) if nh > 1 else []
    for i in range(1, nh):
        ups, downs = [], []
        for j in range(nw):
            r, c = frame_site(frame, rows, cols, i, j)
            ups.append(leg_bond(r, c, fl[1]))
            if i < nh - 1:
                downs.append(leg_bond(r, c, fl[3]))
        legs = units[i].legs
        if i % 2 == 0:       # [up left->right][down right->left]
            side, up_part, down_part = 0, legs[:nw], legs[nw:]
            assert up_part == ups and down_part == downs[::-1]
        else:                # [down left->right][up right->left]
            side, up_part, down_part = 1, legs[len(downs):], legs[:len(downs)]
            assert up_part == ups[::-1] and down_part == downs
        assert up_part == v, "chain legs out of order"
        K = 1
        for b in up_part:
            K = _mul(K, _bond_dim(b, hdim, vdim))
        N = 1
        for b in down_part:
            N = _mul(N, _bond_dim(b, hdim, vdim))
        lk = Link(i, side, K, N, _mul(_mul(K, N), 2))
        if i < nh - 1:
            lk.rescale = slot
            slot += 1
        chain.append(lk)
        v = list(down_part)
    return _finish(rows, cols, hdim, vdim, requested, ROWS, transpose, (0, 0),
                   units, steps, None, slot, chain)


def plan_grid(rows: int, cols: int, D: int = 2, hdim=None, vdim=None,
              order: int = COLSWEEP, quad_h: int = 0, quad_w: int = 0,
              budget: int = 0) -> Plan:
    """Build a plan; raises PlanOverflow if any integer exceeds int64 and
    PlanTooLarge if the plan (or, for HEURISTIC and SWEEP_AUTO, every
    candidate) keeps more than ``budget`` entries of intermediate storage
    (``budget`` <= 0: no limit).  ROWS_T is the row scheme over columns."""
    if rows < 1 or cols < 1:
        raise ValueError("rows and cols must be >= 1")
    if hdim is None:
        hdim = np.full((rows, max(cols - 1, 0)), D, dtype=np.int64)
    if vdim is None:
        vdim = np.full((max(rows - 1, 0), cols), D, dtype=np.int64)
    hdim = np.asarray(hdim, dtype=np.int64).reshape(rows, max(cols - 1, 0))
    vdim = np.asarray(vdim, dtype=np.int64).reshape(max(rows - 1, 0), cols)

    def fits(p):
        return budget <= 0 or p.buffers <= budget

    def checked(p):
        if not fits(p):
            raise PlanTooLarge()
        return p

    if order == COLSWEEP:
        return checked(plan_colsweep(rows, cols, hdim, vdim, 0))
    if order == QUADRANT:
        return checked(plan_quadrant(rows, cols, hdim, vdim, quad_h, quad_w))
    if order in (ROWS, ROWS_T):
        return checked(plan_rows(rows, cols, hdim, vdim, 1 if order == ROWS_T else 0, order))
    if order not in (SWEEP_AUTO, HEURISTIC):
        raise ValueError("unknown order")
    # candidates in enumeration order: sweep, transposed sweep, then (HEURISTIC
    # only) every quadrant split (h, w) lexicographically, the row scheme and
    # the transposed row scheme
    makers = [lambda t=t: plan_colsweep(rows, cols, hdim, vdim, t, order) for t in (0, 1)]
    if order == HEURISTIC:
        if rows >= 2 and cols >= 2:
            makers += [lambda h=h, w=w: plan_quadrant(rows, cols, hdim, vdim, h, w, HEURISTIC)
                       for h in range(1, rows) for w in range(1, cols)]
        makers += [lambda t=t: plan_rows(rows, cols, hdim, vdim, t, HEURISTIC) for t in (0, 1)]
    cands = []
    built = False
    for mk in makers:
        try:
            p = mk()
        except PlanOverflow:
            continue
        built = True
        if fits(p):
            cands.append(p)
    if not cands:
        if built:
            raise PlanTooLarge()
        raise PlanOverflow()
    # smallest bottleneck, then fewest flops, then enumeration order
    best = min(range(len(cands)), key=lambda k: (cands[k].peak, cands[k].flops, k))
    return cands[best]


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
    for k, lk in enumerate(p.chain):
        resc = str(lk.rescale) if lk.rescale >= 0 else "-"
        lines.append(f"link {k} unit={lk.unit} side={lk.side} K={lk.K} N={lk.N}"
                     f" flops={lk.flops} rescale={resc}")
    lines.append(f"totals steps={len(p.steps)} slots={p.slots} peak={p.peak}"
                 f" flops={p.flops} moved={p.moved}")
    return "\n".join(lines) + "\n"
