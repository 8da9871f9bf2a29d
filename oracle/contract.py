"""Pairwise contraction of the planar network following a plan, in FP64.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper contracts tensors pairwise and sequentially (§4) and performs each
pairwise contraction by folding both tensors into matrices and calling a
double-precision matrix product (§6, first paragraph).  Here each step folds
the boundary into (pre, K, post) and the site into (K, N) and contracts with
``numpy.tensordot`` -- a library matrix product, nothing blocked or fused.

Rescaling (the paper normalises the state after each operator set, §5; it
does not rescale inside a contraction): after every step that carries a
rescale slot, e = frexp(max |B|)[1] and B *= 2^-e, E += e.  Powers of two are
exact, so the mantissa of the result is unchanged.  The result is returned
as Z = mantissa * 2^exp2, |mantissa| in [0.5, 1), together with sign and
log|Z| = exp2 * ln 2 + ln|mantissa|.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Sequence

import numpy as np

from . import plan as P


@dataclass
class Result:
    sign: int
    log_abs: float
    mantissa: float
    exp2: int

    @property
    def value(self) -> float:
        if self.sign == 0:
            return 0.0
        try:
            return self.sign * math.ldexp(abs(self.mantissa), self.exp2)
        except OverflowError:
            return self.sign * math.inf


def _result(m: float, E: int) -> Result:
    if m == 0.0:
        return Result(0, -math.inf, 0.0, 0)
    f, e = math.frexp(m)
    return Result(1 if m > 0 else -1, (E + e) * math.log(2.0) + math.log(abs(f)),
                  f, E + e)


def _rescale(B: np.ndarray):
    mx = float(np.max(np.abs(B))) if B.size else 0.0
    if not math.isfinite(mx):
        raise FloatingPointError("non-finite boundary")
    if mx == 0.0:
        return B, 0
    e = math.frexp(mx)[1]
    return np.ldexp(B, -e), e


def staged(site: np.ndarray, step: P.Step) -> np.ndarray:
    """Fold a canonical site tensor into the step's (K, N) matrix."""
    t = np.asarray(site, dtype=np.float64)
    if t.ndim:
        t = t.transpose(step.perm)
    return t.reshape(step.K, step.N)


def run_unit(sites: Sequence[np.ndarray], plan: P.Plan, unit: int):
    """Sweep one unit; returns (tensor, exponent sum)."""
    B = None
    E = 0
    for s in plan.steps:
        if s.unit != unit:
            continue
        S = staged(sites[s.site[0] * plan.cols + s.site[1]], s)
        if s.kind == "INIT":
            B = S.reshape(-1).copy()
        else:
            X = B.reshape(s.pre, s.K, s.post)
            Y = np.tensordot(X, S, axes=([1], [0]))      # (pre, post, N)
            B = np.ascontiguousarray(Y.transpose(0, 2, 1)).reshape(-1)
        if s.rescale >= 0:
            B, e = _rescale(B)
            E += e
    return B, E


def contract(sites: Sequence[np.ndarray], plan: P.Plan) -> Result:
    """Contract the network to its scalar along ``plan``."""
    if plan.order == P.COLSWEEP:
        B, E = run_unit(sites, plan, 0)
        return _result(float(B.reshape(-1)[0]), E)
    if plan.order == P.ROWS:
        # §4, row scheme: each row to one tensor, then the chain of row
        # tensors contracted from the first row on, one matrix-vector product
        # per row, rescaled exactly after each link but the last
        T = [run_unit(sites, plan, u) for u in range(len(plan.units))]
        v, E = T[0]
        for lk in plan.chain:
            R, e = T[lk.unit]
            E += e
            if lk.side == 0:
                v = v.reshape(lk.K) @ R.reshape(lk.K, lk.N)
            else:
                v = R.reshape(lk.N, lk.K) @ v.reshape(lk.K)
            if lk.rescale >= 0:
                v, e = _rescale(v)
                E += e
        return _result(float(np.asarray(v).reshape(-1)[0]), E)
    g = plan.ring
    T = [run_unit(sites, plan, u) for u in range(4)]
    E = sum(t[1] for t in T)
    TL = T[g.xa][0].reshape(g.kx, g.m)
    TR = T[g.xb][0].reshape(g.kx, g.n)
    BL = T[g.ya][0].reshape(g.ky, g.m)
    BR = T[g.yb][0].reshape(g.ky, g.n)
    X = TL.T @ TR            # sum over the top horizontal cut bonds
    Yt = BL.T @ BR           # sum over the bottom horizontal cut bonds
    z = float(np.sum(X * Yt))  # the vertical cut bonds close the ring
    return _result(z, E)


def contract_grid(sites, rows, cols, order=P.COLSWEEP, quad_h=0, quad_w=0) -> Result:
    """Plan from the site shapes, then contract."""
    from .network import dims_of
    d = dims_of(sites, rows, cols)
    hdim = [[d[("h", r, c)] for c in range(cols - 1)] for r in range(rows)]
    vdim = [[d[("v", r, c)] for c in range(cols)] for r in range(rows - 1)]
    p = P.plan_grid(rows, cols, hdim=hdim, vdim=vdim, order=order,
                    quad_h=quad_h, quad_w=quad_w)
    return contract(sites, p)

