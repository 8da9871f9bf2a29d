"""Transformations of a network with a known effect on its value.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The method is exact (abstract and §4: the order of pairwise contractions
changes cost, never the result), so every identity below must hold for any
order up to rounding.

* gauge: insert G and G^-1 on one bond -> Z unchanged.
* rotate90 / reflect: relabel the lattice -> Z unchanged.
* pad: zero-pad every bond D -> D' -> Z unchanged.
* replica: leg-wise Kronecker product of two networks -> Z * Z'.
* scale_site: multiply one site by 2^k -> Z * 2^k exactly.
* add_site: replace one site T_s by T_s + T_s' -> Z + Z' (multilinearity).
"""
from __future__ import annotations

from typing import List, Sequence, Tuple

import numpy as np

from .network import site_bonds


def gauge(sites, rows, cols, bond, G):
    """Multiply the leg of ``bond`` on its first site by G and on its second
    site by G^-1 (as a matrix acting on that leg)."""
    kind, r, c = bond
    r2, c2 = (r, c + 1) if kind == "h" else (r + 1, c)
    out = [np.array(t, copy=True) for t in sites]
    Ginv = np.linalg.inv(G)
    for (rr, cc, M) in ((r, c, G), (r2, c2, Ginv.T)):
        k = rr * cols + cc
        ax = site_bonds(rows, cols, rr, cc).index(bond)
        t = np.tensordot(out[k], M, axes=([ax], [0]))    # leg moves to the end
        out[k] = np.moveaxis(t, -1, ax)
    return out


def rotate90(sites, rows, cols):
    """Rotate the lattice clockwise: new grid is cols x rows; new site
    (r', c') = old (rows-1-c', r'); old legs (left, up, right, down) become
    (up, right, down, left)."""
    nr, nc = cols, rows
    out = []
    for r2 in range(nr):
        for c2 in range(nc):
            r, c = rows - 1 - c2, r2
            t = sites[r * cols + c]
            old = site_bonds(rows, cols, r, c)
            # canonical leg name of each old axis
            names = []
            for b in old:
                kind, br, bc = b
                if kind == "h":
                    names.append("left" if (br, bc) == (r, c - 1) else "right")
                else:
                    names.append("up" if (br, bc) == (r - 1, c) else "down")
            newname = {"left": "up", "up": "right", "right": "down", "down": "left"}
            order = ["left", "up", "right", "down"]
            mapped = [newname[n] for n in names]
            perm = sorted(range(len(mapped)), key=lambda a: order.index(mapped[a]))
            out.append(np.ascontiguousarray(t.transpose(perm)) if t.ndim else t)
    return out, nr, nc


def reflect(sites, rows, cols):
    """Mirror left-right: new site (r, c') = old (r, cols-1-c'); left <-> right."""
    out = []
    for r in range(rows):
        for c2 in range(cols):
            c = cols - 1 - c2
            t = sites[r * cols + c]
            old = site_bonds(rows, cols, r, c)
            names = []
            for b in old:
                kind, br, bc = b
                if kind == "h":
                    names.append("left" if (br, bc) == (r, c - 1) else "right")
                else:
                    names.append("up" if (br, bc) == (r - 1, c) else "down")
            newname = {"left": "right", "right": "left", "up": "up", "down": "down"}
            order = ["left", "up", "right", "down"]
            mapped = [newname[n] for n in names]
            perm = sorted(range(len(mapped)), key=lambda a: order.index(mapped[a]))
            out.append(np.ascontiguousarray(t.transpose(perm)) if t.ndim else t)
    return out


def pad(sites, new_dim: int):
    out = []
    for t in sites:
        p = np.zeros((new_dim,) * t.ndim)
        p[tuple(slice(0, n) for n in t.shape)] = t
        out.append(p)
    return out


def replica(a, b):
    out = []
    for ta, tb in zip(a, b):
        n = ta.ndim
        t = np.multiply.outer(ta, tb)
        t = t.transpose([x for k in range(n) for x in (k, n + k)])
        out.append(t.reshape(tuple(ta.shape[k] * tb.shape[k] for k in range(n))))
    return out


def scale_site(sites, k: int, power: int):
    out = [np.array(t, copy=True) for t in sites]
    out[k] = np.ldexp(out[k], power)
    return out


def add_site(sites, k: int, extra: np.ndarray):
    out = [np.array(t, copy=True) for t in sites]
    out[k] = out[k] + extra
    return out
