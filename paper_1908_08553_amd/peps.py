"""One observable evaluation of a real PEPS on the GPU (paper §3: the norm
and the local quantities m^x_k, m^z_k, c_ij; §5: each is a full contraction
of O|Psi> against <Psi|, L^2 + 2L(L-1) of them per evaluation, which is where
the paper's run time goes).

Every arithmetic step runs in the library: ``tn_double_layer`` builds the
single-layer sites (norm, S^x and S^z at every site) in one call, the
networks of the evaluation are contracted either by one captured batch
launch (``mode="batch"``: one workgroup per network, every network a full
sweep; suited to small lattices) or with cached column environments
(``mode="env"``: the norm network's left and right sweeps are kept, and each
observable network absorbs only the one or two columns holding its operator
sites and closes against the right environment), and ``tn_observables``
forms the ratios.  This module only allocates the buffers and lists which
site tensor each network uses.
"""
from __future__ import annotations

from ._native import (TN_ORDER_SWEEP_AUTO, Batch, EnvSet, tn_double_layer,
                      tn_double_layer_prepare, tn_observables, tn_plan_grid)


# Boundary entries above which mode "auto" uses cached environments (four
# streams): 6 x 6 at chi = 2 (4^7 entries) measures 0.65 ms per evaluation
# batched and 3.1 ms with environments, 8 x 8 (4^9) 10.0 ms and 6.6 ms,
# 10 x 10 (4^11) 459 ms and 25 ms.
AUTO_ENV_ENTRIES = 4 ** 8


def pairs(rows: int, cols: int):
    """Nearest-neighbour pairs in the order tn.h documents: horizontal pairs
    row by row, then vertical pairs row by row (site index r * cols + c)."""
    out = [(r * cols + c, r * cols + c + 1) for r in range(rows) for c in range(cols - 1)]
    out += [(r * cols + c, (r + 1) * cols + c) for r in range(rows - 1) for c in range(cols)]
    return out


class ObservableSet:
    """Networks of one evaluation of a rows x cols state with bond dimension
    ``chi`` and spin dimension ``d``: the norm, S^x and S^z at every site and
    S^z S^z on every pair, contracted as one batch in ``precision``."""

    def __init__(self, rows: int, cols: int, chi: int, d: int = 2, precision: str = "f64",
                 threads: int = 0, device: str = "cuda", mode: str = "auto"):
        import torch
        if mode not in ("auto", "batch", "env"):
            raise ValueError("mode must be 'auto', 'batch' or 'env'")
        if mode == "auto":
            # one workgroup per network while a column-sweep boundary along
            # the shorter side, (chi^2)^(min(rows, cols)+1), stays within a few
            # MB; cached environments, whose column absorptions spread over the
            # whole GPU, beyond
            short = min(rows, cols)
            mode = "env" if (chi * chi) ** (short + 1) > AUTO_ENV_ENTRIES else "batch"
        self.rows, self.cols, self.chi, self.d, self.mode = rows, cols, chi, d, mode
        # cached environments sweep left to right; a lattice taller than wide
        # is evaluated as its transpose (site (r, c) at (c, r), legs left <->
        # up and right <-> down), so the boundary runs along the shorter side
        self.transposed = mode == "env" and rows > cols
        self.n = rows * cols
        self.pairs = pairs(rows, cols)
        self.count = 1 + 2 * self.n + len(self.pairs)
        self.precision, self.device = precision, device
        self.E = [[None] * self.n for _ in range(3)]   # norm, S^x, S^z sites
        for r in range(rows):
            for c in range(cols):
                legs = (c > 0) + (r > 0) + (c < cols - 1) + (r < rows - 1)
                for k in range(3):
                    self.E[k][r * cols + c] = torch.empty((chi * chi,) * legs,
                                                          dtype=torch.float64, device=device)
        self.batch = self.env = None
        if mode == "batch":
            self.plan = tn_plan_grid(rows, cols, chi * chi, order=TN_ORDER_SWEEP_AUTO)
            self.batch = Batch([self.plan] * self.count, precision=precision, threads=threads,
                               device=device)
            self.table = self.batch.prepare(self.networks())   # the buffers never move
        else:
            t = self.site_index
            subst = ([[t(k)] for k in range(self.n)] * 2 +
                     [[t(i), t(j)] for i, j in self.pairs])
            er, ec = (cols, rows) if self.transposed else (rows, cols)
            self.env = EnvSet(er, ec, chi * chi, networks=subst, precision=precision,
                              device=device)
            norm, sx, sz = self.E
            base = [None] * self.n
            for k in range(self.n):
                base[t(k)] = norm[k]
            repl = sx + sz + [sz[x] for ij in self.pairs for x in ij]
            self.table = self.env.prepare(base, repl)

    def site_index(self, k: int) -> int:
        """Index of site k (row-major) in the lattice the networks run on."""
        if not self.transposed:
            return k
        r, c = divmod(k, self.cols)
        return c * self.rows + r

    def leg_perm(self, k: int):
        """For each bond leg of site k's double-layer tensor, the leg of the
        state tensor it comes from (identity unless transposed)."""
        r, c = divmod(k, self.cols)
        present = [c > 0, r > 0, c < self.cols - 1, r < self.rows - 1]
        axis = {leg: sum(present[:leg]) for leg in range(4) if present[leg]}
        order = (1, 0, 3, 2) if self.transposed else (0, 1, 2, 3)   # left, up, right, down
        return [axis[leg] for leg in order if present[leg]]

    def networks(self):
        """Site lists of every network, in the documented order."""
        norm, sx, sz = self.E
        out = [list(norm)]
        for k in range(self.n):
            out.append([sx[i] if i == k else norm[i] for i in range(self.n)])
        for k in range(self.n):
            out.append([sz[i] if i == k else norm[i] for i in range(self.n)])
        for i, j in self.pairs:
            out.append([sz[t] if t in (i, j) else norm[t] for t in range(self.n)])
        return out

    def run(self, peps, sx, sz, stream=None):
        """peps: rows*cols contiguous float64 device tensors [d][bonds...];
        sx, sz: [d][d] device operators.  Returns the batch results and the
        observables (mx, mz per site, czz per pair)."""
        key = tuple(A.data_ptr() for A in peps) + (sx.data_ptr(), sz.data_ptr())
        if key != getattr(self, "_dl_key", None):
            norm, ex, ez = self.E
            work = []
            for k, A in enumerate(peps):
                p = self.leg_perm(k)
                work += [(A, None, norm[k], p), (A, sx, ex[k], p), (A, sz, ez[k], p)]
            self._dl, self._dl_key = tn_double_layer_prepare(work), key
        tn_double_layer(None, stream, prepared=self._dl)
        if self.env is not None:
            results = self.env.run(stream=stream, prepared=self.table)
        else:
            results = self.batch.run(None, stream, prepared=self.table)
        mx, mz, czz = tn_observables(results, self.rows, self.cols)
        return {"results": results, "mx": mx, "mz": mz, "czz": czz}

    def tune(self, peps, sx, sz, reps: int = 5):
        """Pick the batch workgroup size with the autotuner on this state's
        networks (the candidates must agree bit for bit) and rebuild the
        batch with it; returns the autotuner's report."""
        from . import autotune
        if self.batch is None:
            raise ValueError("tune applies to the batch mode")
        self.run(peps, sx, sz)   # builds the double-layer sites the networks point to
        report = autotune.tune_batch([self.plan] * self.count, self.networks(), self.precision,
                                     reps=reps)
        self.batch.close()
        self.batch = Batch([self.plan] * self.count, precision=self.precision,
                           threads=report["best"], device=self.device, split=report["split"])
        self.table = self.batch.prepare(self.networks())
        return report

    def close(self):
        for h in (self.batch, self.env):
            if h is not None:
                h.close()

