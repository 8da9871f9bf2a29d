"""Plain, slow, FP64 CPU oracle for exact planar square-lattice contraction.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The
HIP library never links, imports or calls it, and this package imports
nothing from the HIP library: the two share no code.  Inputs come from the
separate ``lattice_inputs`` module, which holds no contraction arithmetic.

Modules (each function cites the passage of the paper it follows):

* ``network``      -- the plain definition Z = sum over bond indices of the
                       product of all site tensors (paper §4, the planar
                       network with no external indices), brute force over
                       bonds and over Ising spins, the textbook row transfer
                       matrix, and a library-einsum contraction.
* ``plan``         -- an independent re-implementation of the contraction
                       orders of §4 (column sweep = sequential row scheme,
                       quadrant scheme, the minimal-bottleneck heuristic)
                       with the int64 size/flop bookkeeping and the canonical
                       plan text.
* ``contract``     -- pairwise contraction that follows a plan step by step
                       (fold into matrices + matrix product, as the paper's
                       experiments do), with exact power-of-two rescaling.
* ``closed_forms`` -- product-state, all-ones and Ising special cases.
* ``invariants``   -- transformations with a known effect on Z.
* ``peps``         -- norm and expectation-value networks of a real PEPS
                       (paper §3 and §5): double-layer sites, the observable
                       set m^x, m^z, c_ij, and brute-force amplitudes.
* ``ite``          -- imaginary-time evolution of a PEPS (§5: Trotter-Suzuki
                       step, one-body gates, two-body gates split by SVD with
                       truncation, normalisation, energy) and exact
                       diagonalisation of the transverse-field Ising model
                       (§3), pinned in ``tests/test_ite_oracle.py``.

Parity status of every function is stated in its docstring.  Each is pinned
in ``tests/test_oracle_pins.py`` (and ``tests/test_peps_oracle.py`` for
``peps``) by brute force, a closed form, a textbook method or an invariant:
contraction values by brute force over bonds and spins, the row transfer
matrix and closed forms; every plan order, SWEEP_AUTO's orientation rule
included, by closed forms for its bottleneck, flops and first steps.
"""
