"""Plain FP64 CPU checker for the TT/QTT k-eigenvalue power iteration.

TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import, call or link anything here.
The device solver never routes through this package, and this package never
imports the device solver: the two share only the seeded input generator
(``paper_2309_03347_amd.workload``), which holds no arithmetic of the method.

Contents:

* ``sweep``   - exact discrete power iteration by transport sweeps (C, via
                ctypes): eq. Discretized_kNTE, eq. discreteBCs,
                eq. k_eff_fixed_points.
* ``dense``   - dense operators for tiny grids, assembled three independent
                ways (equation rows; the appendix Kronecker form; the paper's
                TT-form Kronecker sums per octant) and the brute-force
                generalized eigensolve.
* ``tt``      - dense reference semantics of tensor trains: reconstruction,
                TT-matrix x TT-vector, rounding with its error bound, the
                projected local system of the alternating solve, dot products.

Parity pins (what fixes each function independently of itself) are listed in
each module's docstring.
"""
