"""CPU oracle for the MPS Vlasov-Poisson time step (Ye & Loureiro, arXiv:2205.11990).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute anything in this package: only the tests, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP library and imports nothing from it; inputs come from the separate
``workloads`` module.

Two plain, slow, FP64 implementations:

* ``oracle.dense`` -- the finite-difference scheme on the full Nx x Nv grid
  (no MPS at all): the plain definition the untruncated MPS step must equal.
* ``oracle.mps``   -- the MPS/MPO algorithm in the paper's order (vector->MPS
  by iterated SVD, MPO x MPS, direct-sum addition, QR left sweep followed by a
  truncated-SVD right-to-left sweep, RK4 with compression levels), written
  with NumPy/LAPACK primitives and no blocking, fusion or reordering.

Every function cites the passage of the paper it follows.  Pins (tests that
tie the oracle to facts other than itself) live in ``tests/test_oracle_*.py``.
Functions without such a pin are marked "parity unpinned" in their docstring.
"""
