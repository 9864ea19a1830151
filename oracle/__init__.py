"""FP64 CPU oracle for the real-space Kohn-Sham hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
executes anything under ``oracle/``; only the tests, ``__graft_entry__.smoke``
and the CPU-baseline leg of ``bench.py`` use it.  The oracle shares no code
with the HIP path (no headers, tables, helpers or pre/post-processing); the
only common inputs come from the seeded generators in ``synthetic``.

Modules (each function cites the passage of Andrade & Aspuru-Guzik,
"Real-space density functional theory on graphical processing units",
that it follows):

  grid      - uniform grid restricted to a sphere/box, point ordering by small
              parallelepipedic sub-grids (Sec. 5.1, Fig. "locality")
  stencil   - high-order finite-difference kinetic operator (Sec. 5.1) and the
              local potential multiply (Sec. 5.2)
  kb        - Kleinman-Bylander non-local potential, eq. (6), its two parts
              and the atom colouring (Sec. 5.3)
  linalg    - overlap, Cholesky orthogonalisation, eqs. (7)-(8); subspace
              Hamiltonian, diagonalisation and rotation, eqs. (9)-(10)
  rmmdiis   - the RMM-DIIS eigensolver step with the filter preconditioner
              (Sec. 3) and the block-wise stopping rule (Sec. 9)
  cpu_hpsi  - a C/OpenMP FP64 H-psi used only to time the CPU baseline

Every function is pinned by tests under ``tests/`` that use the mathematics
(closed forms, invariants, library routines, brute force) rather than the
oracle itself.
"""
