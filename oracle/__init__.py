"""Plain FP64 CPU oracle for deflated BiCGStab on Wilson / twisted-mass systems.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its Python binding)
may import, call or link anything in this package; only the test suite, the smoke check and the
benchmark's CPU-baseline leg do.  It shares no code, tables or constants with the HIP library:
both sides are fed the same seeded inputs from ``synth`` and compared element by element.

Modules:

* ``oracle.wilson``  -- lattice geometry, gamma matrices, the Wilson hopping term and the
  (twisted-mass) Wilson matrix A = I - kappa*H + i*mu*gamma5 (Sec. 1 and the action of Sec. 4).
* ``oracle.solvers`` -- BiCGStab, GMRES-DR(m,k) with harmonic-Ritz deflated restarting,
  D-BiCGStab(k) with left vectors gamma5*V (Sec. 2), and the minimal-residual projection over
  previous solutions for multiple shifts (Sec. 4).
* ``oracle.kappa``   -- kappa_c from the rightmost eigenvalue of the hopping term (Sec. 3).
* ``oracle.force``   -- gradient of Re(eta^H A^{-1} b) with respect to links and source.
* ``oracle.evenodd`` -- the even-odd reduced system of Sec. 3 and Sec. 4: the Schur complement
  Ahat = D - kappa^2 H_eo D^{-1} H_oe on the even sites, its source and the odd-site
  reconstruction.

Every function runs in complex128.  Pins (tests/test_oracle_*.py) check these functions against
closed forms, dense linear algebra and exact invariants, never against themselves.
Parity unpinned: the paper's matrix-vector-product counts (its gauge configurations are not
available), and the exact iteration counts of the iterative solvers (rounding-order dependent).
"""
