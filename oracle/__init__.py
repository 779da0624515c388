"""CPU FP64 oracle for the QTT Fokker-Planck time step -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run anything in this package.  The HIP product
path never calls it, and it never calls the product path.  The only code the
two share is the seeded input package ``workloads``.

Two independent programs written from the paper (Gourianov, Givi, Jaksch,
Pope, "Tensor networks enable the calculation of turbulence probability
distributions"):

* ``oracle.dense``  -- the plain full-grid finite-difference solver of eq. FP2
  with the composition-space ghost rules of eq. compBCs, explicit RK4 / RK2.
* ``oracle.tt`` + ``oracle.stepper`` -- the same scheme with every vector
  stored as a quantics MPS and every matrix as an MPO ("Matrix product state
  algorithm"), with bond truncation by singular value decompositions.

Pins (``tests/test_oracle_*.py``) tie both to facts the paper and the
mathematics fix; see the headers of the modules for what is pinned and what
is not.
"""
