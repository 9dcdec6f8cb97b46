"""CPU FP64 oracle for the D2Q9 lattice-BGK lid-driven cavity.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) imports, calls or links anything in this package.  Only the
tests, the smoke check and the CPU-baseline leg of the benchmark use it.

It is a plain, slow, readable re-statement of the method of Xiang & Shi,
"Flow Simulation of Lid-Driven Rectangular Cavity by Using Lattice Boltzmann
Method" (arXiv 2211.05009):

* ``d2q9``     -- the lattice-BGK update (Sec. 2.1, Eqs. 1-3, 5), the wall
                  treatment, and test-only periodic / body-force switches.
* ``naive``    -- an independent pure-Python push-form twin of ``d2q9`` for
                  tiny lattices (brute force).
* ``monitors`` -- the convergence residual (Sec. 2.2 (iii), Eq. 6), mass,
                  bilinear observing-point probes (Sec. 3.3) and the stream
                  function used in Tables 1-2.
"""
