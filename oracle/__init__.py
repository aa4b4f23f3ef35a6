"""CPU FP64 oracle for the HEOM-2DVS hot path.

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
restatement of the method of Hoshino & Tanimura, "HEOM-based numerical
framework for quantum simulation of two-dimensional vibrational spectra in
molecular liquids (HEOM-2DVS)" (arXiv:2601.20550).  Only the test-suite, the
smoke check and the CPU-baseline leg of the benchmark may import it.  The GPU
library shares no code with it: it is written independently from the paper,
in double precision, with dense matrices throughout (the system-bath operators
V_s are formed as full d x d Kronecker products and multiplied densely).

Modules
    bath       Drude-bath exponential terms (Matsubara and [K-1/K] Pade).
    model      single-mode eigenbasis, product-basis H_S', V_s, dipoles.
    hierarchy  ADO index set and neighbour maps.
    heom       right-hand side, classic RK4, equilibration, dipole
               application, response functions and 2D spectra.
    gradient   least-squares spectrum-fit objective; its derivatives by
               central differences (parameter level and operator level) and
               the adjoint of the spectrum map.

Parity status: every function is pinned by a test in tests/test_oracle_pins.py
or tests/test_oracle_gradient.py against closed forms, exact invariants or
brute force, except the seeded
water-like spectra themselves, which the paper does not print (parity
unpinned beyond the oracle for those end-to-end values).
"""

from . import bath, hierarchy, model, heom, gradient  # noqa: F401
