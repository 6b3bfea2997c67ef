"""FP64 CPU oracle of the Parareal exponential-integrator Q1 FEM (PEIFE-linear).

TEST INFRASTRUCTURE ONLY.  This package is a plain, slow, obviously correct
reference implementation written from the paper.  Only the test suite, the
smoke check and the CPU-baseline leg of the benchmark may import it; the HIP
library never does, and this package never imports the HIP library.

Layout (each module cites the passage it follows):
    fem.py       1D Q1 mass/stiffness assembly and their dense LAPACK
                 diagonalisation (Section 2.1, eqs. (2.2)-(2.5))
    forcing.py   evaluation of the separable descriptors and Galerkin load
                 vectors by element-by-element Gauss quadrature (eq. (2.6): the
                 term P_h f; eq. (2.2): u_h(t0) = P_h u0)
    phi.py       phi_j functions and the weights b_i of eq. (2.7), in mpmath at
                 50+ significant digits (proof of Theorem 3.1)
    eife.py      the EIFE-linear step (eq. (2.6)) in the M-orthonormal
                 eigenbasis, sequential solves and L2 / nodal errors
    parareal.py  Algorithm 1 (PEIFE-linear), literally, with every iterate kept
    mlp.py       FP64 forward/backward of the per-mode coarse-correction MLP

Everything is float64 (mpmath for the phi tables).  Dense matrices, dense
mode products, no fast transforms.
"""
