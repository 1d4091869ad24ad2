"""CPU oracle for the complex finite-element Helmholtz solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package imports, links or
calls this package; only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the HIP path.

Everything here is plain NumPy/SciPy in float64 / complex128, written from
the paper's description of the acoustic problem (Sec. 3.2: the Helmholtz
equation obtained by Fourier-transforming the homogeneous wave equation,
discretised by finite elements) and its solver section (Sec. 4: a CSR
matrix, preconditioned Krylov methods in complex double precision, and a
Schwarz domain decomposition with Robin-type absorbing transmission
conditions).  Readings of what the paper leaves open are stated in the
docstrings of the functions that take them.

Modules
-------
fem        Q1 trilinear hexahedra: element and boundary-face matrices,
           assembly of K, M, per-wall boundary mass, patch mass (COO->CSR).
helmholtz  the operator A(k) = K - k^2 M + i k^2 M_eta + i k B_beta,
           the patch load (Neumann datum, or a Dirichlet condition on the
           source faces by symmetric elimination), the Galerkin
           least-squares mass coefficient, a matrix-free element-by-element
           apply.
parallel   a row-block threaded CSR product (timing on all host cores).
direct     banded LU with partial pivoting (own code) and a SuperLU wrapper.
krylov     right-Jacobi restarted GMRES(m) (MGS + complex Givens) and BiCGStab.
adjoint    receiver energy J and its adjoint gradient.
schwarz    non-overlapping Schwarz iteration with Robin transmission.
"""
