"""FP64 CPU oracle for the HSMA hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product library never calls it,
and it shares no code with the GPU path: it has its own harmonic basis
(monomial null-space polynomials), its own surface quadrature and check
point generators, its own image construction, its own least-squares solve
(NumPy SVD) and its own plain C pair sums.

Contents
  hsma.py      plain HSMA3D / HSMA2D steps in the paper's order (Sec. 2.2)
  ewald.py     independent Ewald3D (tinfoil) and Ewald2D (slab) references
  basis.py     harmonic polynomial basis of degree 1..p (Eq. 5)
  geometry.py  image sets (Eqs. 3-4), check points, surface quadrature
  pairsum.c    direct fp64 charge and dipole sums (plain loops)

Parity status: every function is pinned by the not-gpu tests (closed forms,
brute force, invariants, the NaCl and square-lattice Madelung constants,
independent Ewald sums).  The 2D dielectric least-squares rows follow a
reading of the DtN condition (the paper defers its details to earlier work);
their end-to-end accuracy is pinned only against the Ewald2D image sum.
"""
