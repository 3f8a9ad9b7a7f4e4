"""CPU FP64 oracle for the alternating-direction isogeometric wave solver.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  The product
path (the HIP library and its Python binding) never imports, calls or links
anything here, and this package imports nothing from the product path.

The oracle is a plain, slow, obviously correct NumPy implementation written
from the paper (Los, Behnoudfar, Paszynski, Calo, "Fast isogeometric solvers
for hyperbolic wave propagation problems", arXiv:1911.08158):

* ``bspline``    tensor-product B-spline basis (Section 2, discretization).
* ``quadrature`` Gauss-Legendre rule per element (integrals of Section 2).
* ``matrices``   dense 1D mass / stiffness / mixed matrices (Section 2, the
                 1D matrices M_x, K_x; Section 5, the mixed matrices B_x).
* ``banded``     banded LU without pivoting and line-by-line substitution
                 (Appendix: three 1D banded solves with many right-hand sides).
* ``kron``       Kronecker applies and the x-y-z direction-split solve
                 (Appendix; eq. pwave2).
* ``pwave``      Newmark (beta = 1/4) P-wave step with the split left-hand
                 side (Section 2, eq. scheme / eq. pwave2; standard Newmark
                 reading, see the module header).
* ``elastic``    alternating-triangular elasticity step (Section 5,
                 eq. decom, eq. pre, eq. corr, eq. spill, eq. gen).
* ``pwave2d``, ``elastic2d``  the same two problems in two dimensions, the
                 dimension of the paper's exposition (Sections 2 and 5).
* ``quadref``    element-by-element quadrature of the bilinear forms, used
                 only to pin the Kronecker routes.

Every function is FP64 and unblocked.  Parity pinning of each part is done by
``tests/test_oracle_*.py`` against closed forms, invariants, library routines
and brute force.
"""
