"""Plain FP64 CPU oracle for the fast Fourier spectral collision operator.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import it: only
the tests, the smoke check and the bench's CPU-baseline leg do.  It shares no
code with the HIP library; the two meet only through the seeded inputs of
the ``workloads`` module.

Contents, each written from the paper (Jaiswal, Alexeenko, Hu, "A
discontinuous Galerkin fast spectral method for the full Boltzmann equation
with general collision kernels"), Appendix and Sections 2-4:

* ``dft``        naive separable DFT (matrix form), the transform of the method
* ``quadrature`` velocity grid, signed frequencies, Gauss-Legendre radial rule
* ``kernel``     VHS kernel constant and the kernel modes F, gain and loss weights
* ``spectral``   the operator Q(f,f) in the quadrature form of the kernel modes
* ``direct``     the same discrete operator as an O(N^6) double sum (tiny N)
* ``brute``      brute-force quadrature of the collision integral (tiny N)
* ``conserve``   moments (midpoint rule) and the conservation projection
* ``adjoint``    vector-Jacobian products with respect to f and omega
* ``bkw``        the exact BKW collision operator (pin)
* ``dg``         DG triple-product tensor and the collision term of the weak form
"""
from . import dft, quadrature, kernel, spectral, direct, conserve, adjoint, bkw  # noqa: F401
