"""CPU float64 oracle for the kernel-independent FMM boundary-integral path.

TEST INFRASTRUCTURE ONLY. Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import anything from this package. The GPU library never
imports, links or calls it, and this package imports nothing from the GPU
library; the two share only the seeded input generators in `workloads`.

Contents (each function cites the passage of the paper it follows):
  direct       the plain O(N^2) quadrature sum (Sec. II.A Eq. sum_fmm) for the
               single-layer, double-layer and field kernels, in C (float64)
               with a pure-numpy twin for tiny inputs
  tree         Morton keys, the octree and the U/V/W/X interaction lists,
               written from their plain definitions
  kifmm        the kernel-independent FMM, step by step in float64
  chebyshev    the paper's own far-field form: Chebyshev interpolation with
               the method-2 normal derivative at P2M (Sec. III.A.1 Eq. p2m)
  gmres        restarted GMRES(m) with modified Gram-Schmidt and Givens
               rotations (the solver the paper runs matrix-free, Sec. III)
  operators    the boundary operators of the two model problems
               (Eq. fk_integral_discrete and Eqs. Ax, pol_discret, rhs)
  closed_forms analytic results the paper quotes (demagnetising factor 1/3,
               cube stray-field energy 2*pi/3) and textbook ones (dielectric
               sphere in a uniform field, ellipsoid demagnetising factors)

Parity pins and unpinned parts are listed in each module's docstring.
"""
