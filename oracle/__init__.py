"""Plain FP64 CPU oracle for the batched shifted Laplace-Beltrami solves.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check of the entry
module and the CPU-baseline leg of the benchmark may import anything here.  The
product path (the HIP library and its Python binding) never imports, links or
executes this package, and this package imports nothing from the product.

Every function follows a passage of Harbrecht, Sonderegger and von Rickenbach,
"Simulation of Gaussian random fields on surfaces using the isogeometric
finite element method" (arXiv 2605.24882), cited by section and equation.
The code is deliberately slow and literal: NumPy / SciPy primitives (sparse
matrices, SuperLU, dense eigensolvers) serve as single steps; there is no
blocking, fusion or reordering beyond what the cited definitions state.

Modules
  sinc        scalar Balakrishnan / sinc quadrature rules (Sec. 3.4, eq. beta-approx)
  bspline     Cox-de Boor B-splines, Greville points, knot insertion (Sec. 2.1, 2.3)
  geometry    six-patch cube-sphere, perturbed sphere, NURBS patch maps (Sec. 2.2, 4.1)
  assembly    Gauss quadrature, DOF gluing, mass and stiffness matrices (Sec. 3.1, 3.2)
  fractional  split of beta, integer chain, node solves, quadrature sum (Sec. 3.4)
  noise       element-wise factorised white-noise load b ~ N(0, M) (Sec. 3.3)
  evaluate    point evaluation of a spline field on the surface
  gradient    d loss / d kappa by adjoint solves (one or two passes of the rule), finite
              differences, eigen-expansion
  sqrt_mass   the square root of the mass matrix applied to a vector (Sec. 3.3, eq. sqrt)
"""
