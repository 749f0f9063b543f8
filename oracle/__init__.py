"""FP64 CPU oracle for the low-rank posterior-covariance method of Benner, Qiu
and Stoll (heat equation, space-time source parameter).

This package is TEST INFRASTRUCTURE.  Only the test suite, the smoke check of
the entry module and the CPU-baseline leg of the benchmark may import it.  The
product path (the HIP library and its Python binding) never imports, calls or
links anything here, and nothing here imports the product path.

Every routine is a plain, slow, direct transcription of a definition in the
paper (or of the reading stated in its docstring), in float64:

  fem            Q1 stiffness/mass matrices, two independent assemblies, and
                 the sine-transform eigenpairs of the 1D factors
  spacetime      implicit-Euler forward/adjoint maps, the misfit Hessian and
                 the prior-preconditioned operator (Sec. 2 eqs. postcov1 and
                 prior_pre, Sec. 3 eq. KKT2, Sec. 6.1 eqs. misfit and st_pde)
  posterior      eigenpairs (three independent routes), posterior covariance
                 and variance (Sec. 2, the Sherman-Morrison-Woodbury update),
                 prior variance, posterior samples
  lowrank        dense-SVD truncation and the low-rank Arnoldi process of
                 Sec. 4 Algorithm 1 with modified Gram-Schmidt
  closed_forms   spectra known in closed form (Sec. 5 and its space-time SVD
                 argument) used as pins
  mean           the posterior mean / MAP point (Sec. 2 eq. map1): normal
                 equations, data-space form, and the fully observed closed
                 form mode by mode
  initial        the paper's own experiment setting (Sec. 6, Sec. 6.2): the
                 initial condition as the parameter, nine sensors, prior
                 covariance c I; its Hessian, eigenpairs and posterior
                 variance, pinned by a closed form and an all-at-once route
  convdiff       the SUPG convection-diffusion operator of Sec. 6.3 (element
                 loop with Gauss quadrature, Peclet rule) and the
                 initial-condition problem on it, with transposed adjoint steps

Functions whose results have no independent pin say "parity unpinned" in
their docstring.
"""
