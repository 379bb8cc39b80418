"""RF-DDES oracle: a plain, slow, FP64 CPU implementation of the interface
filter and everything around it (Kalantzis, Xi, Saad, "Beyond AMLS: domain
decomposition with rational filtering", arXiv 1711.09487).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg import this package.  The GPU library never
calls, links or imports it, and it shares no code with the GPU library: the
only common module is ``workloads`` (seeded input generators, no arithmetic
of the method).

Every step uses dense LAPACK through numpy/scipy in FP64 and follows the
paper's definitions directly:

  quadrature()        Sec. 2.1, eqs. (2.1)-(2.3): poles/weights of the
                      rational filter on the circle over [alpha, beta]
  DD                  Sec. 2.3, eqs. (2.5)-(2.6): interior-first reordering
  schur()             Sec. 3.1, eq. (3.1) and the Schur complement below it
  filter_apply()      Sec. 3.1, eq. (3.5): 2 Re sum_l omega_l S(zeta_l)^{-1}
  filter_interface()  Sec. 3.2, Alg. 3.1 taken as a block Krylov process
  interior_basis()    Sec. 4.3 / Alg. 5.1 step 3: eigenvectors V_j
  interior_levels()   Sec. 5.1, eqs. (5.2)-(5.4): Sigma_j, Gamma_j
  rayleigh_ritz()     Alg. 5.1 steps 6-8
  inertia_count()     Sylvester's law of inertia (exact count in [alpha,beta])

Readings where the paper is silent or ambiguous are listed in the design
notes (transpose vs conjugate transpose, factor 2 in the filter, pole rule,
block Krylov steps, deflated resolvent levels, rank tolerances, residual norm).
"""
from .rfdd import *  # noqa: F401,F403
