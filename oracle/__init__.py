"""CPU FP64 oracle for the shared-pole rational approximation of exp(-t M^-1 K) b.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package: only the test suite, the smoke
check and the benchmark's CPU-baseline leg use it.  It shares no code with
the HIP library (``paper_2506_11657_amd``); both take their inputs from the
seeded generators in ``tem_workloads``.

Modules
  yee      explicit assembly of K, M, f and the receiver rows on a Yee grid
           (the lumped-mass edge discretization of Sec. 2, eq. (ode));
  rkfit    the shared-pole rational family of Sec. 3.2, eq. (ratfam), fitted
           by RKFIT, plus the error measures eq. (error)/(uniform_error) and
           the degree arithmetic of Table 1;
  single   the single-time best approximation of type [m/m] of Sec. 3.1 and
           its evaluation eq. (rba) by direct solves of t_k K - xi_i M;
  direct   shifted solves by banded and sparse LU, the residue contraction
           eq. (rmj) as S R, receiver data, dense expm references, and the
           adjoint gradient of Sec. 4;
  mscg     a plain textbook multi-shift CG on the CSR matrices, used as the
           CPU baseline at sizes where a direct factorization does not fit.
"""
