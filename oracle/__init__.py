"""Plain CPU FP64 oracle for the H-matrix Gaussian log-likelihood.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and its
Python binding) may import, call, link or execute anything in this package; only
``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` use it.  It shares no code with the GPU path.

Contents (each function cites the passage of Litvinenko et al., "HLIBCov",
arXiv:1709.08625, that it follows):

* ``oracle.matern``  -- Matérn covariance of Eq. (3) (Sec. 2.1) with K_nu from
  ``scipy.special.kv``; closed forms for half-integer nu; an independent
  arbitrary-precision K_nu (mpmath) used only as a pin.
* ``oracle.dense``   -- dense covariance assembly with nugget (Sec. 4 / 5.2),
  Cholesky (own unblocked and LAPACK), log-determinant, forward solve and the
  exact log-likelihood of Eq. (1); the exact-factor form of Eq. (2).
* ``oracle.brute``   -- arbitrary-precision brute-force log-likelihood for tiny n
  (determinant and solve by mpmath LU), used to pin ``oracle.dense``.
* ``oracle.trees``   -- reference cluster tree (recursive bisection into two
  equal-sized subsets, Sec. 2.2) and eta-admissible block cluster tree
  (standard admissibility, Appendix A); integer results the GPU must match bit
  for bit.
* ``oracle.markov``  -- exact O(n) log-likelihood of the nu=1/2 Matérn
  (exponential) field on points along a line (an AR(1) chain), used to pin the
  H path at sizes where no dense matrix fits.
* ``oracle.nelder_mead`` -- reference Nelder-Mead simplex minimiser
  (Sec. 5 / Appendix B driver), written from Nelder & Mead (1965).
"""
