"""hcov: H-matrix Gaussian log-likelihood of Matérn fields on AMD MI355X.

The HIP library ``libhcov.so`` (C ABI in ``include/hcov.h``) does all the
work; ``paper_1709_08625_amd.hcov`` is its ctypes binding.
"""
from . import hcov  # noqa: F401
from .hcov import HCov, HcovError, Theta, default_opts, matern_eval  # noqa: F401
