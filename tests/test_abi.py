"""The C-ABI library loads and exports every symbol that include/hcov.h
declares (CPU only: no compute call needs a GPU here)."""
import os
import re

import pytest

from paper_1709_08625_amd import hcov

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            names |= set(re.findall(r"\b(hcov_\w+)\s*\(", txt))
    return sorted(names)


def test_library_built():
    assert os.path.exists(hcov.LIB_PATH), "run __graft_entry__.build() first"


def test_every_declared_symbol_is_exported():
    L = hcov.lib()
    names = declared()
    assert "hcov_build" in names and "hcov_loglik" in names
    missing = [s for s in names if not hasattr(L, s)]
    assert not missing, missing


def test_strerror_and_defaults_without_gpu():
    L = hcov.lib()
    assert L.hcov_strerror(0) == b"ok"
    assert L.hcov_strerror(-2) == b"matrix not positive definite"
    o = hcov.default_opts()
    assert o.max_rank == 64 and o.precision == hcov.FP64 and abs(o.aca_eps_factor - 0.1) < 1e-15


def test_argument_validation_on_host():
    # invalid arguments are rejected before any device call
    import numpy as np

    locs = np.random.default_rng(0).random((50, 2))
    bad = [((1.0, 0.1, 0.5, 1e-4), 0.0, 32, 2.0),      # eps
           ((1.0, 0.1, 0.5, 1e-4), 1e-8, 1, 2.0),      # leaf
           ((1.0, 0.1, 0.5, 1e-4), 1e-8, 32, 0.0),     # eta
           ((-1.0, 0.1, 0.5, 1e-4), 1e-8, 32, 2.0),    # sigma2
           ((1.0, 0.0, 0.5, 1e-4), 1e-8, 32, 2.0),     # ell
           ((1.0, 0.1, 0.0, 1e-4), 1e-8, 32, 2.0),     # nu
           ((1.0, 0.1, 0.5, -1.0), 1e-8, 32, 2.0)]     # nugget
    for th, eps, leaf, eta in bad:
        with pytest.raises(hcov.HcovError) as e:
            hcov.HCov(locs, th, eps=eps, leaf=leaf, eta=eta)
        assert e.value.code == hcov.EINVAL
    locs2 = locs.copy()
    locs2[3, 1] = float("nan")
    with pytest.raises(hcov.HcovError) as e:
        hcov.HCov(locs2, (1.0, 0.1, 0.5, 1e-4))
    assert e.value.code == hcov.EINVAL


def test_server_argument_validation_on_host():
    import ctypes as C

    L = hcov.lib()
    h = C.c_void_p()
    assert L.hcov_server_create(0, 0, None, C.byref(h)) == hcov.EINVAL
    assert L.hcov_server_create(65, 0, None, C.byref(h)) == hcov.EINVAL
    assert L.hcov_server_create(2, 0, None, None) == hcov.EINVAL
    t = C.c_uint64()
    assert L.hcov_server_submit(None, None, C.byref(t)) == hcov.EINVAL
    r = hcov.Result()
    assert L.hcov_server_poll(None, 1, C.byref(r)) == hcov.EINVAL
    assert L.hcov_server_wait(None, 1, C.byref(r)) == hcov.EINVAL
    assert L.hcov_strerror(hcov.EAGAIN) == b"not completed yet"


def test_sketch_options_validated_on_host():
    # the oversampling and saturation policy are checked before any device call
    import numpy as np

    locs = np.random.default_rng(0).random((100, 2))
    o = hcov.default_opts()
    assert o.oversample == 10 and o.on_saturation == hcov.SAT_RETRY
    assert o.autotune == 0 and o.seed == 0 and o.initial_rank_cap == 0
    for bad in ({"oversample": 1}, {"oversample": 65}, {"on_saturation": 2}, {"autotune": 2},
                {"initial_rank_cap": -1}, {"initial_rank_cap": 65}, {"max_rank": 16, "initial_rank_cap": 17}):
        with pytest.raises(hcov.HcovError) as e:
            hcov.HCov(locs, (1.0, 0.1, 0.5, 1e-4), eps=1e-8, leaf=32, opts=bad)
        assert e.value.code == hcov.EINVAL
