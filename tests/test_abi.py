"""The C ABI without a GPU: every symbol include/fftpim.h declares is
exported, host-side validation returns the documented status codes, and the
library's host evaluator of G^p (which builds the far-zone table) agrees with
the oracle's."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2312_02376_amd import fftpim as fp

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "fftpim.h")


def _declared():
    text = open(HDR).read()
    return sorted(set(re.findall(r"^(?:int|const char\*)\s+(fftpim_\w+)\s*\(", text, re.M)))


def test_header_and_binding_agree():
    assert _declared() == sorted(fp.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = fp.lib()
    for name in _declared():
        assert hasattr(L, name), name


def test_error_strings():
    L = fp.lib()
    for code in range(9):
        assert L.fftpim_error_string(code)


def _plan_status(problem_kw, **param_kw):
    L = fp.lib()
    pr = fp.make_problem(**problem_kw)
    pm = fp.Params()
    assert L.fftpim_default_params(ctypes.byref(pr), ctypes.byref(pm)) == 0
    for k, v in param_kw.items():
        if k in ("near_n", "far_n"):
            for c in range(3):
                getattr(pm, k)[c] = v[c]
        else:
            setattr(pm, k, v)
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(0x1000)   # never dereferenced: validation fails first
    obs = param_kw.pop("_obs", None)
    return L.fftpim_plan(ctypes.byref(h), ctypes.byref(pr), ctypes.byref(pm), 10, dummy, 0, obs, None)


CUBE = dict(periodic_dims=3, L=[1.0, 1.0, 1.0])


@pytest.mark.parametrize("kw,code", [
    (dict(near_order=0), 1), (dict(near_order=9), 1), (dict(far_order=10), 1),
    (dict(near_n=(12, 16, 16)), 1),          # 2n must be a power of two
    (dict(corr_radius=2), 1),                 # r_c >= q is required
    (dict(n_images=3), 1), (dict(precision=5), 1), (dict(nrhs_max=0), 1),
    (dict(self_mode=1), 8),
])
def test_parameter_validation(kw, code):
    assert _plan_status(CUBE, **kw) == code


def test_real_values_need_static_no_phase():
    k = 2 * math.pi
    assert _plan_status(dict(periodic_dims=2, L=[1, 1], k0=k, kt=[0.3 * k, 0.1 * k]), value_type=0) == 1


def test_unsupported_and_anomaly():
    assert _plan_status(dict(periodic_dims=1, L=[1.0], k0=3.0)) == 5      # 1D Helmholtz
    k = 2 * math.pi
    # k0 = 2 pi / L with no phase: the (+-1, 0) Floquet modes are grazing
    assert _plan_status(dict(periodic_dims=2, L=[1.0, 1.0], k0=k)) == 4


def test_null_arguments():
    L = fp.lib()
    assert L.fftpim_plan(None, None, None, 0, None, 0, None, None) == 1
    assert L.fftpim_apply(None, None, None, 1, None) == 1
    assert L.fftpim_destroy(None) == 0


@pytest.mark.parametrize("dims,k0,kt", [
    (3, 0.0, [0, 0, 0]), (2, 2 * math.pi, [0.6 * math.pi, 0.2 * math.pi, 0]), (2, 0.0, [0, 0, 0]),
    (1, 0.0, [0, 0, 0]), (3, 5.0, [0.3, 0.0, 0.2]), (3, 0.0, [0.5, 0.7, 0.3]),
])
def test_host_evaluator_matches_oracle(dims, k0, kt):
    from oracle import pgf as P
    rng = np.random.default_rng(dims)
    r = rng.uniform(-0.5, 0.5, (25, 3)) + rng.integers(-1, 2, (25, 3)) * (np.arange(3) < dims)
    r[:, 2] = np.where(np.abs(r[:, 2]) < 0.04, 0.04, r[:, 2])
    a = fp.eval_pgf(r, dims, [1, 1, 1], k0, kt)
    b = P.pgf(r, P.Lattice(dims, [1, 1, 1], k0, kt))
    np.testing.assert_allclose(a, b, rtol=1e-12)


@pytest.mark.parametrize("x", [1e-3, 0.1, 0.7, 1.9, 2.0, 2.1, 5.0, 17.0, 40.0])
def test_host_bessel_k0_through_1d_series(x):
    # lgf_1 at x-offset 0 probes sum_m K0(2 pi m rho): compare with SciPy's K0
    from scipy.special import k0
    rho = x / (2 * math.pi)
    got = fp.eval_pgf(np.array([[0.0, rho, 0.0]]), 1, [1.0, 1, 1])[0].real
    m = np.arange(1, int(60.0 / x) + 2)
    want = -math.log(rho) / (2 * math.pi) + np.sum(k0(m * x)[::-1]) / math.pi
    assert got == pytest.approx(want, rel=1e-13, abs=1e-15)
