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
    for code in range(10):
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
    (dict(near_n=(5, 16, 16)), 1),           # at least near_order + 2 nodes
    (dict(near_n=(16, 2049, 16)), 1),        # at most 2048 nodes
    (dict(corr_radius=2), 1),                 # r_c >= q is required
    (dict(n_images=3), 1), (dict(precision=5), 1), (dict(nrhs_max=0), 1),
    (dict(self_mode=2), 1), (dict(far_sum=3), 1),
    (dict(far_sum=2, precision=2), 1),       # the BF16 far modes are direct sums
])
def test_parameter_validation(kw, code):
    assert _plan_status(CUBE, **kw) == code


def test_real_values_need_static_no_phase():
    k = 2 * math.pi
    assert _plan_status(dict(periodic_dims=2, L=[1, 1], k0=k, kt=[0.3 * k, 0.1 * k]), value_type=0) == 1


def test_unsupported_and_anomaly():
    # static with a phase that is a whole multiple of 2 pi / L on every axis:
    # every lateral Floquet wavenumber pair of Eq. (pgf_3) has a 0/0 term
    assert _plan_status(dict(periodic_dims=3, L=[1.0, 1.0, 1.0], kt=[2 * math.pi, 0.0, 0.0])) == 5
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


def test_wavenumber_validation():
    assert _plan_status(dict(periodic_dims=3, L=[1.0, 1.0, 1.0], k0=2.0 + 0.5j)) == 1   # Im k0 > 0
    assert _plan_status(dict(periodic_dims=3, L=[1.0, 1.0, 1.0], k0=-1.0)) == 1         # Re k0 < 0
    assert _plan_status(dict(periodic_dims=2, L=[1.0, 1.0], kt=[float("nan"), 0.0])) == 1


@pytest.mark.parametrize("dims,k0,kt", [
    (1, 2 * math.pi * 0.8, [0.3]),            # lossless 1D Helmholtz: propagating Hankel terms
    (1, 7.0, [1.1]),                          # two propagating orders, |k_rho rho| up to ~10
    (1, 3.0 - 0.5j, [0.7]),                   # lossy k0
    (1, 1.0, [1 - 1j]),                       # the coax case of the paper's potential figure
    (1, 0.0, [0.9]),                          # static with a phase (K0 of real argument)
    (1, 0.0, [0.9 - 0.4j]),                   # static with a complex phase
    (2, 2 * math.pi, [0.6 * math.pi + 0.2j, 0.2 * math.pi - 0.1j]),
    (2, 4.0 - 1.0j, [0.5, -0.3]),
    (3, 0.311, [0.01 - 0.01j] * 3),           # complex phase of the dynamic 3D timing runs, L = 1
    (3, 3.0 - 0.7j, [0.4, 0.0, -0.2]),
])
def test_host_evaluator_complex_wavenumbers(dims, k0, kt):
    from oracle import pgf as P
    rng = np.random.default_rng(40 + dims)
    r = rng.uniform(-0.5, 0.5, (30, 3)) + rng.integers(-1, 2, (30, 3)) * (np.arange(3) < dims)
    if dims == 1:
        # transverse distances from the far-grid scale up to several periods
        rho = np.exp(rng.uniform(np.log(0.02), np.log(3.0), 30))
        ang = rng.uniform(0, 2 * np.pi, 30)
        r[:, 1], r[:, 2] = rho * np.cos(ang), rho * np.sin(ang)
    else:
        r[:, 2] = np.where(np.abs(r[:, 2]) < 0.04, 0.04, r[:, 2])
    a = fp.eval_pgf(r, dims, [1, 1, 1], k0, kt)
    b = P.pgf(r, P.Lattice(dims, [1, 1, 1], k0, kt))
    np.testing.assert_allclose(a, b, rtol=1e-11, atol=1e-13 * np.abs(b).max())


@pytest.mark.parametrize("x", [1e-3, 0.1, 0.7, 1.9, 2.0, 2.1, 5.0, 17.0, 40.0])
def test_host_bessel_k0_through_1d_series(x):
    # lgf_1 at x-offset 0 probes sum_m K0(2 pi m rho): compare with SciPy's K0
    from scipy.special import k0
    rho = x / (2 * math.pi)
    got = fp.eval_pgf(np.array([[0.0, rho, 0.0]]), 1, [1.0, 1, 1])[0].real
    m = np.arange(1, int(60.0 / x) + 2)
    want = -math.log(rho) / (2 * math.pi) + np.sum(k0(m * x)[::-1]) / math.pi
    assert got == pytest.approx(want, rel=1e-13, abs=1e-15)


@pytest.mark.parametrize("dims,L,k0,kt", [
    (3, [1, 1.2, 0.9], 0.0, [0, 0, 0]), (2, [1, 1.3], 0.0, [0, 0]), (1, [1.3], 0.0, [0]),
    (3, [1, 1, 1], 5.0, [0, 0, 0]), (3, [1, 1.2, 0.9], 2.0 - 3.0j, [0.7, -1.1, 0.5]),
    (3, [1, 1, 1], 3.0, [0.3 - 0.2j, 0.1 + 0.1j, -0.2 - 0.1j]), (3, [1, 1.2, 0.9], 0.0, [0.5, 0.3, 0.2]),
    (2, [1, 1], 2 * math.pi, [0.6 * math.pi, 0.2 * math.pi]), (2, [1, 1.2], 2.5 - 3.0j, [0.9, -1.3]),
    (2, [1, 1], 2 * math.pi, [0.6 * math.pi + 0.2j, 0.2 * math.pi - 0.1j]),
    (1, [1.0], 0.8 * 2 * math.pi, [1.1]), (1, [1.0], 1.0, [1 - 1j]), (1, [1.0], 0.0, [0.9 - 0.4j]),
    (1, [1.0], 2.0 - 3.0j, [0.7]),
])
def test_self_evaluator_matches_oracle(dims, L, k0, kt):
    # the library's Ewald-at-zero self coefficient (splitting parameter
    # E L >= 6.8) against the oracle's (E ~ sqrt(pi)/L, different terms)
    from oracle import pgf as P
    got = fp.eval_pgf_self(dims, L, k0, kt)
    want = P.pgf_self(P.Lattice(dims, L, k0, kt))
    assert abs(got - want) <= 2e-12 * abs(want), (got, want)


def test_autotune_and_batch_argument_checks():
    # every check here fails before the library reads the (dummy) points
    L = fp.lib()
    pr = fp.make_problem(3, [1.0, 1.0, 1.0])
    pm = fp.Params()
    assert L.fftpim_default_params(ctypes.byref(pr), ctypes.byref(pm)) == 0
    rep = fp.TuneReport()
    dummy = ctypes.c_void_p(0x1000)
    tune = L.fftpim_autotune
    assert tune(None, 10, dummy, 1e-4, 0, 1, ctypes.byref(pm), ctypes.byref(rep)) == 1
    assert tune(ctypes.byref(pr), 0, dummy, 1e-4, 0, 1, ctypes.byref(pm), ctypes.byref(rep)) == 1
    assert tune(ctypes.byref(pr), 10, dummy, 0.0, 0, 1, ctypes.byref(pm), ctypes.byref(rep)) == 1
    assert tune(ctypes.byref(pr), 10, dummy, 1e-7, 1, 1, ctypes.byref(pm), ctypes.byref(rep)) == 1  # FP32 floor
    assert tune(ctypes.byref(pr), 10, dummy, 1e-4, 0, 0, ctypes.byref(pm), ctypes.byref(rep)) == 1
    h = ctypes.c_void_p()
    plans = (ctypes.c_void_p * 2)(None, None)
    assert L.fftpim_batch_create(ctypes.byref(h), plans, 2, 4, 0) == 1      # null plans
    assert L.fftpim_batch_create(ctypes.byref(h), plans, 0, 4, 0) == 1      # no cells
    assert L.fftpim_batch_create(ctypes.byref(h), plans, 2, 17, 0) == 1     # lanes 1..16
    assert L.fftpim_batch_apply(None, None, None, None, 0, None) == 1
    assert L.fftpim_batch_destroy(None) == 1


def test_separate_observer_argument_checks():
    # both fail before the library reads the (dummy) points
    L = fp.lib()
    pr = fp.make_problem(3, [1.0, 1.0, 1.0])
    pm = fp.Params()
    assert L.fftpim_default_params(ctypes.byref(pr), ctypes.byref(pm)) == 0
    h = ctypes.c_void_p()
    dummy = ctypes.c_void_p(0x1000)
    # an observer array needs n_obs >= 1
    assert L.fftpim_plan(ctypes.byref(h), ctypes.byref(pr), ctypes.byref(pm), 10, dummy, 0, dummy, None) == 1
    # the exclude-self mode has no meaning for separate observers
    pm.self_mode = 1
    assert L.fftpim_plan(ctypes.byref(h), ctypes.byref(pr), ctypes.byref(pm), 10, dummy, 5, dummy, None) == 1
    # without an observer array n_obs is 0 or n_src
    pm.self_mode = 0
    assert L.fftpim_plan(ctypes.byref(h), ctypes.byref(pr), ctypes.byref(pm), 10, dummy, 5, None, None) == 1
