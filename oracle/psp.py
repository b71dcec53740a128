"""Periodic scalar potential, Eq. (1), as a direct FP64 pair sum on the CPU.

Test infrastructure: only the test suite, the smoke check and the benchmark's
CPU-baseline leg use this module.

  u(r_m) = sum_n G^p(r_m - r_n) q_n                      (Eq. (1))

Self term (reading of Eq. (1) against Eq. (5)): for coinciding sources and
observers the singular term (n = m, image i = 0) is dropped and the images of
the source itself are kept, i.e. the n = m coefficient is
lim_{r->0}[G^p(r) - G0(r)] ("images").  With self_mode="exclude" the whole
n = m term is dropped, as Eq. (5) writes it.

The conjugate transpose is w_n = sum_m conj(G^p(r_m - r_n)) v_m.

Rows are evaluated independently and spread over host processes.
"""
import os
from concurrent.futures import ProcessPoolExecutor
import multiprocessing as mp

import numpy as np

from . import pgf as _pgf


def host_workers():
    """Number of host cores this process may use (at most 16)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def _rows_job(args):
    lat, targets, pts, tgt_index, coincide, self_mode, sign, self_value = args
    out = np.empty((len(targets), pts.shape[0]), dtype=complex)
    for j, (t, ti) in enumerate(zip(targets, tgt_index)):
        d = sign * (t[None, :] - pts)
        if coincide:
            mask = np.ones(pts.shape[0], dtype=bool)
            mask[ti] = False
            row = np.empty(pts.shape[0], dtype=complex)
            row[mask] = _pgf.pgf(d[mask], lat)
            row[ti] = self_value if self_mode == "images" else 0.0
        else:
            row = _pgf.pgf(d, lat)
        out[j] = row
    return out


def _kernel_rows(lat, targets, pts, tgt_index, coincide, self_mode, sign, workers):
    """Rows G^p(sign * (target - p)) for every target over all points p."""
    self_value = _pgf.pgf_self(lat) if coincide else 0.0
    T = targets.shape[0]
    workers = host_workers() if workers is None else workers
    if workers <= 1 or T <= 1:
        return _rows_job((lat, targets, pts, tgt_index, coincide, self_mode, sign, self_value))
    chunks = np.array_split(np.arange(T), min(T, 4 * workers))
    jobs = [(lat, targets[c], pts, tgt_index[c], coincide, self_mode, sign, self_value)
            for c in chunks if c.size]
    # spawn: the workers start from a clean interpreter and never inherit a
    # GPU context from the parent
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_rows_job, jobs))
    return np.concatenate(parts, axis=0)


def psp_forward(lat, src, q, obs_index=None, obs=None, self_mode="images", workers=None):
    """Eq. (1) at selected observers.

    src: (N, 3) source positions; q: (nrhs, N) or (N,) amplitudes.
    Either obs_index (observers coincide with these sources) or obs (separate
    observer positions, shape (M, 3)) selects the observers.
    Returns u with shape (nrhs, M) (or (M,) for 1-D q).
    """
    src = np.asarray(src, dtype=float)
    q = np.asarray(q)
    squeeze = q.ndim == 1
    q2 = q.reshape(1, -1) if squeeze else q
    if obs is None:
        obs_index = np.arange(src.shape[0]) if obs_index is None else np.asarray(obs_index)
        targets = src[obs_index]
        rows = _kernel_rows(lat, targets, src, obs_index, True, self_mode, 1.0, workers)
    else:
        targets = np.asarray(obs, dtype=float)
        rows = _kernel_rows(lat, targets, src, np.zeros(len(targets), int), False, self_mode, 1.0, workers)
    u = q2 @ rows.T
    return u[0] if squeeze else u


def psp_adjoint(lat, src, v, src_index=None, obs=None, self_mode="images", workers=None):
    """Conjugate transpose of Eq. (1): w_n = sum_m conj(G^p(r_m - r_n)) v_m,
    at selected sources n (src_index).  Observers are the sources themselves
    unless obs gives separate positions; v has shape (nrhs, M) or (M,)."""
    src = np.asarray(src, dtype=float)
    v = np.asarray(v)
    squeeze = v.ndim == 1
    v2 = v.reshape(1, -1) if squeeze else v
    src_index = np.arange(src.shape[0]) if src_index is None else np.asarray(src_index)
    targets = src[src_index]
    if obs is None:
        rows = _kernel_rows(lat, targets, src, src_index, True, self_mode, -1.0, workers)
    else:
        rows = _kernel_rows(lat, targets, np.asarray(obs, float), src_index, False, self_mode, -1.0, workers)
    w = v2 @ np.conj(rows).T
    return w[0] if squeeze else w
