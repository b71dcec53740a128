"""Separate observer sets (Sec. 2: observers r_m of Eq. (1) other than the
sources) through the C ABI: parity of every part and of the conjugate
transpose with the step-by-step oracle built with the same observers, the
accuracy against the exact sum of Eq. (1) at those observers, observers equal
to the sources against the coinciding plan, and the Bloch relation
G^p(r + R) = exp(-j k_t . R) G^p(r) on a translated and wrapped point set."""
import math

import numpy as np
import pytest

from oracle import pgf as P
from oracle import steps as S
from oracle.psp import host_workers, psp_forward
from paper_2312_02376_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
TWO_PI = 2 * math.pi


def _fp():
    from paper_2312_02376_amd import fftpim
    return fftpim


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


# name: lattice kwargs, point box (periodic axes span the cell), value type, near n, q, rc, far n, qf
CASES = {
    "npsp3_real": (dict(dims=3, L=[1, 1, 1]), (1, 1, 1), "real", (16, 16, 16), 4, 5, (10, 10, 10), 5),
    "helm2_bloch": (dict(dims=2, L=[1, 1], k0=TWO_PI, kt=[0.3 * TWO_PI, 0.1 * TWO_PI]), (1, 1, 0.4), "complex",
                    (16, 16, 8), 4, 4, (10, 10, 8), 5),
    "helm1_bloch": (dict(dims=1, L=[1.0], k0=0.8 * TWO_PI, kt=[1.1]), (1, 0.5, 0.3), "complex", (16, 8, 8), 4, 4,
                    (10, 8, 8), 5),
    "npsp1_real": (dict(dims=1, L=[1.0]), (1, 0.5, 0.3), "real", (16, 8, 8), 3, 3, (10, 8, 8), 4),
    "helm3_cphase": (dict(dims=3, L=[1, 1, 1], k0=3.0, kt=[0.3 - 0.2j, 0.1 + 0.1j, -0.2 - 0.1j]), (1, 1, 1),
                     "complex", (16, 16, 16), 4, 4, (10, 10, 10), 5),
    "phase3_static": (dict(dims=3, L=[1, 1.2, 0.9], k0=0.0, kt=[0.5, 0.3, 0.2]), (1, 1.2, 0.9), "complex",
                      (16, 16, 16), 3, 4, (9, 9, 9), 4),
}


def _setup(name, Ns=257, No=131, seed=5):
    latkw, box, vt, nn, q, rc, nf, qf = CASES[name]
    lat = P.Lattice(latkw["dims"], latkw["L"], latkw.get("k0", 0.0), latkw.get("kt", [0, 0, 0]))
    rng = np.random.default_rng(seed)
    src = rng.random((Ns, 3)) * np.asarray(box)
    obs = rng.random((No, 3)) * np.asarray(box)
    if vt == "real":
        qv = rng.standard_normal((1, Ns))
        qv -= qv.mean()
        vv = rng.standard_normal((1, No))
    else:
        qv = rng.standard_normal((1, Ns)) + 1j * rng.standard_normal((1, Ns))
        vv = rng.standard_normal((1, No)) + 1j * rng.standard_normal((1, No))
    plan = _fp().Plan(torch.tensor(src, device="cuda"), latkw["dims"], latkw["L"], k0=latkw.get("k0", 0.0),
                      kt=latkw.get("kt", [0, 0, 0]), near_n=nn, near_order=q, corr_radius=rc, far_n=nf, far_order=qf,
                      value_type=vt, observers=torch.tensor(obs, device="cuda"))
    ref = S.FFTPIM(lat, S.Params(nn, q, rc, nf, qf, 1), src, obs=obs)
    return lat, src, obs, qv, vv, plan, ref


def _dev(plan, x):
    return torch.tensor(np.ascontiguousarray(x), dtype=plan.dtype, device="cuda")


PARTS = {"near_grid": 1, "near_corr": 2, "far": 4}


@pytest.mark.parametrize("name", list(CASES))
def test_parts_and_adjoint_match_oracle(name):
    print("case", name, flush=True)
    lat, src, obs, qv, vv, plan, ref = _setup(name)
    info = plan.info()
    assert info["n_src"] == len(src) and info["n_obs"] == len(obs) and info["corr_layout_used"] == 1
    for adjoint, x in ((False, qv), (True, vv)):
        xd = _dev(plan, x)
        for part, bit in PARTS.items():
            got = plan.apply_parts(xd, bit, adjoint=adjoint).cpu().numpy()
            want = (ref.adjoint if adjoint else ref.apply)(x, parts=(part,))
            e = rel(got, want)
            print("  adjoint", adjoint, part, "rel %.2e" % e, flush=True)
            assert e < 1e-11, (name, adjoint, part, e)
    u = plan.apply(_dev(plan, qv)).cpu().numpy()
    assert plan.last_status() == 0
    assert rel(u, ref.apply(qv)) < 1e-11
    w = plan.adjoint(_dev(plan, vv)).cpu().numpy()
    want = ref.adjoint(vv)
    if lat.npsp:
        want = want - want.mean(axis=-1, keepdims=True)
    assert rel(w, want) < 1e-11
    # <A q, v> = <q, A^H v> on the two different point sets
    lhs = np.vdot(vv, u)
    rhs = np.vdot(w, qv) if not lat.npsp else np.vdot(w, qv)
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)
    plan.close()


@pytest.mark.parametrize("name", ["npsp3_real", "helm2_bloch"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_many_planes_near_grid(name, precision):
    # 16 or more planes: projection and interpolation run in their tiled
    # forms, each over its own point set (sources or observers)
    latkw, box, vt, nn, q, rc, nf, qf = CASES[name]
    lat = P.Lattice(latkw["dims"], latkw["L"], latkw.get("k0", 0.0), latkw.get("kt", [0, 0, 0]))
    rng = np.random.default_rng(15)
    src = rng.random((301, 3)) * np.asarray(box)
    obs = rng.random((173, 3)) * np.asarray(box)
    nrhs = 40 if vt == "real" else 21
    plan = _fp().Plan(torch.tensor(src, device="cuda"), latkw["dims"], latkw["L"], k0=latkw.get("k0", 0.0),
                      kt=latkw.get("kt", [0, 0, 0]), near_n=nn, near_order=q, corr_radius=rc, far_n=nf, far_order=qf,
                      value_type=vt, observers=torch.tensor(obs, device="cuda"), nrhs_max=nrhs, precision=precision)
    ref = S.FFTPIM(lat, S.Params(nn, q, rc, nf, qf, 1), src, obs=obs)
    tol = 1e-11 if precision == "f64" else 2e-5
    for adjoint, n in ((False, len(src)), (True, len(obs))):
        x = rng.standard_normal((nrhs, n))
        if vt == "complex":
            x = x + 1j * rng.standard_normal((nrhs, n))
        got = plan.apply_parts(_dev(plan, x), PARTS["near_grid"], adjoint=adjoint).cpu().numpy()
        want = (ref.adjoint if adjoint else ref.apply)(x, parts=("near_grid",))
        e = rel(got, want)
        print(name, precision, "adjoint", adjoint, "rel %.2e" % e, flush=True)
        assert e < tol, (name, precision, adjoint, e)
    plan.close()


def test_accuracy_at_separate_observers():
    # 2D-periodic Helmholtz with a phase shift: the library at separate
    # observers against the exact sum of Eq. (1)
    k = TWO_PI
    lat = P.Lattice(2, [1.0, 1.0], k, [0.3 * k, 0.1 * k])
    src = W.smooth_closed_surface(3000, 4)
    rng = np.random.default_rng(8)
    obs = np.c_[rng.random((200, 2)), 0.05 + 0.4 * rng.random(200)]
    q = rng.standard_normal(3000) + 1j * rng.standard_normal(3000)
    plan = _fp().Plan(torch.tensor(src, device="cuda"), 2, [1, 1], k0=k, kt=[0.3 * k, 0.1 * k], near_n=(32, 32, 16),
                      near_order=4, corr_ball=7.5, far_n=(20, 20, 12), far_order=7,
                      observers=torch.tensor(obs, device="cuda"), box=([0, 0, 0.0], [1, 1, 0.5]))
    u = plan.apply(torch.tensor(q, device="cuda")).cpu().numpy()
    exact = psp_forward(lat, src, q, obs=obs, workers=host_workers())
    e = rel(u, exact)
    print("separate observers vs exact: %.2e" % e)
    assert e < 1e-4
    plan.close()


@pytest.mark.parametrize("name", ["helm2_bloch", "npsp3_real", "helm1_bloch"])
def test_observers_equal_to_sources(name):
    # observers given as a copy of the sources: the coinciding plan's result
    # (the zero-distance pairs keep only their grid part, the reading of the
    # n = m term)
    latkw, box, vt, nn, q, rc, nf, qf = CASES[name]
    rng = np.random.default_rng(9)
    src = rng.random((300, 3)) * np.asarray(box)
    kw = dict(k0=latkw.get("k0", 0.0), kt=latkw.get("kt", [0, 0, 0]), near_n=nn, near_order=q, corr_radius=rc,
              far_n=nf, far_order=qf, value_type=vt)
    pos = torch.tensor(src, device="cuda")
    a = _fp().Plan(pos, latkw["dims"], latkw["L"], **kw)
    b = _fp().Plan(pos, latkw["dims"], latkw["L"], observers=pos.clone(), **kw)
    qv = rng.standard_normal(300) + (0 if vt == "real" else 1j * rng.standard_normal(300))
    if vt == "real":
        qv = qv - qv.mean()
    x = _dev(a, qv)
    assert rel(b.apply(x).cpu().numpy(), a.apply(x).cpu().numpy()) < 1e-12
    assert rel(b.adjoint(x).cpu().numpy(), a.adjoint(x).cpu().numpy()) < 1e-12
    a.close()
    b.close()


def test_bloch_relation_under_translation():
    # every source and observer moved by s along x and wrapped into the cell:
    # a wrapped source (moved by -L_x) carries exp(+j k_x0 L_x) on its
    # strength and a wrapped observer sees exp(+j k_x0 L_x) times the
    # unmoved potential, because G^p(r - R) = exp(j k_t . R) G^p(r); the
    # discrete method keeps this to its own accuracy
    k = TWO_PI
    kx0, ky0 = 0.3 * k, 0.1 * k
    kw = dict(k0=k, kt=[kx0, ky0], near_n=(32, 32, 16), near_order=4, corr_ball=7.5, far_n=(20, 20, 12),
              far_order=7, box=([0, 0, 0.0], [1, 1, 0.5]))
    rng = np.random.default_rng(12)
    src = np.c_[rng.random((2000, 2)), 0.05 + 0.4 * rng.random(2000)]
    obs = np.c_[rng.random((300, 2)), 0.05 + 0.4 * rng.random(300)]
    q = rng.standard_normal(2000) + 1j * rng.standard_normal(2000)
    fp = _fp()

    def run(s, o, qq):
        pl = fp.Plan(torch.tensor(s, device="cuda"), 2, [1, 1], observers=torch.tensor(o, device="cuda"), **kw)
        u = pl.apply(torch.tensor(qq, device="cuda")).cpu().numpy()
        pl.close()
        return u

    u0 = run(src, obs, q)
    shift = 0.37
    s2, o2, q2 = src.copy(), obs.copy(), q.copy()
    s2[:, 0] += shift
    o2[:, 0] += shift
    ws, wo = s2[:, 0] >= 1.0, o2[:, 0] >= 1.0
    s2[ws, 0] -= 1.0
    o2[wo, 0] -= 1.0
    q2[ws] *= np.exp(1j * kx0)
    u1 = run(s2, o2, q2)
    want = np.where(wo, np.exp(1j * kx0), 1.0) * u0
    e = rel(u1, want)
    print("Bloch relation under translation: %.2e" % e)
    exact = psp_forward(P.Lattice(2, [1.0, 1.0], k, [kx0, ky0]), src, q, obs=obs, workers=host_workers())
    e0 = rel(u0, exact)
    print("  method error %.2e" % e0)
    assert e < 1e-4 and e < 5 * max(e0, 1e-6)
