"""GPU parity: the HIP library (through its C ABI) against the step-by-step
FP64 oracle of Sec. 3, stage by stage and whole, forward and conjugate
transpose, on small seeded problems that span several grid tiles, odd point
counts and every problem class the library takes."""
import numpy as np
import pytest

from oracle import pgf as P
from oracle import steps as S
from paper_2312_02376_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TWO_PI = 2 * np.pi


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b)))


def elem(a, b):
    """Largest element error in units of the reference's RMS value: one wrong
    row of a few hundred moves the relative L2 error by only 1/sqrt(N) of its
    own error, so the parity tests bound this as well."""
    b = np.asarray(b)
    return float(np.abs(np.asarray(a) - b).max() / np.sqrt(np.mean(np.abs(b) ** 2)))


def _fftpim():
    from paper_2312_02376_amd import fftpim
    return fftpim


# name: (lattice kwargs, points, nrhs, value type, near n, q, rc, far n, qf)
CASES = {
    "npsp3_real": (dict(dims=3, L=[1, 1, 1]), "cube", 3, "real", (16, 16, 16), 4, 5, (10, 10, 10), 5),
    "helm2_bloch": (dict(dims=2, L=[1, 1], k0=TWO_PI, kt=[0.3 * TWO_PI, 0.1 * TWO_PI]), "surface", 2, "complex",
                    (16, 16, 8), 4, 4, (10, 10, 8), 5),
    "phase3_static": (dict(dims=3, L=[1, 1.2, 0.9], k0=0.0, kt=[0.5, 0.3, 0.2]), "cube", 1, "complex",
                      (16, 16, 16), 3, 4, (9, 9, 9), 4),
    "helm3": (dict(dims=3, L=[1, 1, 1], k0=5.0, kt=[0.0, 0.0, 0.0]), "cube", 1, "complex", (16, 16, 16), 4, 4,
              (10, 10, 10), 5),
    "npsp2_real": (dict(dims=2, L=[1, 1.3]), "slab", 2, "real", (16, 16, 8), 4, 4, (10, 10, 8), 5),
    "npsp1_real": (dict(dims=1, L=[1.0]), "rod", 2, "real", (16, 8, 8), 2, 3, (10, 8, 8), 3),
    # complex wavenumbers and 1D Helmholtz (Sec. 2: possibly complex phase shifts)
    "helm1_bloch": (dict(dims=1, L=[1.0], k0=0.8 * TWO_PI, kt=[1.1]), "rod", 2, "complex", (16, 8, 8), 4, 4,
                    (10, 8, 8), 5),
    "coax_dyn": (dict(dims=1, L=[1.0], k0=1.0, kt=[1 - 1j]), "coax", 1, "complex", (16, 16, 16), 4, 4,
                 (9, 10, 10), 5),
    "helm3_cphase": (dict(dims=3, L=[1, 1, 1], k0=3.0, kt=[0.3 - 0.2j, 0.1 + 0.1j, -0.2 - 0.1j]), "cube", 1,
                     "complex", (16, 16, 16), 4, 4, (10, 10, 10), 5),
    "helm2_lossy": (dict(dims=2, L=[1, 1], k0=5.0 - 1.0j, kt=[0.4, -0.2]), "surface", 1, "complex",
                    (16, 16, 8), 4, 4, (10, 10, 8), 5),
    "phase1_cstatic": (dict(dims=1, L=[1.0], k0=0.0, kt=[0.9 - 0.4j]), "rod", 1, "complex", (16, 8, 8), 3, 3,
                       (10, 8, 8), 4),
    # near grids that are not powers of two (Sec. 4.2, Table near-zone:
    # 17^3 upwards); the transforms pad to the next power of two >= 2n - 1
    "npsp3_odd": (dict(dims=3, L=[1, 1, 1]), "cube", 3, "real", (17, 17, 17), 4, 5, (10, 10, 10), 5),
    "helm2_odd": (dict(dims=2, L=[1, 1], k0=TWO_PI, kt=[0.3 * TWO_PI, 0.1 * TWO_PI]), "surface", 2, "complex",
                  (20, 24, 11), 4, 4, (10, 10, 8), 5),
}


def _points(kind, N, seed):
    rng = np.random.default_rng(seed)
    if kind == "cube":
        return W.uniform_cube(N, seed, (1.0, 1.0, 1.0))
    if kind == "surface":
        return W.smooth_closed_surface(N, seed)
    if kind == "slab":
        p = rng.random((N, 3)) * np.array([1.0, 1.3, 0.4])
        return p
    if kind == "rod":
        p = rng.random((N, 3)) * np.array([1.0, 0.5, 0.3])
        return p
    if kind == "coax":
        return W.coax_shells_random(N, seed)
    raise ValueError(kind)


class _CachedRef:
    """The oracle of one case with its results kept: several tests compare
    different library paths (layouts, precisions, the fused pair) with the
    same oracle products, which are computed once per test session."""

    def __init__(self, ref):
        self._ref = ref
        self._memo = {}

    def __getattr__(self, k):
        return getattr(self._ref, k)

    def _call(self, kind, x, rows, parts):
        x = np.asarray(x)
        key = (kind, None if rows is None else np.asarray(rows).tobytes(), tuple(parts), x.shape, x.tobytes())
        if key not in self._memo:
            fn = self._ref.apply if kind == "apply" else self._ref.adjoint
            self._memo[key] = fn(x, rows=rows, parts=parts)
        return np.array(self._memo[key], copy=True)

    def apply(self, q, rows=None, parts=("near_grid", "near_corr", "far")):
        return self._call("apply", q, rows, parts)

    def adjoint(self, v, rows=None, parts=("near_grid", "near_corr", "far")):
        return self._call("adjoint", v, rows, parts)


_REFS = {}


def _oracle(name, N, seed, corr_ball, self_mode):
    key = (name, N, seed, corr_ball, self_mode)
    if key not in _REFS:
        latkw, kind, nrhs0, vt, nn, q, rc, nf, qf = CASES[name]
        lat = P.Lattice(latkw["dims"], latkw["L"], latkw.get("k0", 0.0), latkw.get("kt", [0, 0, 0]))
        src = _points(kind, N, seed)
        if kind == "cube":
            src = src * np.asarray((latkw["L"] + [1, 1, 1])[:3])
        _REFS[key] = (lat, src, _CachedRef(S.FFTPIM(lat, S.Params(nn, q, rc, nf, qf, 1, corr_ball=corr_ball), src,
                                                    self_mode=self_mode)))
    return _REFS[key]


def _setup(name, N=257, seed=31, precision="f64", nrhs=None, corr_layout="auto", self_mode="images",
           corr_ball=0.0, far_sum="auto"):
    latkw, kind, nrhs0, vt, nn, q, rc, nf, qf = CASES[name]
    nrhs = nrhs0 if nrhs is None else nrhs
    lat, src, ref = _oracle(name, N, seed, corr_ball, self_mode)
    rng = np.random.default_rng(seed + 1)
    if vt == "real":
        qv = rng.standard_normal((nrhs, N))
        qv -= qv.mean(axis=1, keepdims=True)
    else:
        qv = rng.standard_normal((nrhs, N)) + 1j * rng.standard_normal((nrhs, N))
    fp = _fftpim()
    pos = torch.tensor(src, dtype=torch.float64, device="cuda")
    plan = fp.Plan(pos, latkw["dims"], latkw["L"], k0=latkw.get("k0", 0.0), kt=latkw.get("kt", [0, 0, 0]),
                   near_n=nn, near_order=q, corr_radius=rc, far_n=nf, far_order=qf, n_images=1,
                   precision=precision, value_type=vt, nrhs_max=max(4, nrhs), corr_layout=corr_layout,
                   self_mode=self_mode, corr_ball=corr_ball, far_sum=far_sum)
    return lat, ref, plan, qv


def _to_dev(plan, x):
    return torch.tensor(np.ascontiguousarray(x), dtype=plan.dtype, device="cuda")


PARTS = {"near_grid": 1, "near_corr": 2, "far": 4}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("adjoint", [False, True])
def test_stage_parity_fp64(name, adjoint):
    print("case", name, "adjoint", adjoint, flush=True)
    lat, ref, plan, qv = _setup(name)
    qd = _to_dev(plan, qv)
    for part, bit in PARTS.items():
        got = plan.apply_parts(qd, bit, adjoint=adjoint).cpu().numpy()
        want = (ref.adjoint if adjoint else ref.apply)(qv, parts=(part,))
        err, em = rel(got, want), elem(got, want)
        print("  ", part, "rel %.2e max elem %.2e" % (err, em), flush=True)
        assert err < 1e-11 and em < 1e-10, (name, part, adjoint, err, em)
    got = plan.apply_parts(qd, 7, adjoint=adjoint).cpu().numpy()
    want = (ref.adjoint if adjoint else ref.apply)(qv)
    assert rel(got, want) < 1e-11 and elem(got, want) < 1e-10


@pytest.mark.parametrize("name", ["npsp3_real", "helm2_bloch", "helm1_bloch", "coax_dyn", "helm3_cphase"])
def test_full_apply_and_adjoint(name):
    lat, ref, plan, qv = _setup(name)
    qd = _to_dev(plan, qv)
    u = plan.apply(qd).cpu().numpy()
    assert plan.last_status() == 0
    assert rel(u, ref.apply(qv)) < 1e-11 and elem(u, ref.apply(qv)) < 1e-10
    w = plan.adjoint(qd).cpu().numpy()
    want = ref.adjoint(qv)
    if lat.npsp:
        # only the zero-mean part of A^H v is defined for the neutral static case
        want = want - want.mean(axis=-1, keepdims=True)
    assert rel(w, want) < 1e-11 and elem(w, want) < 1e-10


@pytest.mark.parametrize("name", ["npsp3_real", "helm2_bloch", "helm1_bloch", "coax_dyn", "helm3_cphase", "npsp1_real",
                                  "npsp2_real", "helm2_odd"])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_far_sum_by_fft(name, precision):
    # the far grid sum of Eq. (8) as a zero-padded FFT convolution: the far
    # part against the oracle's term-by-term sum, forward and adjoint, and
    # against the library's direct sum on the same plan parameters
    print("case", name, precision, flush=True)
    lat, ref, plan, qv = _setup(name, precision=precision, far_sum="fft")
    _, _, plan_d, _ = _setup(name, precision=precision, far_sum="direct")
    info = plan.info()
    nf = CASES[name][7]
    assert all(m >= 2 * n - 1 and (m & (m - 1)) == 0 for m, n in zip(info["far_fft"], nf)), info["far_fft"]
    assert plan_d.info()["far_fft"] == [0, 0, 0]
    qd = _to_dev(plan, qv)
    tol = 1e-11 if precision == "f64" else 2e-5
    for adjoint in (False, True):
        got = plan.apply_parts(qd, PARTS["far"], adjoint=adjoint).cpu().numpy()
        direct = plan_d.apply_parts(qd, PARTS["far"], adjoint=adjoint).cpu().numpy()
        want = (ref.adjoint if adjoint else ref.apply)(qv, parts=("far",))
        e, ed, em = rel(got, want), rel(got, direct), elem(got, want)
        print("  adjoint", adjoint, "vs oracle %.2e (max elem %.2e) vs direct %.2e" % (e, em, ed), flush=True)
        assert e < tol and ed < tol and em < 5 * tol
    plan.close()
    plan_d.close()


@pytest.mark.parametrize("name", ["npsp3_real", "helm2_bloch"])
def test_fp32_mode(name):
    lat, ref, plan, qv = _setup(name, precision="f32")
    qd = _to_dev(plan, qv)
    u = plan.apply_parts(qd, 7).cpu().numpy()
    assert rel(u, ref.apply(qv)) < 2e-5 and elem(u, ref.apply(qv)) < 1e-4
    w = plan.apply_parts(qd, 7, adjoint=True).cpu().numpy()
    assert rel(w, ref.adjoint(qv)) < 2e-5 and elem(w, ref.adjoint(qv)) < 1e-4


def test_adjoint_identity_on_device():
    lat, ref, plan, qv = _setup("helm2_bloch", N=301, seed=5)
    rng = np.random.default_rng(6)
    v = rng.standard_normal(qv.shape) + 1j * rng.standard_normal(qv.shape)
    Aq = plan.apply(_to_dev(plan, qv)).cpu().numpy()
    AHv = plan.adjoint(_to_dev(plan, v)).cpu().numpy()
    lhs = np.vdot(v, Aq)
    rhs = np.vdot(AHv, qv)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_plan_order_io_and_permutation():
    latkw, kind, nrhs, vt, nn, q, rc, nf, qf = CASES["npsp3_real"]
    fp = _fftpim()
    src = W.uniform_cube(300, 41)
    qv = W.gaussian_neutral(2, 300, 41)
    pos = torch.tensor(src, dtype=torch.float64, device="cuda")
    kw = dict(near_n=nn, near_order=q, corr_radius=rc, far_n=nf, far_order=qf, value_type="real", nrhs_max=2)
    pu = fp.Plan(pos, 3, [1, 1, 1], order="user", **kw)
    pp = fp.Plan(pos, 3, [1, 1, 1], order="plan", **kw)
    perm = pu.permutation().cpu().numpy().astype(np.int64)
    assert sorted(perm.tolist()) == list(range(300))
    uu = pu.apply(torch.tensor(qv, device="cuda")).cpu().numpy()
    up = pp.apply(torch.tensor(qv[:, perm].copy(), device="cuda")).cpu().numpy()
    np.testing.assert_allclose(up, uu[:, perm], rtol=0, atol=1e-13 * np.abs(uu).max())


def test_non_neutral_input_is_reported():
    fp = _fftpim()
    src = W.uniform_cube(200, 3)
    pos = torch.tensor(src, dtype=torch.float64, device="cuda")
    plan = fp.Plan(pos, 3, [1, 1, 1], near_n=(16, 16, 16), corr_radius=4, far_n=(10, 10, 10), far_order=5,
                   value_type="real")
    q = torch.ones(200, dtype=torch.float64, device="cuda")
    plan.apply(q)
    assert plan.last_status() == 3
    q2 = torch.tensor(W.plus_minus_charges(200, 3), device="cuda")
    plan.apply(q2)
    assert plan.last_status() == 0


def test_repeated_applies_bitwise_identical():
    lat, ref, plan, qv = _setup("helm2_bloch", N=333, seed=8)
    qd = _to_dev(plan, qv)
    a = plan.apply(qd).cpu().numpy()
    b = plan.apply(qd).cpu().numpy()
    assert np.array_equal(a, b)


def test_single_point_and_tiny_problems():
    fp = _fftpim()
    lat = P.Lattice(2, [1, 1], TWO_PI, [0.3 * TWO_PI, 0.1 * TWO_PI])
    src = np.array([[0.25, 0.5, 0.3]])
    ref = S.FFTPIM(lat, S.Params((16, 16, 8), 4, 4, (10, 10, 8), 5, 1), src)
    plan = fp.Plan(torch.tensor(src, device="cuda"), 2, [1, 1], k0=TWO_PI, kt=[0.3 * TWO_PI, 0.1 * TWO_PI],
                   near_n=(16, 16, 8), corr_radius=4, far_n=(10, 10, 8), far_order=5)
    q = np.array([1.0 + 0.5j])
    u = plan.apply(torch.tensor(q, device="cuda")).cpu().numpy()
    np.testing.assert_allclose(u, ref.apply(q), rtol=1e-11)


@pytest.mark.parametrize("name,nrhs", [("npsp3_real", 19), ("helm2_bloch", 9), ("helm2_bloch", 40)])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_many_right_hand_sides(name, nrhs, precision):
    # more than four planes: the correction runs as a lanes-over-planes SpMM
    lat, ref, plan, qv = _setup(name, N=211, seed=13, precision=precision, nrhs=nrhs)
    qd = _to_dev(plan, qv)
    tol = 1e-11 if precision == "f64" else 2e-5
    for adjoint in (False, True):
        for part, bit in PARTS.items():
            got = plan.apply_parts(qd, bit, adjoint=adjoint).cpu().numpy()
            want = (ref.adjoint if adjoint else ref.apply)(qv, parts=(part,))
            assert rel(got, want) < tol and elem(got, want) < 5 * tol, (part, adjoint, elem(got, want))


@pytest.mark.parametrize("name,nrhs", [("npsp3_odd", 37), ("helm2_odd", 21), ("npsp1_real", 33), ("helm1_bloch", 16),
                                       ("phase3_static", 23), ("npsp2_real", 64)])
@pytest.mark.parametrize("precision", ["f64", "f32"])
def test_many_planes_near_grid(name, nrhs, precision):
    # 16 or more planes: the projection runs in its own-list form (each
    # thread sums the points covering its two nodes); grids that are not
    # multiples of its tile, 1D and 2D cells, and plane counts that leave
    # a partial last pass
    print("case", name, nrhs, precision, flush=True)
    lat, ref, plan, qv = _setup(name, N=311, seed=71, precision=precision, nrhs=nrhs)
    qd = _to_dev(plan, qv)
    tol = 1e-11 if precision == "f64" else 2e-5
    for adjoint in (False, True):
        got = plan.apply_parts(qd, PARTS["near_grid"], adjoint=adjoint).cpu().numpy()
        want = (ref.adjoint if adjoint else ref.apply)(qv, parts=("near_grid",))
        e, em = rel(got, want), elem(got, want)
        print("  adjoint", adjoint, "rel %.2e max elem %.2e" % (e, em), flush=True)
        assert e < tol and em < 5 * tol, (name, adjoint, e, em)
    plan.close()


@pytest.mark.parametrize("name", list(CASES))
def test_symmetric_block_layout(name):
    # the in-cell correction stored once per box pair (+ a close-image CSR)
    # must give the same operator, forward and conjugate transpose
    lat, ref, plan, qv = _setup(name, N=400, seed=17, corr_layout="sym")
    qd = _to_dev(plan, qv)
    for adjoint in (False, True):
        got = plan.apply_parts(qd, 2, adjoint=adjoint).cpu().numpy()
        want = (ref.adjoint if adjoint else ref.apply)(qv, parts=("near_corr",))
        assert rel(got, want) < 1e-11, adjoint
        got = plan.apply_parts(qd, 7, adjoint=adjoint).cpu().numpy()
        want = (ref.adjoint if adjoint else ref.apply)(qv)
        assert rel(got, want) < 1e-11, adjoint


def test_symmetric_layout_dense_boxes_many_rhs():
    # clustered points (many per box) and several planes through the block path
    lat, ref, plan, qv = _setup("helm2_bloch", N=1500, seed=19, corr_layout="sym", nrhs=3)
    qd = _to_dev(plan, qv)
    for adjoint in (False, True):
        got = plan.apply_parts(qd, 2, adjoint=adjoint).cpu().numpy()
        want = (ref.adjoint if adjoint else ref.apply)(qv, parts=("near_corr",))
        assert rel(got, want) < 1e-11, adjoint


@pytest.mark.parametrize("name", list(CASES))
def test_csr_layout(name):
    # every corrected triple in one CSR (rows processed in tile order)
    lat, ref, plan, qv = _setup(name, N=400, seed=23, corr_layout="csr")
    qd = _to_dev(plan, qv)
    for adjoint in (False, True):
        got = plan.apply_parts(qd, 2, adjoint=adjoint).cpu().numpy()
        want = (ref.adjoint if adjoint else ref.apply)(qv, parts=("near_corr",))
        assert rel(got, want) < 1e-11, adjoint


@pytest.mark.parametrize("name", ["npsp3_real", "npsp2_real", "npsp1_real"])
@pytest.mark.parametrize("nrhs", [3, 19, 80])
def test_tile_layout(name, nrhs):
    # real correction values in dense 16-observer tiles on the matrix cores
    lat, ref, plan, qv = _setup(name, N=400, seed=29, nrhs=nrhs, corr_layout="tile")
    assert plan.info()["corr_layout_used"] == 3
    qd = _to_dev(plan, qv)
    for adjoint in (False, True):
        got = plan.apply_parts(qd, 2, adjoint=adjoint).cpu().numpy()
        want = (ref.adjoint if adjoint else ref.apply)(qv, parts=("near_corr",))
        assert rel(got, want) < 1e-11, adjoint


def test_tile_layout_rejects_complex_values():
    fp = _fftpim()
    latkw, kind, nrhs, vt, nn, q, rc, nf, qf = CASES["helm3"]
    src = W.uniform_cube(100, 4)
    with pytest.raises(fp.FFTPIMError):
        fp.Plan(torch.tensor(src, device="cuda"), 3, latkw["L"], k0=latkw["k0"], near_n=nn, near_order=q,
                corr_radius=rc, far_n=nf, far_order=qf, corr_layout="tile")


@pytest.mark.parametrize("name", ["helm2_bloch", "phase3_static"])
def test_autograd_amplitude_gradient(name):
    # L = Re(c^H A q): the autograd gradient must equal A^H c (oracle) and the
    # central differences of L in the real and imaginary parts of q
    lat, ref, plan, qv = _setup(name, N=120, seed=37, nrhs=1)
    fp = _fftpim()
    rng = np.random.default_rng(38)
    c = rng.standard_normal(qv.shape) + 1j * rng.standard_normal(qv.shape)
    cd = torch.tensor(c, device="cuda")
    q = _to_dev(plan, qv).requires_grad_(True)
    loss = torch.real(torch.sum(torch.conj(cd) * fp.apply_autograd(plan, q)))
    loss.backward()
    g = q.grad.cpu().numpy()
    assert rel(g, ref.adjoint(c)) < 1e-11

    def L(qq):
        with torch.no_grad():
            return float(torch.real(torch.sum(torch.conj(cd) * plan.apply(qq))))
    h = 1e-3
    for k in (0, 17, 63):
        e = torch.zeros_like(q)
        e[0, k] = 1.0
        base = q.detach()
        dre = (L(base + h * e) - L(base - h * e)) / (2 * h)
        dim = (L(base + 1j * h * e) - L(base - 1j * h * e)) / (2 * h)
        assert abs(complex(dre, dim) - g[0, k]) < 1e-9 * max(1.0, abs(g[0, k])), k


@pytest.mark.parametrize("name,layout,nrhs,N", [
    ("helm2_bloch", "sym", 2, 400), ("helm2_bloch", "csr", 2, 400), ("helm2_bloch", "sym", 3, 1500),
    ("phase3_static", "sym", 1, 400), ("helm3", "auto", 1, 400), ("npsp3_real", "sym", 3, 400),
    ("npsp3_real", "tile", 19, 400), ("npsp1_real", "csr", 2, 400), ("npsp2_real", "auto", 4, 400)])
def test_apply_pair(name, layout, nrhs, N):
    # (A q, A^H v) in one call: each equals the oracle and the two single
    # calls (the box-pair layout carries q's and v's planes through one pass)
    print("case", name, layout, nrhs, N, flush=True)
    lat, ref, plan, qv = _setup(name, N=N, seed=41, nrhs=nrhs, corr_layout=layout)
    rng = np.random.default_rng(42)
    if plan.value_type == "real":
        v = rng.standard_normal(qv.shape)
    else:
        v = rng.standard_normal(qv.shape) + 1j * rng.standard_normal(qv.shape)
    qd, vd = _to_dev(plan, qv), _to_dev(plan, v)
    want_w = ref.adjoint(v)
    if lat.npsp:
        want_w = want_w - want_w.mean(axis=-1, keepdims=True)
    want_u = ref.apply(qv)
    for k in (nrhs, 1):
        u, w = plan.apply_pair(qd[:k], vd[:k])
        assert plan.last_status() == 0
        u1 = plan.apply(qd[:k]).cpu().numpy()
        w1 = plan.adjoint(vd[:k]).cpu().numpy()
        u, w = u.cpu().numpy(), w.cpu().numpy()
        assert rel(u, u1) < 1e-14 and rel(w, w1) < 1e-14, (k, rel(u, u1), rel(w, w1))
        assert rel(u, want_u[:k]) < 1e-11 and rel(w, want_w[:k]) < 1e-11, k


def test_apply_pair_fp32():
    lat, ref, plan, qv = _setup("helm2_bloch", N=400, seed=43, precision="f32", corr_layout="sym")
    rng = np.random.default_rng(44)
    v = rng.standard_normal(qv.shape) + 1j * rng.standard_normal(qv.shape)
    u, w = plan.apply_pair(_to_dev(plan, qv), _to_dev(plan, v))
    u, w = u.cpu().numpy(), w.cpu().numpy()
    assert rel(u, ref.apply(qv)) < 2e-5 and elem(u, ref.apply(qv)) < 1e-4
    assert rel(w, ref.adjoint(v)) < 2e-5 and elem(w, ref.adjoint(v)) < 1e-4


@pytest.mark.parametrize("name", ["npsp3_real", "npsp2_real"])
def test_far_bf16_modes(name):
    # the far grid sum on bfloat16 inputs (FP32 accumulation) once planes are
    # batched.  Rounding K and the grid amplitudes to 8 significant bits
    # (unit roundoff 2^-8 against 2^-24) may cost up to 2^16 times the FP32
    # path's error on the same (cancellation-prone, neutral-source) far sum;
    # the three-product split keeps about 16 bits (2^-16: up to 2^8 times the
    # FP32 error).  Each result must be worse than FP32 (its path ran) but
    # within its factor, the split much better than plain bfloat16, and the
    # whole apply's error the far part's error diluted by the far part's
    # share of the result
    lat, ref, plan16, qv = _setup(name, N=400, seed=47, nrhs=19, precision="f32_farbf16")
    plan3 = _setup(name, N=400, seed=47, nrhs=19, precision="f32_farbf16x3")[2]
    plan32 = _setup(name, N=400, seed=47, nrhs=19, precision="f32")[2]
    qd = _to_dev(plan16, qv)
    for adjoint in (False, True):
        op = ref.adjoint if adjoint else ref.apply
        want = op(qv, parts=("far",))
        whole_want = op(qv)
        share = np.linalg.norm(want) / np.linalg.norm(whole_want)
        e = {}
        for key, pl in (("bf16", plan16), ("bf16x3", plan3), ("fp32", plan32)):
            e[key] = rel(pl.apply_parts(qd, 4, adjoint=adjoint).cpu().numpy(), want)
            ew = rel(pl.apply_parts(qd, 7, adjoint=adjoint).cpu().numpy(), whole_want)
            print(name, adjoint, key, "far rel %.2e whole %.2e (far share %.2f)" % (e[key], ew, share), flush=True)
            assert ew < 1.5 * e[key] * share + 2e-5, (key, ew, e[key], share)
        assert 10 * e["fp32"] < e["bf16"] < 2.0 ** 16 * e["fp32"] and e["bf16"] < 0.1, e
        assert e["bf16x3"] < e["bf16"] / 20 and e["bf16x3"] < 2.0 ** 8 * e["fp32"], e


def _bf16(x):
    """float32 values rounded to bfloat16 (nearest, ties to even, on the upper
    half of the binary32 encoding), returned as float64."""
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def _bf16_product(K, Q, split):
    """Q @ K.T with both operands taken through bfloat16 (float32 first), the
    products exact and summed in float64; split: the three-product form
    lo.hi + hi.lo + hi.hi with hi = bf16(x), lo = bf16(x - hi)."""
    K32, Q32 = K.astype(np.float32), Q.astype(np.float32)
    Kh, Qh = _bf16(K32), _bf16(Q32)
    if not split:
        return Qh @ Kh.T
    Kl = _bf16((K32.astype(np.float64) - Kh).astype(np.float32))
    Ql = _bf16((Q32.astype(np.float64) - Qh).astype(np.float32))
    return Ql @ Kh.T + Qh @ Kl.T + Qh @ Kh.T


@pytest.mark.parametrize("name", ["npsp3_real", "npsp2_real"])
def test_far_bf16_modes_match_host_emulation(name):
    # the far part of both bfloat16 modes against a host emulation of the
    # same rounding: the oracle's far grid amplitudes and kernel table taken
    # to float32 and then to bfloat16 (or split into two bfloat16 parts),
    # their products summed in float64, and the oracle's interpolation.  The
    # library differs from the emulation only by float32 accumulation and by
    # the float32 rounding of its grid amplitudes (which can move a value
    # across a bfloat16 rounding boundary): the difference must stay within
    # four times the float32 mode's own far-part error, and for plain
    # bfloat16 under a hundredth of the mode's departure from the unrounded
    # far part (the split mode's departure is only about ten times the
    # float32 error)
    _, ref32, plan32, qv32 = _setup(name, N=400, seed=47, nrhs=19, precision="f32")
    e32 = {}
    for adjoint in (False, True):
        got = plan32.apply_parts(_to_dev(plan32, qv32), PARTS["far"], adjoint=adjoint).cpu().numpy()
        e32[adjoint] = rel(got, (ref32.adjoint if adjoint else ref32.apply)(qv32, parts=("far",)).real)
    plan32.close()
    for prec, split in (("f32_farbf16", False), ("f32_farbf16x3", True)):
        lat, ref, plan, qv = _setup(name, N=400, seed=47, nrhs=19, precision=prec)
        qd = _to_dev(plan, qv)
        K = ref._far_matrix().real  # static lattices: a real far kernel
        for adjoint in (False, True):
            if adjoint:
                Qg = S._spread(ref.fst_obs, qv, ref.Ngf).real
                emu = S._interp(ref.fst_src, _bf16_product(K.T, Qg, split), np.arange(ref.src.shape[0]))
            else:
                Qg = S._spread(ref.fst_src, qv, ref.Ngf).real
                emu = S._interp(ref.fst_obs, _bf16_product(K, Qg, split), np.arange(ref.obs.shape[0]))
            exact = (ref.adjoint if adjoint else ref.apply)(qv, parts=("far",)).real
            got = plan.apply_parts(qd, PARTS["far"], adjoint=adjoint).cpu().numpy()
            d_lib, d_mode = rel(got, emu), rel(emu, exact)
            print(name, prec, "adjoint", adjoint, "library vs emulation %.2e, emulation vs unrounded %.2e, "
                  "float32 mode %.2e" % (d_lib, d_mode, e32[adjoint]), flush=True)
            assert d_lib < 4 * e32[adjoint], (name, prec, adjoint, d_lib, e32[adjoint])
            if not split:
                assert d_lib < 0.01 * d_mode, (name, prec, adjoint, d_lib, d_mode)
        plan.close()


@pytest.mark.parametrize("near_n", [(32, 32, 32), (64, 64, 32), (256, 16, 16)])
def test_fp32_register_fft_lengths(near_n):
    # FP32 strided passes run the register transform (line lengths 64, 128
    # and 512 here; 16, 32 and 256 are covered by the other FP32 tests), FP64
    # the LDS-stage kernel: with one plane both near grid parts are compared
    # with the oracle's, and with batched planes FP32 with FP64, forward and
    # adjoint, to FP32 rounding
    fp = _fftpim()
    rng = np.random.default_rng(53)
    N = 1500
    src = rng.random((N, 3))
    pos = torch.tensor(src, dtype=torch.float64, device="cuda")
    ref = S.FFTPIM(P.Lattice(3, [1.0, 1.0, 1.0], 3.0, [0.4, 0.2, 0.1]), S.Params(near_n, 3, 3, (8, 8, 8), 3, 1), src)
    for nrhs in (1, 12):
        plans = [fp.Plan(pos, 3, [1.0, 1.0, 1.0], k0=3.0, kt=[0.4, 0.2, 0.1], near_n=near_n, near_order=3,
                         corr_radius=3, far_n=(8, 8, 8), far_order=3, precision=prec, nrhs_max=nrhs)
                 for prec in ("f64", "f32")]
        q = rng.standard_normal((nrhs, N)) + 1j * rng.standard_normal((nrhs, N))
        for adjoint in (False, True):
            u64 = plans[0].apply_parts(_to_dev(plans[0], q), 1, adjoint=adjoint).cpu().numpy()
            u32 = plans[1].apply_parts(_to_dev(plans[1], q), 1, adjoint=adjoint).cpu().numpy()
            if nrhs == 1:
                want = (ref.adjoint if adjoint else ref.apply)(q, parts=("near_grid",))
                e64, e32, m32 = rel(u64, want), rel(u32, want), elem(u32, want)
                print(near_n, adjoint, "near grid vs oracle: fp64 %.2e fp32 %.2e (max elem %.2e)" % (e64, e32, m32),
                      flush=True)
                assert e64 < 1e-11 and e32 < 2e-5 and m32 < 1e-4, (near_n, adjoint, e64, e32, m32)
            err = rel(u32, u64)
            print(near_n, nrhs, adjoint, "fp32 vs fp64 near grid rel %.2e" % err, flush=True)
            assert err < 2e-5, (near_n, nrhs, adjoint, err)
        for p in plans:
            p.close()


def test_far_bf16_modes_fall_back_below_eight_planes():
    # with fewer than 8 planes the far grid sum is not a GEMM and every mode
    # uses the FP32 grid sum: the results equal the FP32 mode's bitwise
    outs = {}
    for prec in ("f32", "f32_farbf16", "f32_farbf16x3"):
        lat, ref, plan, qv = _setup("npsp3_real", N=300, seed=59, nrhs=3, precision=prec)
        outs[prec] = plan.apply_parts(_to_dev(plan, qv), 4).cpu().numpy()
        plan.close()
    assert np.array_equal(outs["f32"], outs["f32_farbf16"])
    assert np.array_equal(outs["f32"], outs["f32_farbf16x3"])


def test_apply_pair_rejects_bad_arguments():
    fp = _fftpim()
    lat, ref, plan, qv = _setup("helm2_bloch", N=200, seed=61, nrhs=2)
    qd = _to_dev(plan, qv)
    big = torch.zeros((plan.params.nrhs_max + 1, plan.N), dtype=plan.dtype, device="cuda")
    with pytest.raises(fp.FFTPIMError):
        plan.apply_pair(big, big)
    with pytest.raises(ValueError):
        plan.apply_pair(qd, qd[:1])
    # a valid call after the rejected ones still matches the single calls
    u, w = plan.apply_pair(qd, qd)
    assert rel(u.cpu().numpy(), plan.apply(qd).cpu().numpy()) < 1e-14
    assert rel(w.cpu().numpy(), plan.adjoint(qd).cpu().numpy()) < 1e-14
    plan.close()


@pytest.mark.parametrize("name", ["npsp3_real", "helm2_bloch", "helm1_bloch", "coax_dyn", "npsp1_real"])
def test_self_exclude(name):
    # Eq. (5) read literally (n != m): the library subtracts its own
    # lim_{r->0}[G^p - G0] q_m, the oracle its own; forward, conjugate
    # transpose, one stage alone and the fused pair
    print("case", name, flush=True)
    lat, ref, plan, qv = _setup(name, self_mode="exclude")
    qd = _to_dev(plan, qv)
    u = plan.apply(qd).cpu().numpy()
    assert rel(u, ref.apply(qv)) < 1e-11
    want_w = ref.adjoint(qv)
    if lat.npsp:
        want_w = want_w - want_w.mean(axis=-1, keepdims=True)
    w = plan.adjoint(qd).cpu().numpy()
    assert rel(w, want_w) < 1e-11
    got = plan.apply_parts(qd, PARTS["far"]).cpu().numpy()
    assert rel(got, ref.apply(qv, parts=("far",))) < 1e-11
    up, wp = plan.apply_pair(qd, qd)
    assert rel(up.cpu().numpy(), ref.apply(qv)) < 1e-11
    assert rel(wp.cpu().numpy(), want_w) < 1e-11
    # the difference from the default mode is exactly C_self q_m
    lat2, ref2, plan2, _ = _setup(name)
    d = plan2.apply(qd).cpu().numpy() - u
    cs = _fftpim().eval_pgf_self(lat.dims, lat.L[:lat.dims], lat.k0, lat.kt[:lat.dims])
    np.testing.assert_allclose(d, cs * qv if plan.value_type == "complex" else cs.real * qv,
                               rtol=1e-9, atol=1e-12 * np.abs(u).max())


@pytest.mark.parametrize("name,layout,nrhs", [
    ("npsp3_real", "sym", None), ("npsp3_real", "csr", None), ("npsp3_real", "tile", 19),
    ("helm2_bloch", "sym", None), ("helm2_bloch", "csr", None), ("helm1_bloch", "auto", None),
    ("npsp2_real", "auto", None), ("helm3_cphase", "csr", None),
])
def test_ball_region(name, layout, nrhs):
    # the ball correction region of Eq. (er) (radius in units of the largest
    # near-grid spacing; anisotropic spacings in the slab and surface cases)
    print("case", name, layout, flush=True)
    lat, ref, plan, qv = _setup(name, corr_layout=layout, nrhs=nrhs, corr_ball=7.0)
    qd = _to_dev(plan, qv)
    for adjoint in (False, True):
        got = plan.apply_parts(qd, PARTS["near_corr"], adjoint=adjoint).cpu().numpy()
        want = (ref.adjoint if adjoint else ref.apply)(qv, parts=("near_corr",))
        assert rel(got, want) < 1e-11, adjoint
        got = plan.apply_parts(qd, 7, adjoint=adjoint).cpu().numpy()
        want = (ref.adjoint if adjoint else ref.apply)(qv)
        assert rel(got, want) < 1e-11, adjoint
    up, wp = plan.apply_pair(qd, qd)
    want_w = ref.adjoint(qv)
    if lat.npsp:
        want_w = want_w - want_w.mean(axis=-1, keepdims=True)
    assert rel(up.cpu().numpy(), ref.apply(qv)) < 1e-11
    assert rel(wp.cpu().numpy(), want_w) < 1e-11


def test_ball_region_rejects_too_small_radius():
    fp = _fftpim()
    src = W.uniform_cube(100, 2)
    with pytest.raises(fp.FFTPIMError):
        fp.Plan(torch.tensor(src, device="cuda"), 3, [1, 1, 1], near_n=(16, 16, 16), near_order=4,
                far_n=(10, 10, 10), far_order=5, corr_ball=6.0)   # 4 sqrt(3) = 6.93 needed
