"""Argument checks of the Python binding that run before any library call:
inputs and caller-supplied outputs must have the plan's dtype and device, the
input's shape, be contiguous, and (for the fused pair) not overlap.  A stub
plan on the CPU device stands in for a planned one, so these run without a
GPU and never reach the library."""
import pytest

torch = pytest.importorskip("torch")

from paper_2312_02376_amd import fftpim as fp  # noqa: E402


def _stub(N=7, dtype=torch.complex128, M=None):
    p = fp.Plan.__new__(fp.Plan)
    p.N = N
    p.M = N if M is None else M
    p.dtype = dtype
    p.device = torch.device("cpu")
    p._h = None
    return p


def test_input_checks():
    p = _stub()
    with pytest.raises(TypeError):
        p._io(torch.zeros(7, dtype=torch.complex64), None)
    with pytest.raises(ValueError):
        p._io(torch.zeros(6, dtype=torch.complex128), None)
    x2, out, sq = p._io(torch.zeros(2, 7, dtype=torch.complex128), None)
    assert out.shape == (2, 7) and not sq


@pytest.mark.parametrize("bad,exc", [
    (lambda: torch.zeros(2, 7, dtype=torch.complex64), TypeError),          # wrong dtype
    (lambda: torch.zeros(2, 6, dtype=torch.complex128), ValueError),         # wrong shape
    (lambda: torch.zeros(1, 14, dtype=torch.complex128), ValueError),        # same size, other shape
    (lambda: torch.zeros(7, 2, dtype=torch.complex128).t(), ValueError),     # not contiguous
    (lambda: torch.zeros(2, 7, dtype=torch.float64), TypeError),             # real for complex
    (lambda: [0.0] * 14, TypeError),                                         # not a tensor
])
def test_output_checks(bad, exc):
    p = _stub()
    with pytest.raises(exc):
        p._io(torch.zeros(2, 7, dtype=torch.complex128), bad())


def test_output_may_not_alias_input():
    p = _stub()
    x = torch.zeros(2, 7, dtype=torch.complex128)
    with pytest.raises(ValueError):
        p._io(x, x)
    with pytest.raises(ValueError):
        p._io(x[1], x[1])


def test_vector_input_accepts_vector_output():
    p = _stub()
    x2, out, sq = p._io(torch.zeros(7, dtype=torch.complex128), torch.zeros(7, dtype=torch.complex128))
    assert sq and out.shape == (1, 7)


def test_pair_outputs_may_not_overlap():
    p = _stub()
    q = torch.zeros(2, 7, dtype=torch.complex128)
    v = torch.zeros(2, 7, dtype=torch.complex128)
    buf = torch.zeros(3, 7, dtype=torch.complex128)
    with pytest.raises(ValueError):
        p.apply_pair(q, v, out_u=buf[0:2], out_w=buf[1:3])
    with pytest.raises(ValueError):
        p.apply_pair(q, v, out_u=v.clone(), out_w=q)


def test_separate_observer_shapes():
    # 7 sources, 5 observers: apply takes 7 and gives 5, the adjoint the reverse
    p = _stub(7, M=5)
    x2, out, sq = p._io(torch.zeros(2, 7, dtype=torch.complex128), None)
    assert out.shape == (2, 5)
    x2, out, sq = p._io(torch.zeros(2, 5, dtype=torch.complex128), None, adjoint=True)
    assert out.shape == (2, 7)
    with pytest.raises(ValueError):
        p._io(torch.zeros(2, 5, dtype=torch.complex128), None)
    with pytest.raises(ValueError):
        p._io(torch.zeros(2, 7, dtype=torch.complex128), torch.zeros(2, 7, dtype=torch.complex128))
    x2, out, sq = p._io(torch.zeros(7, dtype=torch.complex128), torch.zeros(5, dtype=torch.complex128))
    assert sq and out.shape == (1, 5)
