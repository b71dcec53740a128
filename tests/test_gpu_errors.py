"""Error paths of the C ABI on the GPU, forced from the host: points outside
the cell on a periodic axis (OUT_OF_CELL, for sources and for separate
observers), a device-memory cap below what the plan needs (NO_MEMORY), and
that a plan made afterwards on the same device works and matches the oracle
(no state is left behind by the failed plans)."""
import numpy as np
import pytest

from oracle import pgf as P
from oracle import steps as S
from paper_2312_02376_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KW = dict(near_n=(16, 16, 16), near_order=4, corr_radius=4, far_n=(10, 10, 10), far_order=5, value_type="real")


def _fp():
    from paper_2312_02376_amd import fftpim
    return fftpim


@pytest.mark.parametrize("bad", [1.0, -1e-9, 1.5])
def test_points_outside_the_cell(bad):
    fp = _fp()
    src = W.uniform_cube(200, 3)
    src[17, 1] = bad  # y is periodic: [0, 1) only
    with pytest.raises(fp.FFTPIMError) as e:
        fp.Plan(torch.tensor(src, device="cuda"), 3, [1, 1, 1], **KW)
    assert e.value.code == 2
    good = W.uniform_cube(200, 3)
    obs = W.uniform_cube(50, 4)
    obs[3, 0] = bad
    with pytest.raises(fp.FFTPIMError) as e:
        fp.Plan(torch.tensor(good, device="cuda"), 3, [1, 1, 1], observers=torch.tensor(obs, device="cuda"), **KW)
    assert e.value.code == 2


def test_points_outside_the_box_and_not_finite():
    fp = _fp()
    src = np.c_[W.uniform_cube(200, 9)[:, :2], 0.1 + 0.3 * W.uniform_cube(200, 10)[:, 2]]
    kw = dict(KW, box=([0, 0, 0.0], [1, 1, 0.5]))
    pos = src.copy()
    pos[5, 2] = 0.6  # z is not periodic: the given box is [0, 0.5]
    with pytest.raises(fp.FFTPIMError) as e:
        fp.Plan(torch.tensor(pos, device="cuda"), 2, [1, 1], **kw)
    assert e.value.code == 2
    pos = src.copy()
    pos[7, 0] = np.nan
    with pytest.raises(fp.FFTPIMError) as e:
        fp.Plan(torch.tensor(pos, device="cuda"), 2, [1, 1], **kw)
    assert e.value.code == 1


def test_memory_cap():
    fp = _fp()
    src = W.uniform_cube(300, 5)
    pos = torch.tensor(src, device="cuda")
    plan = fp.Plan(pos, 3, [1, 1, 1], nrhs_max=2, **KW)
    need = plan.info()["device_bytes"]
    q = torch.tensor(W.gaussian_neutral(2, 300, 6), device="cuda")
    want = plan.apply(q)
    plan.close()
    with pytest.raises(fp.FFTPIMError) as e:
        fp.Plan(pos, 3, [1, 1, 1], nrhs_max=2, max_bytes=need // 2, **KW)
    assert e.value.code == 6
    # a cap the plan fits in is accepted; the first fused pair call then
    # allocates beyond it and is refused, and the plan stays usable
    plan = fp.Plan(pos, 3, [1, 1, 1], nrhs_max=2, max_bytes=need + 4096, **KW)
    assert plan.info()["device_bytes"] == need
    with pytest.raises(fp.FFTPIMError) as e:
        plan.apply_pair(q, q)
    assert e.value.code == 6
    assert torch.equal(plan.apply(q), want)
    assert plan.last_status() == 0
    plan.close()


def test_a_plan_after_the_failures_matches_the_oracle():
    fp = _fp()
    src = W.uniform_cube(300, 7)
    q = W.gaussian_neutral(1, 300, 8)
    plan = fp.Plan(torch.tensor(src, device="cuda"), 3, [1, 1, 1], **KW)
    u = plan.apply(torch.tensor(q, device="cuda")).cpu().numpy()
    assert plan.last_status() == 0
    ref = S.FFTPIM(P.Lattice(3, [1, 1, 1]), S.Params((16, 16, 16), 4, 4, (10, 10, 10), 5, 1), src).apply(q)
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) < 1e-11
    plan.close()
