"""Many independent cells (fftpim_autotune, fftpim_batch_*) through the C
ABI: eight cells of uneven size with mixed periodicity, static and
Helmholtz kernels (workloads.multi_cell), each planned with the parameters
the cost model picks for a target error, applied together in one batch
and compared with the single-cell applies (bit for bit: the same
kernels on the same data) and with exact sums of Eq. (1) (tests/golden)."""
import os

import numpy as np
import pytest

from paper_2312_02376_amd import workloads as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _fp():
    from paper_2312_02376_amd import fftpim
    return fftpim


@pytest.fixture(scope="module")
def cells():
    fp = _fp()
    cs = W.multi_cell(8, 21, 2000, 12000)
    gold = np.loadtxt(os.path.join(GOLD, "multi_cell_small_rows.txt"))
    out = []
    for c, cell in enumerate(cs):
        pos = torch.tensor(cell["pos"], device="cuda")
        kw, rep = fp.autotune(pos, cell["dims"], cell["L"], 1e-4, k0=cell["k0"], kt=cell["kt"])
        print("cell", c, "dims", cell["dims"], "k0 %.2f" % cell["k0"], "N", len(cell["q"]), kw, rep, flush=True)
        plan = fp.Plan(pos, cell["dims"], cell["L"], k0=cell["k0"], kt=cell["kt"], **kw)
        sel = gold[:, 0] == c
        out.append(dict(plan=plan, q=torch.tensor(cell["q"], device="cuda"), rep=rep, kw=kw,
                        rows=gold[sel, 1].astype(np.int64), exact=gold[sel, 2] + 1j * gold[sel, 3]))
    yield out
    for x in out:
        x["plan"].close()


def test_autotuned_cells_meet_the_target(cells):
    for c, x in enumerate(cells):
        assert x["rep"]["predicted_rel_err"] <= 1e-4
        u = x["plan"].apply(x["q"]).cpu().numpy()
        assert x["plan"].last_status() == 0
        e = float(np.linalg.norm(u[x["rows"]] - x["exact"]) / np.linalg.norm(x["exact"]))
        print("cell", c, "rel err %.2e (predicted %.2e)" % (e, x["rep"]["predicted_rel_err"]), flush=True)
        assert e <= 1e-4, (c, e)


GRAPH_OFF = ("recording the batch as a HIP graph is switched off in the library: its first run ended in a host "
             "segmentation fault whose cause was not found; the library returns UNSUPPORTED for it")


@pytest.mark.parametrize("graph", [False, pytest.param(True, marks=pytest.mark.skip(reason=GRAPH_OFF))])
@pytest.mark.parametrize("adjoint", [False, True])
def test_batch_matches_single_cell_applies(cells, graph, adjoint):
    fp = _fp()
    plans = [x["plan"] for x in cells]
    ins = [x["q"] for x in cells]
    want = [(p.adjoint if adjoint else p.apply)(q) for p, q in zip(plans, ins)]
    torch.cuda.synchronize()
    batch = fp.Batch(plans, lanes=4, graph=graph)
    outs = [torch.empty_like(q) for q in ins]
    for rep in range(3):
        # eager work of the program between the (replayed) batch calls
        for o in outs:
            o.fill_(float("nan"))
        got = batch.apply(ins, outs, adjoint=adjoint)
        torch.cuda.synchronize()
        for c, (g, w) in enumerate(zip(got, want)):
            assert torch.equal(g, w), (graph, adjoint, rep, c)
        scratch = torch.randn(1 << 20, device="cuda")
        scratch.mul_(2.0)
        torch.cuda.synchronize()
    batch.close()


def test_batch_argument_checks(cells):
    fp = _fp()
    with pytest.raises(fp.FFTPIMError):
        fp.Batch([x["plan"] for x in cells], graph=True)
    with pytest.raises(ValueError):
        fp.Batch([x["plan"] for x in cells]).apply([cells[0]["q"]])
    with pytest.raises(fp.FFTPIMError):
        fp.Batch([x["plan"] for x in cells], lanes=0)
