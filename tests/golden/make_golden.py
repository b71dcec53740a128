"""Write the stored exact potentials used by the full-size workload tests.

Every value is computed by the FP64 direct-sum oracle (oracle.psp) on the
seeded inputs of paper_2312_02376_amd.workloads; nothing here touches the GPU
library.  Run from the repository root:

    python tests/golden/make_golden.py [coulomb_1k] [helmholtz_100k] [coulomb_1m] [dynamic_cube_20k]
        [multi_cell_small] [multi_cell_48] [forces_2m]

forces_2m is not in the default list: it takes about half an hour on 8 cores.
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import grad as OG  # noqa: E402
from oracle import pgf as P  # noqa: E402
from oracle.psp import host_workers, psp_adjoint, psp_forward  # noqa: E402
from paper_2312_02376_amd import workloads as W  # noqa: E402

OUT = os.path.dirname(os.path.abspath(__file__))


def _save(name, header, cols):
    path = os.path.join(OUT, name)
    np.savetxt(path, np.column_stack(cols), header=header, fmt="%.17g")
    print("wrote", path)


def coulomb_1k():
    src, q = W.coulomb_cube_1k()
    lat = P.Lattice(3, [1.0, 1.0, 1.0])
    u = psp_forward(lat, src, q, workers=host_workers())
    _save("coulomb_cube_1k_exact.txt",
          "3D-periodic Coulomb, unit cube, 1000 uniform points, +-1 charges (workloads.coulomb_cube_1k);\n"
          "exact u = sum_n G^p(r_m - r_n) q_n (singular self image dropped), all 1000 observers.\n"
          "columns: index, u", [np.arange(1000), u.real])


def helmholtz_100k(nrows=256):
    src, q64 = W.helmholtz_surface_100k()
    q = q64.astype(np.complex128)
    v = W.gaussian_complex(1, len(src), 102)[0].astype(np.complex128)
    k = 2 * np.pi
    lat = P.Lattice(2, [1.0, 1.0], k, [0.3 * k, 0.1 * k])
    rows = np.sort(np.random.default_rng(7).choice(len(src), nrows, replace=False))
    u = psp_forward(lat, src, q, obs_index=rows, workers=host_workers())
    w = psp_adjoint(lat, src, v, src_index=rows, workers=host_workers())
    _save("helmholtz_surface_100k_rows.txt",
          "2D-periodic Helmholtz, k0 = 2 pi, kt = (0.3, 0.1) k0, 100k surface points "
          "(workloads.helmholtz_surface_100k);\nexact forward u = A q and conjugate transpose w = A^H v "
          "(v = workloads.gaussian_complex(1, N, 102)) at sampled rows.\ncolumns: row, Re u, Im u, Re w, Im w",
          [rows, u.real, u.imag, w.real, w.imag])


def coulomb_1m(nrows=128):
    src, q = W.coulomb_cube_1m_batched()
    lat = P.Lattice(3, [1.0, 1.0, 1.0])
    rows = np.sort(np.random.default_rng(11).choice(len(src), nrows, replace=False))
    u = psp_forward(lat, src, q.astype(np.float64), obs_index=rows, workers=host_workers())
    cols = [np.repeat(rows, q.shape[0]), np.tile(np.arange(q.shape[0]), nrows), u.real.T.ravel()]
    _save("coulomb_cube_1m_rows.txt",
          "3D-periodic Coulomb, 1M uniform points, 64 neutral Gaussian right-hand sides "
          "(workloads.coulomb_cube_1m_batched);\nexact u at sampled rows.\ncolumns: row, rhs, u", cols)


def dynamic_cube_20k(nrows=32):
    # Sec. 4.2 (Fig. complex_real): a 100^3 cube of points in a 3D-periodic
    # cell of period 101, k0 chosen so that the mean spacing is lambda/20,
    # phase wavenumbers 0.01 - 0.01j on every axis; the static (NPSP)
    # counterpart uses neutral real strengths on the same points
    src, q = W.dynamic_cube(20000, 8)
    k0 = W.dynamic_cube_k0(len(src))
    lat = P.Lattice(3, [101.0] * 3, k0, [0.01 - 0.01j] * 3)
    rows = np.sort(np.random.default_rng(13).choice(len(src), nrows, replace=False))
    u = psp_forward(lat, src, q.astype(np.complex128), obs_index=rows, workers=host_workers())
    qs = W.gaussian_neutral(1, len(src), 8)[0]
    us = psp_forward(P.Lattice(3, [101.0] * 3), src, qs, obs_index=rows, workers=host_workers())
    _save("dynamic_cube_20k_rows.txt",
          "3D-periodic cell of period 101, 20000 points uniform in a centred 100^3 cube (workloads.dynamic_cube(20000, 8));\n"
          "dynamic: k0 = workloads.dynamic_cube_k0(20000), kt = (0.01 - 0.01j)(1, 1, 1), strengths of dynamic_cube;\n"
          "static: k0 = 0, kt = 0, strengths workloads.gaussian_neutral(1, 20000, 8).\n"
          "exact u at sampled rows. columns: row, Re u_dyn, Im u_dyn, u_static",
          [rows, u.real, u.imag, us.real])


def multi_cell_48(nrows=4):
    # the 48-cell workload of the benchmark (workloads.multi_cell(48, 4)):
    # N log-uniform in [5e3, 5e5], mixed periodicity, static and Helmholtz
    cells = W.multi_cell(48, 4)
    cols = [[], [], [], []]
    for c, cell in enumerate(cells):
        lat = P.Lattice(cell["dims"], cell["L"], cell["k0"], cell["kt"])
        n = len(cell["q"])
        rows = np.sort(np.random.default_rng(200 + c).choice(n, nrows, replace=False))
        u = psp_forward(lat, cell["pos"], cell["q"], obs_index=rows, workers=host_workers())
        cols[0].append(np.full(nrows, c))
        cols[1].append(rows)
        cols[2].append(u.real)
        cols[3].append(u.imag)
        print("cell", c, "done", flush=True)
    _save("multi_cell_48_rows.txt",
          "48 independent cells, workloads.multi_cell(48, 4);\n"
          "exact u = A q at sampled rows of each cell.\ncolumns: cell, row, Re u, Im u",
          [np.concatenate(x) for x in cols])


def multi_cell_small(nrows=16):
    # eight independent cells of uneven size (workloads.multi_cell(8, 21,
    # 2000, 12000)): mixed periodicity, static and Helmholtz
    cells = W.multi_cell(8, 21, 2000, 12000)
    cols = [[], [], [], []]
    for c, cell in enumerate(cells):
        lat = P.Lattice(cell["dims"], cell["L"], cell["k0"], cell["kt"])
        n = len(cell["q"])
        rows = np.sort(np.random.default_rng(100 + c).choice(n, nrows, replace=False))
        u = psp_forward(lat, cell["pos"], cell["q"], obs_index=rows, workers=host_workers())
        cols[0].append(np.full(nrows, c))
        cols[1].append(rows)
        cols[2].append(u.real)
        cols[3].append(u.imag)
    _save("multi_cell_small_rows.txt",
          "eight independent cells, workloads.multi_cell(8, 21, 2000, 12000);\n"
          "exact u = A q at sampled rows of each cell.\ncolumns: cell, row, Re u, Im u",
          [np.concatenate(x) for x in cols])


def _forces_row(args):
    src, q, k = args
    return OG.psp_grad(P.Lattice(3, [1.0, 1.0, 1.0]), src, q, q, [k])[0]


def forces_2m(nrows=8):
    # the 2M-point 3D-periodic Coulomb cell of the forces record: 2M uniform
    # points (seed 5), one neutral Gaussian right-hand side (seed 5, drawn in
    # float32 as the record does); dL/dr_k of L = q . (A q) at sampled rows
    import multiprocessing as mp
    N = 2_000_000
    src = W.uniform_cube(N, 5)
    q = W.gaussian_neutral(1, N, 5, np.float32)[0].astype(np.float64)
    rows = np.sort(np.random.default_rng(13).choice(N, nrows, replace=False))
    with mp.get_context("fork").Pool(min(nrows, host_workers())) as pool:
        g = np.array(pool.map(_forces_row, [(src, q, int(k)) for k in rows]))
    _save("forces_cube_2m_rows.txt",
          "3D-periodic Coulomb, unit cube, 2M uniform points (workloads.uniform_cube(2000000, 5)), one neutral\n"
          "Gaussian right-hand side q (workloads.gaussian_neutral(1, N, 5, float32)); exact dL/dr_k of\n"
          "L = q . (A q) at sampled rows (oracle.grad.psp_grad).\ncolumns: row, dL/dx, dL/dy, dL/dz",
          [rows, g[:, 0], g[:, 1], g[:, 2]])


if __name__ == "__main__":
    which = sys.argv[1:] or ["coulomb_1k", "helmholtz_100k", "coulomb_1m", "dynamic_cube_20k", "multi_cell_small",
                             "multi_cell_48"]
    for w in which:
        globals()[w]()
