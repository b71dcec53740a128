"""Benchmark: observer points/s per FFT-PIM apply (forward + conjugate
transpose) on one MI355X.

Workload (the paper's Helmholtz case with a phase shift, synthetic): a
2D-periodic cell of 1 x 1 wavelengths (k0 = 2 pi), phase shifts
k_x0 = 0.3 k0 and k_y0 = 0.1 k0, 100,000 points area-uniform on a random smooth
closed surface inside the cell (z in [0, 0.5]), complex N(0,1) strengths
(drawn as complex64, computed in FP64).  Near grid 64 x 64 x 32, Lagrange
degree 4, correction region the ball of Eq. (er) of radius 10.5 times the
largest near-grid spacing; far grid 24 x 24 x 16, degree 7; one near image
layer.  Inputs and outputs stay in the plan's point order (the
iterative-solver use case) and are resident in HBM before timing starts.

One step = u = A q and w = A^H v for two different inputs, both computed in
full by one fftpim_apply_pair call (the box-pair correction reads each stored
block once for both products).  value = N / (time per step), the time per step
being the host wall time of exactly `steps` steps between two device
synchronisations; the median of per-step HIP event times is reported beside
it.  The per-stage HIP-event times behind the roofline entry come from a second
pass of the same steps with stage timing switched on, so the events never sit
inside the timed pass.  The same step made of the two single calls
(fftpim_apply, then fftpim_apply_adjoint) is timed too and reported under
"separate_calls".
The accuracy of the timed configuration is measured in the same run: the
CPU-baseline leg evaluates the direct FP64 pair sum (the oracle) on a sample of
observers, and the relative L2 error of the GPU result on that sample is
reported.
A nested "batched" record times the 1M-point, 64-right-hand-side Coulomb cell
(FP32 bulk, FP64 correction) the same way, with its dominant kernel's roofline,
its error on the stored exact rows, and the same cell with one FP64
right-hand side for the batched-versus-single comparison.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "observer points/s per FFT-PIM apply (fwd+adjoint) at rel-L2 ≤1e-6 vs FP64 oracle"
HBM_PEAK_GBS = 8000.0

WORKLOAD = dict(
    name="2D-periodic Helmholtz with phase shift, 100k points on a closed surface",
    N=100_000, k0=2 * math.pi, kt=(0.3 * 2 * math.pi, 0.1 * 2 * math.pi), L=(1.0, 1.0),
    near_n=(64, 64, 32), near_order=4, corr_radius=10, corr_ball=10.5, far_n=(24, 24, 16), far_order=7,
    n_images=1,
)

# secondary workloads (--workload): timed the same way, without the oracle leg
SECONDARY = {
    "coulomb_1k": dict(name="3D-periodic Coulomb, unit cube, 1000 uniform points, +-1 charges, FP64",
                       dims=3, L=(1.0, 1.0, 1.0), precision="f64", value_type="real", nrhs=1,
                       near_n=(16, 16, 16), near_order=4, corr_radius=14, far_n=(16, 16, 16), far_order=7),
    "coulomb_1m_batched": dict(name="3D-periodic Coulomb, 1M uniform points, 64 neutral Gaussian right-hand "
                                    "sides, FP32 bulk with FP64 correction",
                               dims=3, L=(1.0, 1.0, 1.0), precision="f32", value_type="real", nrhs=64,
                               near_n=(128, 128, 128), near_order=4, corr_radius=5, far_n=(14, 14, 14),
                               far_order=5),
    # the batched workload with the far grid sum on bfloat16 inputs (FP32
    # accumulation); everything else as above
    "coulomb_1m_batched_farbf16": dict(name="3D-periodic Coulomb, 1M uniform points, 64 neutral Gaussian right-hand "
                                            "sides, FP32 bulk, far grid sum with bfloat16 inputs and FP32 "
                                            "accumulation, FP64 correction",
                                       dims=3, L=(1.0, 1.0, 1.0), precision="f32_farbf16", value_type="real",
                                       nrhs=64, near_n=(128, 128, 128), near_order=4, corr_radius=5,
                                       far_n=(14, 14, 14), far_order=5),
    "coulomb_1m_batched_farbf16x3": dict(name="3D-periodic Coulomb, 1M uniform points, 64 neutral Gaussian "
                                              "right-hand sides, FP32 bulk, far grid sum with split (three-product) "
                                              "bfloat16 inputs and FP32 accumulation, FP64 correction",
                                         dims=3, L=(1.0, 1.0, 1.0), precision="f32_farbf16x3", value_type="real",
                                         nrhs=64, near_n=(128, 128, 128), near_order=4, corr_radius=5,
                                         far_n=(14, 14, 14), far_order=5),
    # the same cell and parameters with one FP64 right-hand side (the first of
    # the batch): the single-RHS side of the batched-versus-single comparison
    "coulomb_1m_single_f64": dict(name="3D-periodic Coulomb, 1M uniform points, one Gaussian right-hand side "
                                       "(the first of the batched set), FP64",
                                  dims=3, L=(1.0, 1.0, 1.0), precision="f64", value_type="real", nrhs=1,
                                  near_n=(128, 128, 128), near_order=4, corr_radius=5, far_n=(14, 14, 14),
                                  far_order=5),
}
GOLD_1M = os.path.join(ROOT, "tests", "golden", "coulomb_cube_1m_rows.txt")


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def time_steps(step, steps, warmup):
    """Wall time of exactly `steps` calls of step() between two device
    synchronisations (ms per step), and the median of per-step HIP event
    times on the current stream (ms)."""
    import torch
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    ev[0].record()
    for k in range(steps):
        step()
        ev[k + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = sorted(ev[k].elapsed_time(ev[k + 1]) for k in range(steps))
    return 1e3 * wall / steps, per[len(per) // 2]


def staged_pass(plan, step, steps):
    """Per-stage HIP-event times over `steps` more steps (a pass of its own)."""
    import torch
    torch.cuda.synchronize()
    plan.stage_times(True)
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    return plan.stage_times(False)


def run_secondary(args, key):
    import numpy as np
    import torch

    from paper_2312_02376_amd import fftpim as fp
    from paper_2312_02376_amd import workloads as W
    wl = SECONDARY[key]
    if key == "coulomb_1k":
        src, q = W.coulomb_cube_1k()
        q = q[None, :]
    else:
        src, q = W.coulomb_cube_1m_batched()
        if wl["nrhs"] == 1:
            q = q[:1].astype(np.float64)
    N, nrhs = src.shape[0], q.shape[0]
    dev = torch.device("cuda:0")
    t0 = time.perf_counter()
    plan = fp.Plan(torch.tensor(src, device=dev), wl["dims"], list(wl["L"]), near_n=wl["near_n"],
                   near_order=wl["near_order"], corr_radius=wl["corr_radius"], far_n=wl["far_n"],
                   far_order=wl["far_order"], n_images=1, precision=wl["precision"],
                   value_type=wl["value_type"], order="plan", nrhs_max=nrhs)
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    perm = plan.permutation().long()
    qd = torch.tensor(q, device=dev)[:, perm].contiguous()
    u = torch.empty_like(qd)
    w = torch.empty_like(qd)
    for _ in range(args.warmup):
        plan.apply(qd, out=u)
        plan.adjoint(qd, out=w)
    torch.cuda.synchronize()
    plan.stage_times(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        plan.apply(qd, out=u)
        plan.adjoint(qd, out=w)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stages = plan.stage_times(False)
    ms = 1e3 * elapsed / args.steps
    info = plan.info()
    acc = None
    if key != "coulomb_1k" and os.path.exists(GOLD_1M):
        # forward error on the rows whose exact sums are stored
        g = np.loadtxt(GOLD_1M)
        rows = np.unique(g[:, 0].astype(np.int64))
        gold = g[:, 2].reshape(len(rows), -1).T[:nrhs]
        inv = torch.empty_like(perm)
        inv[perm] = torch.arange(N, device=dev)
        got = u[:, inv[torch.tensor(rows, device=dev)]].double().cpu().numpy()
        acc = float(np.linalg.norm(got - gold) / np.linalg.norm(gold))
    print("stages (ms per launch): " + ", ".join(
        "%s %.4f" % (k, t / c) for k, (t, c) in stages.items() if c), file=sys.stderr, flush=True)
    alone = None
    if args.isolated_parts:
        # each part of the forward apply on its own (no concurrent streams):
        # the launch times a kernel takes without sharing the GPU
        alone = {}
        for bit, part in ((1, "near_grid"), (2, "near_corr"), (4, "far")):
            plan.apply_parts(qd, bit, out=u)
            st = staged_pass(plan, lambda: plan.apply_parts(qd, bit, out=u), args.steps)
            alone[part] = {k: t / c for k, (t, c) in st.items() if c and k not in ("pack", "unpack")}
        print("stages alone (ms per launch): %s" % json.dumps(alone), file=sys.stderr, flush=True)
    print(json.dumps({"workload": wl["name"], "value": N * nrhs / (ms * 1e-3), "unit": "observer points/s",
                      "ms_per_step": ms, "steps": args.steps, "N": N, "nrhs": nrhs, "dtype": wl["precision"],
                      "corr_nnz": info["corr_nnz"], "corr_layout_used": info["corr_layout_used"],
                      "corr_tile_values": info["corr_tile_values"], "plan_seconds": plan_s,
                      "rel_l2_vs_oracle_rows": acc,
                      "stages_ms": {k: t / c for k, (t, c) in stages.items() if c},
                      "stages_alone_ms": alone}), flush=True)
    plan.close()


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "hbm_traffic_near_correction_helmholtz_surface_100k.json")
CORR_SOURCES = ["paper_2312_02376_amd/csrc/kernels_sym.hip", "paper_2312_02376_amd/csrc/kernels_corr.hip"]


def corr_source_hash():
    import hashlib
    h = hashlib.sha256()
    for s in CORR_SOURCES:
        h.update(open(os.path.join(ROOT, s), "rb").read())
    return h.hexdigest()


def measured_traffic(nnz):
    """HBM bytes per apply of the near-zone correction kernels from the
    committed rocprofv3 FETCH_SIZE / WRITE_SIZE summary (scaled by a plain copy
    of known size), or None when that summary was taken on a different kernel
    source or workload."""
    try:
        rec = json.load(open(TRAFFIC_RECORD))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != corr_source_hash() or rec.get("corr_nnz") != nnz:
        return None
    return rec["traffic_bytes_per_launch"]


def correction_bytes(info, N, planes, amp_bytes=16):
    """Algorithmic bytes of one correction apply: every stored FP64 value once
    (box-pair blocks; CSR values with their int32 columns and int64 row
    pointers), the amplitudes once and the result once."""
    vb = info["corr_value_bytes"]
    b = info["corr_sym_values"] * vb
    if info["corr_csr_nnz"] > 0 or info["corr_layout_used"] == 1:
        b += info["corr_csr_nnz"] * (vb + 4) + (N + 1) * 8
    return b + 2 * N * planes * amp_bytes


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--corr-ball", type=float, default=WORKLOAD["corr_ball"],
                    help="radius of the ball correction region in near-grid spacings (0: the cube of 10 boxes)")
    ap.add_argument("--oracle-rows", type=int, default=24)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="helmholtz_100k",
                    choices=["helmholtz_100k", "multicell_48", "dynamic_cube_1m"] + sorted(SECONDARY))
    ap.add_argument("--target", type=float, default=1e-4, help="error target of the multi-cell parameter choice")
    ap.add_argument("--lanes", type=int, default=4, help="streams of the multi-cell batch")
    ap.add_argument("--no-batched", action="store_true", help="skip the nested 1M-point batched record")
    ap.add_argument("--isolated-parts", action="store_true",
                    help="secondary workloads: also time each part of the apply on its own")
    ap.add_argument("--no-forces", action="store_true", help="skip the nested 2M-point position-gradient record")
    ap.add_argument("--no-separate", action="store_true",
                    help="skip the timing of the step made of two single calls")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (scale for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: measures one GPU only; multi-GPU runs are not supported "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        nbytes = 1 << 30
        x = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "launches": 3}))
        return

    if args.workload == "multicell_48":
        print(json.dumps(multicell_record(args)), flush=True)
        return
    if args.workload == "dynamic_cube_1m":
        print(json.dumps(dynamic_cube_record(args)), flush=True)
        return
    if args.workload != "helmholtz_100k":
        run_secondary(args, args.workload)
        return

    from paper_2312_02376_amd import fftpim as fp
    from paper_2312_02376_amd import workloads as W

    fp.lib()  # fail loudly if the HIP library is not built
    wl = dict(WORKLOAD)
    wl["corr_ball"] = args.corr_ball
    N = wl["N"]
    src, q64 = W.helmholtz_surface_100k(N)
    q = q64.astype(np.complex128)
    v = W.gaussian_complex(1, N, 102)[0].astype(np.complex128)
    dev = torch.device("cuda:0")
    pos = torch.tensor(src, dtype=torch.float64, device=dev)
    t0 = time.perf_counter()
    plan = fp.Plan(pos, 2, list(wl["L"]), k0=wl["k0"], kt=wl["kt"], near_n=wl["near_n"],
                   near_order=wl["near_order"], corr_radius=wl["corr_radius"], far_n=wl["far_n"],
                   far_order=wl["far_order"], n_images=wl["n_images"], precision="f64",
                   value_type="complex", order="plan", nrhs_max=1, corr_ball=wl["corr_ball"])
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    info = plan.info()
    perm = plan.permutation().long()
    qd = torch.tensor(q, device=dev)[perm].contiguous()
    vd = torch.tensor(v, device=dev)[perm].contiguous()
    u = torch.empty_like(qd)
    w = torch.empty_like(vd)
    print("plan: %.2f s, correction nnz %d, device bytes %.2f GB" % (plan_s, info["corr_nnz"],
                                                                   info["device_bytes"] / 1e9),
          file=sys.stderr, flush=True)

    separate = None
    if not args.no_separate:
        # the same step as two single calls
        for _ in range(args.warmup):
            plan.apply(qd, out=u)
            plan.adjoint(vd, out=w)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            plan.apply(qd, out=u)
            plan.adjoint(vd, out=w)
        torch.cuda.synchronize()
        sep_ms = 1e3 * (time.perf_counter() - t0) / args.steps
        separate = {"ms_per_step": sep_ms, "value": N / (sep_ms * 1e-3),
                    "calls": "fftpim_apply + fftpim_apply_adjoint"}
        print("separate calls: %.3f ms per step" % sep_ms, file=sys.stderr, flush=True)

    def pair_step():
        plan.apply_pair(qd, vd, out_u=u, out_w=w)

    ms_per_step, ms_median = time_steps(pair_step, args.steps, args.warmup)
    if plan.last_status() != 0:
        raise RuntimeError("device-reported error during the timed applies")
    value = N * 1 / (ms_per_step * 1e-3)
    stages = staged_pass(plan, pair_step, args.steps)
    print("stages (ms per launch): " + ", ".join(
        "%s %.4f" % (k, t / c) for k, (t, c) in stages.items() if c), file=sys.stderr, flush=True)

    # dominant kernel: the FP64 near-zone correction (Sec. 3.3 Step 4), one
    # launch per step carrying both products (two planes in, two out)
    corr_ms, corr_calls = stages["near_corr"]
    corr_avg_s = corr_ms / max(corr_calls, 1) * 1e-3
    nnz = info["corr_nnz"]
    corr_bytes = correction_bytes(info, N, 2)
    kname = ("k_sym_apply + k_sym_gather (near-zone correction of A q and A^H v in one pass, FP64 complex "
             "box-pair blocks)" if info["corr_layout_used"] == 2
             else "k_corr_spmv (near-zone correction, FP64 complex CSR, A q then A^H v)")
    roofline = {
        "kernel": kname,
        "bound": "hbm",
        "achieved": corr_bytes / corr_avg_s / 1e9,
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": corr_bytes / corr_avg_s / 1e9 / HBM_PEAK_GBS,
        "traffic": measured_traffic(nnz),
        "bytes_per_launch": corr_bytes,
        "avg_launch_ms": corr_avg_s * 1e3,
    }

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "observer points/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "ms_per_step_median": ms_median,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": wl["name"],
            "N": N, "nrhs": 1, "periodicity": "2D (x, y)", "k0": wl["k0"], "kt": list(wl["kt"]),
            "near_grid": list(wl["near_n"]), "near_order": wl["near_order"],
            "corr_region": ("ball, radius %g near-grid spacings" % wl["corr_ball"]) if wl["corr_ball"] > 0
            else "cube, %d boxes" % wl["corr_radius"],
            "far_grid": list(wl["far_n"]), "far_order": wl["far_order"], "n_images": wl["n_images"],
            "corr_nnz": nnz, "plan_seconds": plan_s, "io_order": "plan",
        },
        "roofline": roofline,
        "step": "fftpim_apply_pair (A q and A^H v, both in full)",
        "separate_calls": separate,
        "stage_pass": "roofline launch times from a second pass of %d steps with stage events on" % args.steps,
    }

    if not args.no_cpu_baseline:
        from oracle import pgf as P
        from oracle.psp import host_workers, psp_adjoint, psp_forward
        lat = P.Lattice(2, list(wl["L"]), wl["k0"], list(wl["kt"]))
        rng = np.random.default_rng(2024)
        rows = np.sort(rng.choice(N, args.oracle_rows, replace=False))
        workers = host_workers()
        t0 = time.perf_counter()
        uref = psp_forward(lat, src, q, obs_index=rows, workers=workers)
        wref = psp_adjoint(lat, src, v, src_index=rows, workers=workers)
        cpu_s = time.perf_counter() - t0
        inv = torch.empty_like(perm)
        inv[perm] = torch.arange(N, device=dev)
        ipos = inv.cpu().numpy()[rows]
        ug = u.cpu().numpy()[ipos]
        wg = w.cpu().numpy()[ipos]
        e_fwd = float(np.linalg.norm(ug - uref) / np.linalg.norm(uref))
        e_adj = float(np.linalg.norm(wg - wref) / np.linalg.norm(wref))
        result["cpu_baseline"] = {
            "value": len(rows) / cpu_s,
            "unit": "observer points/s",
            "cores": workers,
            "cpu": cpu_model(),
            "kind": "oracle",
            "sample": "%d observers (forward) and %d sources (conjugate transpose) of the same workload, "
                      "direct FP64 pair sum over images (Ewald / Floquet series), %.1f s" % (len(rows), len(rows), cpu_s),
        }
        result["rel_l2_vs_oracle"] = {"forward": e_fwd, "adjoint": e_adj, "sample_rows": len(rows)}
    plan.close()
    if not args.no_batched:
        result["batched"] = batched_record(args)
    if not args.no_forces:
        result["forces"] = forces_record(args)
    print(json.dumps(result), flush=True)


def dynamic_cube_record(args):
    """The timing case of Sec. 4.2 (Fig. complex_real) at its largest size:
    10^6 points in a centred 100^3 cube of a period-101 cell, dynamic
    (k0 from a mean spacing of lambda/20, a period of about five wavelengths,
    phase wavenumbers 0.01 - 0.01j) and static (neutral real strengths), each
    at the relative errors 1e-3 and 1e-5 with parameters from
    fftpim_autotune; FP64, one step = one fftpim_apply.  The 1e-3 results
    are compared with the 1e-5 ones."""
    import numpy as np
    import torch

    from paper_2312_02376_amd import fftpim as fp
    from paper_2312_02376_amd import workloads as W
    fp.lib()
    dev = torch.device("cuda:0")
    N = 1_000_000
    src, qd = W.dynamic_cube(N, 9)
    qs = W.gaussian_neutral(1, N, 9)[0]
    k0 = W.dynamic_cube_k0(N)
    pos = torch.tensor(src, device=dev)
    out, results = {}, {}
    for case in ("dynamic", "static"):
        for target in (1e-3, 1e-5):
            kw_p = dict(k0=k0, kt=[0.01 - 0.01j] * 3) if case == "dynamic" else {}
            vt = "complex" if case == "dynamic" else "real"
            q = qd.astype(np.complex128) if case == "dynamic" else qs
            t0 = time.perf_counter()
            kw, rep = fp.autotune(pos, 3, [101.0] * 3, target, value_type=vt, **kw_p)
            t1 = time.perf_counter()
            plan = fp.Plan(pos, 3, [101.0] * 3, **kw_p, **kw)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            x = torch.tensor(q, device=dev)
            u = torch.empty_like(x)
            ms, med = time_steps(lambda: plan.apply(x, out=u), max(3, args.steps // 4), 1)
            plan.apply(x, out=u)
            results[(case, target)] = u.cpu().numpy()
            if plan.last_status() != 0:
                raise RuntimeError("device-reported error in the dynamic-cube apply")
            inf = plan.info()
            out["%s_%g" % (case, target)] = {
                "ms_per_apply": ms, "ms_median": med, "plan_seconds": t2 - t1, "tune_seconds": t1 - t0,
                "near_n": list(kw["near_n"]), "near_order": kw["near_order"], "corr_ball": round(kw["corr_ball"], 2),
                "far_n": list(kw["far_n"]), "far_order": kw["far_order"], "far_fft": inf["far_fft"],
                "corr_nnz": inf["corr_nnz"], "predicted_rel_err": rep["predicted_rel_err"]}
            print(case, target, json.dumps(out["%s_%g" % (case, target)]), flush=True)
            plan.close()
            del x, u
            torch.cuda.empty_cache()
    rec = {"metric": "ms per apply", "unit": "ms", "workload": "dynamic and static 3D-periodic cube, 1M points, "
           "period 101 (about 5 wavelengths), FP64", "k0": k0, "results": out,
           "dynamic_over_static": {"1e-3": out["dynamic_0.001"]["ms_per_apply"] / out["static_0.001"]["ms_per_apply"],
                                   "1e-5": out["dynamic_1e-05"]["ms_per_apply"] / out["static_1e-05"]["ms_per_apply"]},
           # the exact sum at 10^6 points is out of the oracle's reach (its
           # Ewald sums at this k0 L take hours per row set); the 1e-3
           # results are checked against the 1e-5 ones instead, and both
           # parameter rules against the exact sum at 20,000 points in
           # the tests
           "rel_diff_1e-3_vs_1e-5": {c: float(np.linalg.norm(results[(c, 1e-3)] - results[(c, 1e-5)]) /
                                              np.linalg.norm(results[(c, 1e-5)])) for c in ("dynamic", "static")}}
    return rec


def multicell_record(args):
    """48 independent cells (N log-uniform in [5e3, 5e5], 5.9M points in all;
    1D, 2D and 3D periodicity; static and Helmholtz; Gaussian blobs; complex
    strengths): parameters per cell from fftpim_autotune for the error target
    in FP32 (FP64 correction), one step = one fftpim_batch_apply over all
    cells; also timed as one lane (cells in turn) and as separate applies."""
    import numpy as np
    import torch

    from paper_2312_02376_amd import fftpim as fp
    from paper_2312_02376_amd import workloads as W
    fp.lib()
    dev = torch.device("cuda:0")
    cells = W.multi_cell(48, 4)
    plans, ins, tune_s, plan_s, preds, infos = [], [], 0.0, 0.0, [], []
    for c, cell in enumerate(cells):
        pos = torch.tensor(cell["pos"], device=dev)
        t0 = time.perf_counter()
        kw, rep = fp.autotune(pos, cell["dims"], cell["L"], args.target, k0=cell["k0"], kt=cell["kt"],
                              precision="f32")
        t1 = time.perf_counter()
        plan = fp.Plan(pos, cell["dims"], cell["L"], k0=cell["k0"], kt=cell["kt"], order="plan", **kw)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        tune_s += t1 - t0
        plan_s += t2 - t1
        perm = plan.permutation().long()
        ins.append(torch.tensor(cell["q"], dtype=torch.complex64, device=dev)[perm].contiguous())
        plans.append(plan)
        preds.append(rep)
        inf = plan.info()
        infos.append(dict(N=len(cell["q"]), dims=cell["dims"], k0=cell["k0"], near_n=list(kw["near_n"]),
                          q=kw["near_order"], corr_ball=round(kw["corr_ball"], 2), far_n=list(kw["far_n"]),
                          far_order=kw["far_order"], corr_nnz=inf["corr_nnz"],
                          predicted_rel_err=rep["predicted_rel_err"]))
        print("cell %d N %d dims %d k0 %.2f tuned in %.2fs planned in %.2fs" %
              (c, len(cell["q"]), cell["dims"], cell["k0"], t1 - t0, t2 - t1), flush=True)
    outs = [torch.empty_like(x) for x in ins]
    Ntot = sum(len(c["q"]) for c in cells)

    def timed(fn, steps, warm):
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    steps = max(3, args.steps // 4)
    batch = fp.Batch(plans, lanes=args.lanes)
    ms = timed(lambda: batch.apply(ins, outs), steps, 1)
    one = fp.Batch(plans, lanes=1)
    ms_one = timed(lambda: one.apply(ins, outs), steps, 1)
    ms_sep = timed(lambda: [p.apply(x, out=o) for p, x, o in zip(plans, ins, outs)], steps, 1)
    batch.apply(ins, outs)
    torch.cuda.synchronize()
    # accuracy on the stored exact rows (plan order: the row's position in
    # the plan's permutation)
    errs = []
    gpath = os.path.join(ROOT, "tests", "golden", "multi_cell_48_rows.txt")
    if os.path.exists(gpath):
        g = np.loadtxt(gpath)
        for c, plan in enumerate(plans):
            sel = g[:, 0] == c
            rows = g[sel, 1].astype(np.int64)
            inv = torch.empty_like(plan.permutation().long())
            perm = plan.permutation().long()
            inv[perm] = torch.arange(len(perm), device=dev)
            u = outs[c][inv[torch.tensor(rows, device=dev)]].cpu().numpy()
            ex = g[sel, 2] + 1j * g[sel, 3]
            errs.append(float(np.linalg.norm(u - ex) / np.linalg.norm(ex)))
    for p in plans:
        if p.last_status() != 0:
            raise RuntimeError("device-reported error in the multi-cell batch")
    rec = {"metric": "observer points/s per multi-cell apply", "value": Ntot / (ms * 1e-3),
           "unit": "observer points/s", "n_gpus": 1, "steps": steps, "warmup": 1, "ms_per_step": ms,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32 (FP64 correction)",
           "data": "synthetic",
           "config": {"workload": "48 independent cells, N log-uniform in [5e3, 5e5] (%d points), mixed 1D/2D/3D "
                                  "periodicity, static and Helmholtz, Gaussian blobs, complex strengths" % Ntot,
                      "target_rel_err": args.target, "lanes": args.lanes},
           "ms_one_lane": ms_one, "ms_separate_applies": ms_sep, "tune_seconds": tune_s, "plan_seconds": plan_s,
           "max_predicted_rel_err": max(r["predicted_rel_err"] for r in preds),
           "rel_err_vs_oracle_rows": {"max": max(errs), "median": float(np.median(errs)), "cells": len(errs),
                                      "rows_per_cell": 4} if errs else None,
           "cells": infos}
    batch.close()
    one.close()
    for p in plans:
        p.close()
    return rec


def forces_record(args):
    """Potential and position gradient of a 3D-periodic Coulomb cell with 2M
    uniform points and one neutral Gaussian right-hand side (FP32 bulk, FP64
    correction): one step = u = A q and dL/dr for L = q . (A q) (twice the
    electrostatic energy; the forces are -dL/dr / 2)."""
    import numpy as np
    import torch

    from paper_2312_02376_amd import fftpim as fp
    from paper_2312_02376_amd import workloads as W
    dev = torch.device("cuda:0")
    N = 2_000_000
    src = W.uniform_cube(N, 5)
    q = W.gaussian_neutral(1, N, 5, np.float32)[0]
    t0 = time.perf_counter()
    plan = fp.Plan(torch.tensor(src, device=dev), 3, [1.0, 1.0, 1.0], near_n=(128, 128, 128), near_order=4,
                   corr_radius=5, far_n=(14, 14, 14), far_order=5, precision="f32", value_type="real", order="plan")
    torch.cuda.synchronize()
    plan_s = time.perf_counter() - t0
    perm = plan.permutation().long()
    qd = torch.tensor(q, device=dev)[perm].contiguous()
    u = torch.empty_like(qd)
    g = torch.empty((N, 3), dtype=torch.float64, device=dev)

    def step():
        plan.apply(qd, out=u)
        plan.grad_positions(qd, qd, out=g)

    steps = 3
    ms, med = time_steps(step, steps, 1)
    apply_ms, _ = time_steps(lambda: plan.apply(qd, out=u), steps, 1)
    if plan.last_status() != 0:
        raise RuntimeError("device-reported error during the force steps")
    info = plan.info()
    rec = {"workload": "3D-periodic Coulomb, 2M uniform points, one neutral Gaussian right-hand side, FP32 bulk "
                       "with FP64 correction: potential and position gradient",
           "value": N / (ms * 1e-3), "unit": "points/s (potential and forces)", "ms_per_step": ms,
           "ms_per_step_median": med, "apply_ms": apply_ms, "gradient_ms": ms - apply_ms, "steps": steps, "N": N,
           "corr_nnz": info["corr_nnz"], "plan_seconds": plan_s,
           "step": "fftpim_apply + fftpim_grad_positions"}
    plan.close()
    del qd, u, g
    torch.cuda.empty_cache()
    return rec


def near_kernels_alone(plan, info, wl, qd, u, N, nrhs, steps):
    """The projection, FFT convolution and interpolation of one forward apply
    with no concurrent streams: launch time (HIP events) and algorithmic
    bytes of each, against the 8 TB/s HBM peak.  Bytes: the projection and
    the interpolation read every point's 1D weights (3 (q+1) doubles), its
    box (3 ints) and its P planes once and write (read) every grid node's P
    planes once; the FFT counts each of its five pruned passes reading its
    input and writing its output once, plus the spectrum."""
    P = (nrhs + 1) // 2 if wl["value_type"] == "real" else nrhs
    eb = 8 if wl["precision"] != "f64" else 16  # bytes of one complex plane value
    n0, n1, n2 = info["near_n"]
    M0, M1, M2 = info["near_fft"]
    q = wl["near_order"]
    pts = N * (3 * (q + 1) * 8 + 12 + P * eb)
    grid = n0 * n1 * n2 * P * eb
    fft = P * eb * (2 * (n0 * n1 * n2 + n0 * n1 * M2) + 2 * (n0 * n1 * M2 + n0 * M1 * M2) + 2 * n0 * M1 * M2) \
        + M0 * M1 * M2 * eb
    plan.apply_parts(qd, 1, out=u)
    st = staged_pass(plan, lambda: plan.apply_parts(qd, 1, out=u), steps)
    out = {}
    for name, stage, nbytes in (("projection", "near_spread", pts + grid), ("fft_convolution", "near_fft", fft),
                                ("interpolation", "near_interp", pts + grid)):
        t, c = st[stage]
        ms = t / max(c, 1)
        out[name] = {"ms": ms, "algorithmic_GB": nbytes / 1e9, "GB_s": nbytes / (ms * 1e-3) / 1e9,
                     "frac_hbm_peak": nbytes / (ms * 1e-3) / 8e12}
    return out


def batched_record(args):
    """The 1M-point, 64-right-hand-side Coulomb cell (FP32 bulk, FP64
    correction), one step = fftpim_apply_pair over all right-hand sides, and
    the same cell with one FP64 right-hand side; errors on the stored exact
    rows."""
    import numpy as np
    import torch

    from paper_2312_02376_amd import fftpim as fp
    from paper_2312_02376_amd import workloads as W
    dev = torch.device("cuda:0")
    src, q = W.coulomb_cube_1m_batched()
    N = src.shape[0]
    gold = np.loadtxt(GOLD_1M) if os.path.exists(GOLD_1M) else None
    out = {}
    for key in ("coulomb_1m_batched", "coulomb_1m_single_f64"):
        wl = SECONDARY[key]
        qq = q if wl["nrhs"] > 1 else q[:1].astype(np.float64)
        nrhs = qq.shape[0]
        t0 = time.perf_counter()
        plan = fp.Plan(torch.tensor(src, device=dev), 3, [1.0, 1.0, 1.0], near_n=wl["near_n"],
                       near_order=wl["near_order"], corr_radius=wl["corr_radius"], far_n=wl["far_n"],
                       far_order=wl["far_order"], n_images=1, precision=wl["precision"],
                       value_type=wl["value_type"], order="plan", nrhs_max=nrhs)
        torch.cuda.synchronize()
        plan_s = time.perf_counter() - t0
        info = plan.info()
        perm = plan.permutation().long()
        qd = torch.tensor(qq, device=dev)[:, perm].contiguous()
        vd = torch.roll(qd, 1, dims=0).contiguous() if nrhs > 1 else (-qd).contiguous()
        u, w = torch.empty_like(qd), torch.empty_like(vd)

        def step():
            plan.apply_pair(qd, vd, out_u=u, out_w=w)

        steps = max(5, args.steps // 2)
        ms, med = time_steps(step, steps, 2)
        if plan.last_status() != 0:
            raise RuntimeError("device-reported error during the batched applies")
        rec = {"workload": wl["name"], "value": N * nrhs / (ms * 1e-3), "unit": "observer points/s",
               "ms_per_step": ms, "ms_per_step_median": med, "steps": steps, "N": N, "nrhs": nrhs,
               "dtype": "f32 (FP64 correction)" if wl["precision"] == "f32" else "f64",
               "corr_layout_used": info["corr_layout_used"], "corr_tile_values": info["corr_tile_values"],
               "plan_seconds": plan_s, "step": "fftpim_apply_pair over all right-hand sides"}
        if gold is not None:
            rows = np.unique(gold[:, 0].astype(np.int64))
            g = gold[:, 2].reshape(len(rows), -1).T[:nrhs]
            inv = torch.empty_like(perm)
            inv[perm] = torch.arange(N, device=dev)
            got = u[:, inv[torch.tensor(rows, device=dev)]].double().cpu().numpy()
            rec["rel_l2_vs_oracle_rows"] = float(np.linalg.norm(got - g) / np.linalg.norm(g))
            rec["max_rel_elem_vs_oracle_rows"] = float(np.abs(got - g).max() / np.abs(g).max())
            rec["oracle_rows"] = int(len(rows))
        if key == "coulomb_1m_batched":
            stages = staged_pass(plan, step, steps)
            rec["stages_ms"] = {k: t / c for k, (t, c) in stages.items() if c}
            # dominant kernel: the dense FP64 correction tiles on the matrix
            # cores, two launches (A q, A^H v) inside the correction stage
            corr_ms, calls = stages["near_corr"]
            launch_s = corr_ms / max(calls, 1) / 2 * 1e-3
            flops = 2.0 * info["corr_tile_values"] * nrhs
            tbytes = info["corr_tile_values"] * 8.0
            rec["roofline"] = {"kernel": "k_corr_tile (FP64 MFMA 16x16x4, dense 16-observer tiles)",
                               "bound": "mfma", "achieved": flops / launch_s / 1e12, "peak": 78.6,
                               "unit": "TFLOP/s", "frac": flops / launch_s / 1e12 / 78.6, "traffic": None,
                               "flops_per_launch": flops, "avg_launch_ms": launch_s * 1e3,
                               "hbm_GBps_stored_values": tbytes / launch_s / 1e9}
            rec["near_kernels_alone"] = near_kernels_alone(plan, info, wl, qd, u, N, nrhs, steps)
        out[key] = rec
        plan.close()
        del qd, vd, u, w
        torch.cuda.empty_cache()
    b, s1 = out["coulomb_1m_batched"], out["coulomb_1m_single_f64"]
    b["single_rhs_f64"] = s1
    b["batched_over_single_per_rhs"] = b["value"] / s1["value"]
    return b


if __name__ == "__main__":
    main()
