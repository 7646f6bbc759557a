"""Benchmark: LOBPCG iterations/s of the HIP path on one MI355X.

Workload (default): the 64-atom diamond-like cell -- 2x2x2 conventional
diamond supercell, L = 13.48 bohr, 48^3 grid, 160 bands (128 tracked),
Gaussian local potential and s+p Gaussian Kleinman-Bylander projectors,
complex128 throughout, Teter-Payne-Allan preconditioner.  Inputs are seeded
and synthetic.  A step is one full LOBPCG iteration: residual and
preconditioner, block orthonormalisation, H-apply (batched 3D FFT, local and
nonlocal terms), Gram GEMMs, Cholesky + two triangular solves + Hermitian
eigensolve + back-transform, rotation GEMMs.

Prints ONE JSON line.  Extra legs: time to 1e-6 Ha (fresh solve from the
initial block against the stored oracle eigenvalues) and the CPU oracle
timed on the host for one LOBPCG iteration of the same cell.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time to 1e-6 Ha eigenpairs & LOBPCG iter/s: FP64 vs mixed+learned precond"
WORKLOADS = {
    "C1": "diamond 8-atom cell, L=6.74 bohr, 16^3 grid, 16 bands, local potential only",
    "C2": "diamond-like 2x2x2 supercell, 64 atoms, L=13.48 bohr, 48^3 grid, 160 bands, s+p KB projectors",
    "C3": "diamond-like 3x3x3 supercell, 216 atoms, L=20.22 bohr, 96^3 grid, 480 bands, s+p KB projectors",
    "C4": "bcc 4x4x4 supercell, 128 atoms, L=23.92 bohr, 112^3 grid, 960 bands, s+p+d KB projectors",
}
# HBM bytes per launch of a kernel family, from FETCH_SIZE and WRITE_SIZE
# counter runs scaled by a known-size copy (the per-dispatch table and the
# commands are in profiles/hbm_traffic_fp64_c2.md).  A value holds only
# while the kernel source it was measured on is unchanged (sha256 below).
MEASURED_TRAFFIC = {
    ("C2", "fp64", "gram"): (2.6337e9, "paper_2512_04447_amd/csrc/gemm.hip",
                             "ca2ed848dd0136ad8d302c7494b9380d81e4ee92cc048422c78d4ddac899512a"),
}
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFS = 78.6
FP32_PEAK_TFS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="C2")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="fp64 (the default workload) or mixed (complex64 blocks, FP32 products)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-tta", action="store_true")
    ap.add_argument("--compare", default=None,
                    help="time-to-1e-6-Ha comparison on one cell (C2, C3 or C4) instead of the throughput bench")
    ap.add_argument("--mixed-lock", type=float, default=1e-4)
    ap.add_argument("--weights", default=None, help="FP32 parameters of the learned preconditioner on r (.npy)")
    ap.add_argument("--weights-tpa", default=None, help="FP32 parameters of the residual network on TPA(r) (.npy)")
    ap.add_argument("--maxit", type=int, default=150)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MB",
                    help="first run one plain device-to-device copy of MB megabytes (a known-size dispatch for "
                         "scaling hardware byte counters)")
    return ap.parse_args()


def compare(args):
    """Time to 1e-6 Ha from the same initial block: FP64 + TPA (the plain
    path, run to residual 1e-8; its final Ritz values are the reference),
    then the mixed-precision path with TPA and with the trained network.
    The FP64 run's own time to 1e-6 Ha is read from its history."""
    import torch

    import ksinputs as ki
    from paper_2512_04447_amd import binding as b
    from paper_2512_04447_amd import learned as lr

    cfg = ki.config(args.compare)
    cell = ki.make_cell(cfg)
    t0 = time.perf_counter()
    X0 = ki.make_x0(cfg)
    log(f"[compare] {cfg.name}: n={cfg.n} nb={cfg.nb} ntrack={cfg.ntrack} X0 in {time.perf_counter() - t0:.1f}s")
    proj = b.ProjectorArrays.from_cell(cell) if cell.nproj else None
    x0 = torch.from_numpy(X0).cuda()
    del X0
    out = {}

    def leg(name, prec, pc, lock, ref=None, res_tol=0.0, params=None):
        plan = b.Plan(cell.n, cell.L, proj, cfg.nb, prec)
        dt = torch.float64 if prec == b.KS_FP64 else torch.float32
        v = torch.from_numpy(cell.V).to(dt).cuda()
        xs = x0 if prec == b.KS_FP64 else x0.to(torch.complex64)
        r = lr.run_to_tolerance(plan, v, xs, cfg.ntrack, pc, lock, args.maxit, ref=ref, res_tol=res_tol,
                                cnn_params=params, log=log)
        lob = r.pop("lobpcg")
        th = lob.theta[: cfg.ntrack].cpu().numpy()
        hist = r.pop("history")
        log(f"[compare] {name}: {r['iterations']} iterations, {r['seconds']:.2f}s, max res {r['max_res']:.2e}")
        r["max_res_history"] = [float(f"{h[1]:.3e}") for h in hist]
        del lob, xs, v
        torch.cuda.empty_cache()
        return r, hist, th

    r64, h64, ref = leg("fp64+tpa", b.KS_FP64, b.KS_PRECOND_TPA, 0.1 * cfg.res_tol, res_tol=cfg.res_tol)
    # FP64's own time to 1e-6 Ha against its converged values
    first = next((i for i, h in enumerate(h64) if np.abs(h[3] - ref).max() <= 1e-6), len(h64) - 1)
    out["fp64_tpa"] = {"seconds_to_1e-6_Ha": round(h64[first][0], 3), "iterations_to_1e-6_Ha": first + 1,
                       "converged_iterations": r64["iterations"], "final_max_res": r64["max_res"],
                       "s_per_iter": round(r64["seconds"] / r64["iterations"], 4),
                       "max_res_history": r64["max_res_history"]}
    rm, hm, thm = leg("mixed+tpa", b.KS_MIXED_FP32, b.KS_PRECOND_TPA, args.mixed_lock, ref=ref)
    out["mixed_tpa"] = {"seconds_to_1e-6_Ha": round(rm["seconds"], 3), "iterations_to_1e-6_Ha": rm["iterations"],
                        "max_err_Ha": rm["max_err"], "s_per_iter": round(rm["seconds"] / rm["iterations"], 4),
                        "reached": bool(rm["max_err"] <= 1e-6), "max_res_history": rm["max_res_history"]}
    for key, kind, wpath in (("mixed_cnn", b.KS_PRECOND_CNN, args.weights or lr.WEIGHTS),
                             ("mixed_cnn_tpa", b.KS_PRECOND_CNN_TPA, args.weights_tpa or lr.WEIGHTS_TPA)):
        if not os.path.exists(wpath):
            continue
        params = torch.from_numpy(np.load(wpath)).cuda()
        rc, hc, thc = leg(key.replace("_", "+", 1), b.KS_MIXED_FP32, kind, args.mixed_lock, ref=ref, params=params)
        out[key] = {"seconds_to_1e-6_Ha": round(rc["seconds"], 3), "iterations_to_1e-6_Ha": rc["iterations"],
                    "max_err_Ha": rc["max_err"], "s_per_iter": round(rc["seconds"] / rc["iterations"], 4),
                    "reached": bool(rc["max_err"] <= 1e-6), "switched_to_tpa_at": rc["switched_to_tpa_at"],
                    "max_res_history": rc["max_res_history"]}
    print(json.dumps({"metric": METRIC, "compare": cfg.name, "n_gpus": 1, "data": "synthetic",
                      "config": {"workload": cfg.name, "Ng": cfg.Ng, "bands": cfg.nb, "tracked": cfg.ntrack},
                      "legs": out}))


def measured_traffic(cfg_name, precision, family):
    """Counter-measured bytes per launch, or None when not measured or when
    the kernel source has changed since."""
    import hashlib

    ent = MEASURED_TRAFFIC.get((cfg_name, precision, family))
    if ent is None:
        return None
    value, src, digest = ent
    try:
        with open(os.path.join(ROOT, src), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != digest:
                return None
    except OSError:
        return None
    return value


def family_work(cfg, es):
    """Algorithmic flops / bytes per step for each kernel family; es is the
    bytes of one complex element of the blocks (16 FP64, 8 mixed)."""
    Ng, nb = cfg.Ng, cfg.nb
    m = 3 * nb
    blk = Ng * nb * es
    n_h = 3  # H-applies per step: W, P and the new X
    # mixed path: re-orthonormalisation of X (one more self-Gram and rotation)
    extra = 1 if es == 8 else 0
    return {
        # Hermitian triangles of the W and P self-Grams (S only) and of the
        # basis Gram (S and H); the full X^H W of the projection W - X X^H W
        "gram_flops": 8 * Ng * (nb * (nb + 1) / 2 * (2 + extra) + nb * nb + 2 * m * (m + 1) / 2),
        # W and P orthonormalising rotations, the projection update, and one
        # pass over V giving X' = V C and P' = V[:, nb:] C[nb:]
        "rotate_flops": 8 * Ng * (nb * nb * (3 + extra) + m * nb + 2 * nb * nb),
        # pass A: kinetic-energy FFT of X (R+W), residual (2R+W), H-applies (R+W)
        "pass_a_bytes": blk * (2 + 3 + 2 * n_h),
        # pass B: kinetic reduction (R), TPA (R+W), kinetic (R+W) per H-apply
        "pass_b_bytes": blk * (1 + 2 + 2 * n_h),
        # pass C: TPA (R+W), H (tmp R + psi R + W) per H-apply
        "pass_c_bytes": blk * (2 + 3 * n_h),
    }


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus above 1 is not supported",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch

    import ksinputs as ki
    from paper_2512_04447_amd import binding as b

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy > 0:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {nbytes} bytes read and {nbytes} bytes written")
        del src, dst
    if args.compare:
        compare(args)
        return
    cfg = ki.config(args.config)
    cell = ki.make_cell(cfg)
    X0 = ki.make_x0(cfg)
    log(f"[bench] {cfg.name}: n={cfg.n} nb={cfg.nb} atoms={cell.natoms} nproj={cell.nproj}")
    mixed = args.precision == "mixed"
    plan = b.Plan(cell.n, cell.L, b.ProjectorArrays.from_cell(cell) if cell.nproj else None, cfg.nb,
                  b.KS_MIXED_FP32 if mixed else b.KS_FP64)
    v = torch.from_numpy(cell.V).cuda()
    x0 = torch.from_numpy(X0).cuda()
    if cfg.name not in ("C1", "C2"):
        del X0  # large cells: the host copy is not needed again
    if mixed:
        v, x0 = v.float(), x0.to(torch.complex64)
    lob = b.Lobpcg(plan, v, x0)
    lob.init()
    tol = cfg.res_tol
    for _ in range(args.warmup):
        lob.step(b.KS_PRECOND_TPA, 0.1 * tol)
    torch.cuda.synchronize()
    fams = [b.KF_GRAM, b.KF_ROTATE, b.KF_PASS_A, b.KF_PASS_B, b.KF_PASS_C, b.KF_NL_PROJECT, b.KF_HEGV, b.KF_ZGEMM]
    names = ["gram", "rotate", "pass_a", "pass_b", "pass_c", "nl_project", "hegv", "zgemm"]
    # timed region without event instrumentation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lob.step(b.KS_PRECOND_TPA, 0.1 * tol)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    log(f"[bench] {args.steps} steps in {wall:.3f}s")
    # same number of steps again with HIP events around each kernel family
    for f in fams:
        b.kernel_timer(True, f)
    for _ in range(args.steps):
        lob.step(b.KS_PRECOND_TPA, 0.1 * tol)
    torch.cuda.synchronize()
    fam_ms = {}
    for f, nm in zip(fams, names):
        ms, n = b.kernel_timer_read(f)
        b.kernel_timer(False, f)
        fam_ms[nm] = (ms / args.steps, n / args.steps)
    log("[bench] per-step ms by family: " + ", ".join(f"{k}={v[0]:.3f} ({v[1]:.0f} launches)" for k, v in fam_ms.items()))
    work = family_work(cfg, 8 if mixed else 16)
    mma_peak = FP32_PEAK_TFS if mixed else FP64_PEAK_TFS
    rates = {
        "gram": ("mfma", work["gram_flops"] / 1e12 / (fam_ms["gram"][0] / 1e3), mma_peak, "TFLOP/s",
                 work["gram_flops"] / max(fam_ms["gram"][1], 1)),
        "rotate": ("mfma", work["rotate_flops"] / 1e12 / (fam_ms["rotate"][0] / 1e3), mma_peak, "TFLOP/s",
                   work["rotate_flops"] / max(fam_ms["rotate"][1], 1)),
        "pass_a": ("hbm", work["pass_a_bytes"] / 1e9 / (fam_ms["pass_a"][0] / 1e3), HBM_PEAK_GBS, "GB/s",
                   work["pass_a_bytes"] / max(fam_ms["pass_a"][1], 1)),
        "pass_b": ("hbm", work["pass_b_bytes"] / 1e9 / (fam_ms["pass_b"][0] / 1e3), HBM_PEAK_GBS, "GB/s",
                   work["pass_b_bytes"] / max(fam_ms["pass_b"][1], 1)),
        "pass_c": ("hbm", work["pass_c_bytes"] / 1e9 / (fam_ms["pass_c"][0] / 1e3), HBM_PEAK_GBS, "GB/s",
                   work["pass_c_bytes"] / max(fam_ms["pass_c"][1], 1)),
    }
    dom = max(rates, key=lambda k: fam_ms[k][0])
    bound, ach, peak, unit, per_launch = rates[dom]
    roofline = {"kernel": dom, "bound": bound, "achieved": round(ach, 3), "peak": peak, "unit": unit,
                "frac": round(ach / peak, 4), "traffic": measured_traffic(cfg.name, args.precision, dom),
                "algorithmic_per_launch": per_launch,
                "avg_launch_ms": fam_ms[dom][0] / max(fam_ms[dom][1], 1)}
    others = {k: {"achieved": round(r[1], 3), "unit": r[3], "frac": round(r[1] / r[2], 4),
                  "ms_per_step": round(fam_ms[k][0], 4)} for k, r in rates.items()}
    others["hegv"] = {"ms_per_step": round(fam_ms["hegv"][0], 4)}
    others["nl_project"] = {"ms_per_step": round(fam_ms["nl_project"][0], 4)}

    # time to 1e-6 Ha against the stored oracle eigenvalues
    tta = None
    ref_path = os.path.join(ROOT, "tests", "golden", "c2_eigenvalues.txt")
    if not args.no_tta and cfg.name == "C2" and os.path.exists(ref_path):
        ref = np.loadtxt(ref_path, comments="#", usecols=1)[: cfg.ntrack]
        lob2 = b.Lobpcg(plan, v, x0)
        torch.cuda.synchronize()
        s0 = time.perf_counter()
        lob2.init()
        it = 0
        while it < 200:
            lob2.step(b.KS_PRECOND_TPA, 0.1 * tol)
            it += 1
            th = lob2.theta_host[: cfg.ntrack]
            if np.abs(th - ref).max() <= 1e-6:
                break
        torch.cuda.synchronize()
        tta = {"seconds": round(time.perf_counter() - s0, 4), "iterations": it,
               "max_abs_err_Ha": float(np.abs(th - ref).max())}
        log(f"[bench] time to 1e-6 Ha: {tta}")

    cpu = None
    # the oracle step is timed on the FP64 workloads small enough for it
    if not args.no_cpu_baseline and not mixed and cfg.name in ("C1", "C2"):
        from oracle import hamiltonian as oh
        from oracle import lobpcg as olob

        cores = len(os.sched_getaffinity(0))
        oc = oh.oracle_cell(cfg, cell.D)
        st = olob.initial_state(oc, X0)
        pc = olob.tpa_preconditioner(oc)
        c0 = time.perf_counter()
        olob.step(oc, st, pc, 0.1 * tol)
        dt = time.perf_counter() - c0
        cpu = {"value": round(1.0 / dt, 5), "unit": "LOBPCG iter/s", "cores": cores, "kind": "oracle",
               "sample": f"one oracle LOBPCG iteration on the same cell after its initialisation ({dt:.1f} s)"}
        log(f"[bench] cpu oracle: {dt:.2f}s per iteration on {cores} cores")

    out = {
        "metric": METRIC,
        "value": round(args.steps / wall, 4),
        "unit": "LOBPCG iter/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * wall / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOADS.get(cfg.name, cfg.name) + (", complex64 blocks, FP32 products, FP64 subspace solve"
                                                                   if mixed else ", complex128")
                               + ", TPA preconditioner",
                   "Ng": cfg.Ng, "bands": cfg.nb, "precision": args.precision},
        "roofline": roofline,
        "kernels": others,
        "time_to_1e-6_Ha": tta,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
