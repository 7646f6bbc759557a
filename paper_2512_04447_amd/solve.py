"""Drivers around lobpcg_step: a run to a tolerance, the time-to-tolerance
criterion (eigenvalues and subspace angles), and the mixed-precision run
finished by FP64 refinement.

Orchestration only.  Every arithmetic step runs in libksh.so, the angle
check included (ks_subspace_sin); the one conversion done here is the
exact widening of a complex64 block to complex128 when a mixed-precision
run hands its block over to the FP64 plan (a type change without rounding).
Each LOBPCG iteration costs one device-to-host copy (theta, res, status).

The time-to-tolerance criterion: the first iteration at which every tracked
|theta_i - lambda_i| <= tol_ha and the sine of the largest principal angle
between the first k Ritz vectors and the reference's is <= tol_angle, with k
the largest cut at or below the tracked count where the reference spectrum
has a gap above 1e-3 Ha (subspaces split inside a near-degenerate cluster
are not comparable).  The angle check's own time is excluded from the
reported wall time.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import binding as b


def angle_cut(ref_all: np.ndarray, ntrack: int, gap: float = 1e-3) -> int:
    """Largest k <= ntrack with ref[k] - ref[k-1] > gap (ref ascending,
    more entries than ntrack); 0 when there is none."""
    for k in range(min(ntrack, len(ref_all) - 1), 0, -1):
        if ref_all[k] - ref_all[k - 1] > gap:
            return k
    return 0


@dataclass
class Criterion:
    """Reference eigenvalues (tracked) and Ritz vectors (first k, FP64
    device rows) for the time-to-tolerance test."""

    ref_theta: np.ndarray
    ref_X: Optional[object]  # torch complex128 (k, Ng) or None (eigenvalues only)
    plan64: Optional[object]
    k: int
    tol_ha: float = 1e-6
    tol_angle: float = 1e-5
    last_sin: Optional[float] = None
    check_seconds: float = 0.0

    def eigen_ok(self, th: np.ndarray) -> bool:
        return float(np.abs(th - self.ref_theta).max()) <= self.tol_ha

    def angle_ok(self, lob) -> bool:
        """Needs an FP64 run (the reference subspace is FP64)."""
        if self.ref_X is None or self.k == 0:
            return True
        import torch

        if lob.plan.precision != b.KS_FP64:
            return False
        t0 = time.perf_counter()
        out = b.ks_subspace_sin(self.plan64, self.ref_X, lob.X, self.k)
        self.last_sin = float(out.item())
        self.check_seconds += time.perf_counter() - t0
        return self.last_sin <= self.tol_angle


@dataclass
class Run:
    lob: object
    history: list = field(default_factory=list)  # (seconds, max res, max err, theta, sin or None)
    iterations: int = 0
    reached: bool = False
    switched_to_tpa_at: Optional[int] = None


def iterate(run: Run, ntrack: int, precond: int, lock_tol: float, maxit: int, t0: float, crit: Criterion = None,
            res_tol: float = 0.0, cnn_params=None, switch_to_tpa: bool = True, stall_exit: bool = False,
            exit_res: float = 0.0, log=print) -> str:
    """Steps an initialised run; returns why it stopped: "criterion",
    "res_tol", "stall" (stall_exit and no 10% drop of the max tracked
    residual over 3 iterations), "exit_res" (max tracked residual <=
    exit_res) or "maxit".  Times are relative to t0 minus the criterion's
    check time."""
    lob = run.lob
    pc = precond
    for _ in range(maxit):
        learned = pc in (b.KS_PRECOND_CNN, b.KS_PRECOND_CNN_TPA)
        lob.step(pc, lock_tol, cnn_params if learned else None)
        run.iterations += 1
        it = run.iterations
        th, res = lob.theta_host[:ntrack], lob.res_host[:ntrack]
        status = lob.status_host
        if status[b.KS_ST_FLAGS] & (b.KS_FLAG_SOLVE_FAILED | b.KS_FLAG_NONFINITE):
            raise b.KsError(f"LOBPCG step {it} failed: status {status.tolist()}")
        rmax = float(res.max())
        err = float(np.abs(th - crit.ref_theta).max()) if crit is not None else None
        sin = None
        done = False
        if crit is not None and crit.eigen_ok(th):
            done = crit.angle_ok(lob)
            sin = crit.last_sin
        elapsed = time.perf_counter() - t0 - (crit.check_seconds if crit is not None else 0.0)
        run.history.append((elapsed, rmax, err, th.copy(), sin))
        if it % 5 == 0 or done:
            log(f"[solve] iteration {it}: max res {rmax:.3e}" + (f", max err {err:.3e}" if err is not None else "")
                + (f", sin {sin:.2e}" if sin is not None else "") + f", {elapsed:.2f}s")
        if done:
            run.reached = True
            return "criterion"
        if res_tol > 0.0 and rmax <= res_tol:
            return "res_tol"
        if exit_res > 0.0 and rmax <= exit_res:
            return "exit_res"
        stalled = len(run.history) > 3 and rmax > 0.9 * run.history[-4][1]
        if learned and switch_to_tpa and stalled:
            pc = b.KS_PRECOND_TPA
            run.switched_to_tpa_at = it
            log(f"[solve] learned preconditioner stalled at iteration {it}; switching to TPA")
        elif stall_exit and stalled:
            return "stall"
    return "maxit"


def run_to_tolerance(plan, v, X0, ntrack: int, precond: int, lock_tol: float, maxit: int, ref=None,
                     tol_ha: float = 1e-6, res_tol: float = 0.0, cnn_params=None, switch_to_tpa: bool = True,
                     crit: Criterion = None, log=print):
    """LOBPCG on one plan from X0 until the criterion (``crit``, or the
    eigenvalue part alone from ``ref``), a tracked residual of res_tol, or
    maxit.  Returns a dict with the wall time from X0 (initialisation
    included, checks excluded), iterations, history and the run."""
    import torch

    if crit is None and ref is not None:
        crit = Criterion(np.asarray(ref), None, None, 0, tol_ha)
    lob = b.Lobpcg(plan, v, X0)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lob.init()
    run = Run(lob)
    why = iterate(run, ntrack, precond, lock_tol, maxit, t0, crit, res_tol, cnn_params, switch_to_tpa, log=log)
    torch.cuda.synchronize()
    h = run.history[-1]
    return {"seconds": h[0], "iterations": run.iterations, "max_res": h[1], "max_err": h[2], "sin": h[4],
            "stopped": why, "reached": run.reached, "switched_to_tpa_at": run.switched_to_tpa_at,
            "history": run.history, "lobpcg": lob}


def run_mixed_refined(plan_m, v_m, plan_64, v_64, X0, ntrack: int, precond: int, lock_m: float, crit: Criterion,
                      maxit: int, cnn_params=None, handover_res: float = 2e-4, lock_64: float = 1e-9,
                      res_tol_64: float = 0.0, log=print):
    """Mixed-precision LOBPCG (complex64 blocks) until the max tracked
    residual is at most handover_res or stops falling, then the block is
    widened to complex128 and the FP64 plan continues (Cholesky-QR,
    Rayleigh-Ritz, TPA steps) until the criterion holds.  The FP32 residual
    floor (about 1e-4 here) bounds what the mixed steps alone can reach:
    eigenvalues within 1e-6 Ha, but subspace angles of order
    residual / gap; the FP64 steps close the rest.  Without a criterion
    (crit None) the FP64 steps run until the max tracked residual is at
    most res_tol_64."""
    import torch

    lob = b.Lobpcg(plan_m, v_m, X0.to(torch.complex64))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    lob.init()
    run = Run(lob)
    why = iterate(run, ntrack, precond, lock_m, maxit, t0, crit, 0.0, cnn_params, True, stall_exit=True,
                  exit_res=handover_res, log=log)
    mixed_iters = run.iterations
    switched = run.switched_to_tpa_at
    if not run.reached:
        log(f"[solve] handover to FP64 after {mixed_iters} mixed iterations ({why})")
        Xw = lob.X.to(torch.complex128)  # exact widening
        del lob
        run.lob = None
        torch.cuda.empty_cache()  # the complex64 blocks' memory back to the device for the FP64 ones
        lob64 = b.Lobpcg(plan_64, v_64, Xw)
        del Xw
        lob64.init()
        run.lob = lob64
        iterate(run, ntrack, b.KS_PRECOND_TPA, lock_64, maxit, t0, crit, res_tol_64, log=log)
    torch.cuda.synchronize()
    h = run.history[-1]
    return {"seconds": h[0], "iterations": run.iterations, "mixed_iterations": mixed_iters,
            "fp64_iterations": run.iterations - mixed_iters, "max_res": h[1], "max_err": h[2], "sin": h[4],
            "reached": run.reached, "switched_to_tpa_at": switched, "history": run.history, "lobpcg": run.lob}
