"""The self-consistent field loop around the LOBPCG eigensolve.

Orchestration only: the density, the Hartree potential (periodic Poisson
equation on the FFT passes), the local-density exchange-correlation
potential, the effective potential with its grid sums and the density
mixing all run in libksh.so (ks_density, ks_scf_potential,
ks_mix_density), and every eigensolve is lobpcg_init plus lobpcg_step on
the updated potential, started from the previous orbitals.

Loop: the first eigensolve in V_ion gives n_in; then V_eff[n_in], an
eigensolve of the occupied bands to a residual of inner_tol, n_out, and
linear mixing n_in <- (1 - alpha) n_in + alpha n_out, until
||n_out - n_in||_2 <= tol.  The electronic energy (without ion-ion terms)
is sum_i f_i theta_i - (1/2) sum V_H n - sum v_xc n + sum e_xc n, f_i = 2.
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import binding as b


@dataclass
class ScfRun:
    n: object  # device float64, electrons per grid point (the last output density)
    theta: np.ndarray
    energy: float
    iterations: int
    lobpcg_steps: int
    seconds: float
    history: list = field(default_factory=list)  # (||n_out - n_in||, energy, lobpcg steps)
    lobpcg: object = None


def run_scf(plan, v_ion, X0, nocc: int, alpha: float = 0.3, tol: float = 1e-7, maxit: int = 60,
            inner_tol: float = 1e-9, inner_maxit: int = 200, precond: int = b.KS_PRECOND_TPA, log=print) -> ScfRun:
    """v_ion: device float64 (Ng); X0: device block (nb, Ng) of the plan's
    complex type, nb >= nocc."""
    import torch

    dev = v_ion.device
    Ng = plan.Ng
    v_eff = v_ion.to(plan.real_dtype).clone()
    lob = b.Lobpcg(plan, v_eff, X0)
    n_in = torch.zeros(Ng, dtype=torch.float64, device=dev)
    n_out = torch.zeros_like(n_in)
    n_next = torch.zeros_like(n_in)
    terms = torch.zeros(4, dtype=torch.float64, device=dev)
    resid = torch.zeros(1, dtype=torch.float64, device=dev)
    work = b._scf_work(plan, dev)
    steps = [0]

    def solve():
        lob.init()
        for _ in range(inner_maxit):
            lob.step(precond, 0.1 * inner_tol)
            steps[0] += 1
            st = lob.status_host
            if st[b.KS_ST_FLAGS] & (b.KS_FLAG_SOLVE_FAILED | b.KS_FLAG_NONFINITE):
                raise b.KsError(f"LOBPCG step failed inside the SCF loop: status {st.tolist()}")
            if float(lob.res_host[:nocc].max()) <= inner_tol:
                return

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    solve()
    b.ks_density(plan, lob.X, nocc, n_in)
    hist = []
    e = float("nan")
    it = 0
    for it in range(1, maxit + 1):
        b.ks_scf_potential(plan, n_in, v_ion, v_eff, terms, work)
        solve()
        b.ks_density(plan, lob.X, nocc, n_out)
        b.ks_mix_density(plan, alpha, n_in, n_out, n_next, resid, work)
        r = float(resid.item())
        tt = terms.cpu().numpy()
        th = lob.theta_host[:nocc]
        e = float(2.0 * th.sum() - 0.5 * tt[0] - tt[1] + tt[2])
        hist.append((r, e, steps[0]))
        log(f"[scf] iteration {it}: ||n_out - n_in|| {r:.3e}, energy {e:.10f} Ha, electrons {tt[3]:.10f}, "
            f"{steps[0]} LOBPCG steps")
        if r <= tol:
            break
        n_in, n_next = n_next, n_in
    torch.cuda.synchronize()
    return ScfRun(n_out, lob.theta_host.copy(), e, it, steps[0], time.perf_counter() - t0, hist, lob)
