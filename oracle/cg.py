"""Oracle projected conjugate-gradient solve for training pairs, FP64.

Part of the CPU oracle (test infrastructure only).

A training target for the learned preconditioner is the correction t that
solves the Jacobi-Davidson-projected equation (Sleijpen and van der Vorst,
SIAM J. Matrix Anal. Appl. 17 (1996))

    P (H - theta_i) P t = r_i,   P = I - X X^H,   t in range(P),

for a Ritz pair (theta_i, x_i) with residual r_i.  The literal (H - theta)^-1 r
would return x_i itself, which carries no information.  When theta_i lies
below the lowest eigenvalue of H restricted to range(P), the projected
operator is positive definite there and plain CG (Hestenes and Stiefel)
converges; a non-positive curvature p^H A p <= 0 ends the solve as a skip.
"""
from __future__ import annotations

from typing import Callable

import numpy as np


def projected_cg(apply_h: Callable, X: np.ndarray, theta: float, r: np.ndarray,
                 rtol: float = 1e-6, maxit: int = 500):
    """Returns (t, iterations, ok).  X is band-major (nb, Ng) orthonormal."""

    def proj(v):
        return v - (np.conj(X) @ v) @ X

    def op(v):
        pv = proj(v)
        return proj(apply_h(pv[None, :])[0] - theta * pv)

    b = proj(np.asarray(r, dtype=np.complex128))
    bnorm = np.linalg.norm(b)
    t = np.zeros_like(b)
    if bnorm == 0.0:
        return t, 0, True
    res = b.copy()
    p = res.copy()
    rr = np.vdot(res, res).real
    for it in range(1, maxit + 1):
        Ap = op(p)
        curv = np.vdot(p, Ap).real
        if curv <= 0.0:
            return t, it, False
        alpha = rr / curv
        t = t + alpha * p
        res = res - alpha * Ap
        rr_new = np.vdot(res, res).real
        if np.sqrt(rr_new) <= rtol * bnorm:
            return proj(t), it, True
        p = res + (rr_new / rr) * p
        rr = rr_new
    return proj(t), maxit, False
