"""Oracle LOBPCG for H X = X Theta, plain FP64 (B = I).

Part of the CPU oracle (test infrastructure only).

The paper forms the subspace matrices H and S of LOBPCG by dense products
and solves H X = lambda S X through Cholesky, two triangular solves and a
Hermitian eigensolve (SCF task list; Eq. 1 and the paragraph after it).
The iteration itself is Knyazev's LOBPCG (the method cited in the task
list), Rayleigh-Ritz on V = [X, W, P]; the overlap metric is the identity
because the pseudopotentials are norm-conserving (benchmark-target
paragraph).

Readings of points the paper leaves open (each listed in the design notes):
* W is the preconditioned residual, made orthogonal to X by one classical
  Gram-Schmidt pass, W <- W - X (X^H W).  Soft locking with fixed shapes: a
  band whose residual norm is at most ``lock_tol`` contributes an
  exactly-zero column to W and to P (its X column stays in the Rayleigh-Ritz
  step).
* W and P are each orthonormalised *within their own block* before the Gram
  matrices are formed: columns are scaled to unit length (a zero column
  stays zero), then B <- B L^-H with L L^H = B^H B (Cholesky-QR; a zero
  column gets a unit pivot).  The Cholesky deflates: a column whose pivot
  is not above 1e-14 of the largest diagonal entry depends numerically on
  the columns before it and becomes a zero column (the Cholesky-QR of the
  remaining ones is exact).  Without this orthonormalisation the basis
  loses rank as the residuals fall and the iteration stalls near 1e-6
  (Hetmaniuk and Lehoucq, "Basis selection in LOBPCG", J. Comput. Phys. 218
  (2006), analyse the same loss).
* No orthogonalisation *across* blocks, so S != I (the X-W, X-P and W-P
  blocks are full) and the Cholesky plus two-solve reduction does real work.
* A zero column k of [W, P] is decoupled from the subspace problem:
  S_kk = 1 and H_kk = 2 max_i |H_ii| + 1 (its other entries are exactly
  zero), so it sits above every retained Ritz value and gets zero weight.
* The Cholesky of the subspace overlap deflates in the same way: a basis
  vector that depends numerically on the vectors before it in [X, W, P] is
  dropped (zero Ritz coefficients), and the reduction and eigensolve run on
  the remaining ones.  No step of the iteration is repeated.
* H_s and S_s are Hermitised, (A + A^H)/2, before the reduction.
* AX and AP are formed by applying H to the new X and P every iteration,
  not by rotating AV with the Ritz coefficients: the rotated products drift
  from H X once the basis is ill-conditioned (the drift grows geometrically
  and ends the convergence), while a fresh H-apply has no memory.

Blocks are stored band-major, shape (nb, Ng); as matrices they are the
transposes (Ng x nb).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, Optional

import numpy as np

from .hamiltonian import OracleCell, apply_h
from .linalg import cholesky_lower, cholesky_lower_deflate, hegv_two_trsm_deflate, jacobi_eigh, solve_lower
from .precond import band_kinetic_energy, tpa_apply


def _herm(A: np.ndarray) -> np.ndarray:
    return 0.5 * (A + np.conj(A.T))


def gram(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """A^H B for band-major blocks: G[i, j] = sum_r conj(a_i(r)) b_j(r)."""
    return np.conj(A) @ B.T


def rotate(V: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Band-major result of the matrix product V_mat C (V_mat = V.T)."""
    return C.T @ V


def cholesky_qr(X: np.ndarray):
    """X <- X L^-H with L = chol(X^H X); returns (Xq, L, info)."""
    G = _herm(gram(X, X))
    L, info = cholesky_lower(G)
    if info:
        return None, None, info
    # X_new^H = L^-1 X^H  (rows of the band-major block are the columns)
    Xq = np.conj(solve_lower(L, np.conj(X)))
    return Xq, L, 0


@dataclass
class State:
    X: np.ndarray
    AX: np.ndarray
    theta: np.ndarray
    P: Optional[np.ndarray] = None
    AP: Optional[np.ndarray] = None
    iteration: int = 0
    events: list = field(default_factory=list)


def initial_state(cell: OracleCell, X0: np.ndarray) -> State:
    """Cholesky-QR of X0, then Rayleigh-Ritz on span(X0) with S = I."""
    X, _, info = cholesky_qr(np.asarray(X0, dtype=np.complex128))
    if info:
        raise np.linalg.LinAlgError("initial block is rank deficient")
    AX = apply_h(cell, X)
    Hs = _herm(gram(X, AX))
    w, Z = jacobi_eigh(Hs)
    Xr = rotate(X, Z)
    return State(Xr, apply_h(cell, Xr), w.copy())


def residual(st: State):
    R = st.AX - st.theta[:, None] * st.X
    return R, np.linalg.norm(R, axis=1)


def orthonormalise_block(B: np.ndarray, AB: Optional[np.ndarray] = None):
    """Unit-normalise the columns of B, then Cholesky-QR: B <- B D L^-H.

    D = diag(1/||b_i||) (0 for a zero column) and L L^H = D B^H B D with a
    unit pivot for zero columns, from the deflating Cholesky: a dead
    (numerically dependent) column becomes a zero column, the live ones are
    orthonormalised by the live part of L.  AB (= H B) receives the same
    transform.  Returns (B', AB', number of dead columns).
    """
    nrm = np.linalg.norm(B, axis=1)
    d = np.where(nrm > 0.0, 1.0 / np.where(nrm > 0.0, nrm, 1.0), 0.0)
    Bs = B * d[:, None]
    ABs = None if AB is None else AB * d[:, None]
    G = _herm(gram(Bs, Bs))
    zero = np.real(np.diag(G)) == 0.0
    G[zero, zero] = 1.0
    L, dead = cholesky_lower_deflate(G)
    live = np.nonzero(~dead)[0]
    Ll = L[np.ix_(live, live)]
    Bq = np.zeros_like(Bs)
    Bq[live] = np.conj(solve_lower(Ll, np.conj(Bs[live])))
    ABq = None
    if ABs is not None:
        ABq = np.zeros_like(ABs)
        ABq[live] = np.conj(solve_lower(Ll, np.conj(ABs[live])))
    return Bq, ABq, int(np.sum(dead))


def decouple_zero_columns(Hs: np.ndarray, Ss: np.ndarray):
    """S_kk = 1 and H_kk = 2 max|H_ii| + 1 wherever column k is zero."""
    zero = np.real(np.diag(Ss)) == 0.0
    if np.any(zero):
        big = 2.0 * float(np.max(np.abs(np.real(np.diag(Hs))))) + 1.0
        Ss = Ss.copy()
        Hs = Hs.copy()
        Ss[zero, zero] = 1.0
        Hs[zero, zero] = big
    return Hs, Ss, int(np.sum(zero))


def step(cell: OracleCell, st: State, precond: Optional[Callable] = None,
         lock_tol: float = 0.0) -> State:
    """One LOBPCG iteration from (X, AX, Theta, P, AP)."""
    nb = st.X.shape[0]
    events = []
    R, res = residual(st)
    active = (res > lock_tol).astype(np.float64)
    R = R * active[:, None]
    W = R if precond is None else precond(R, st)
    W = W - rotate(st.X, gram(st.X, W))
    W, _, ndead = orthonormalise_block(W)
    if ndead:
        events.append(f"w_deflated_{ndead}")
    AW = apply_h(cell, W)
    blocks = [st.X, W]
    ablocks = [st.AX, AW]
    if st.P is not None:
        P, _, ndead = orthonormalise_block(st.P * active[:, None])
        if ndead:
            events.append(f"p_deflated_{ndead}")
        blocks.append(P)
        ablocks.append(apply_h(cell, P))
    V = np.concatenate(blocks, axis=0)
    AV = np.concatenate(ablocks, axis=0)
    Ss = _herm(gram(V, V))
    Hs = _herm(gram(V, AV))
    Hs, Ss, _ = decouple_zero_columns(Hs, Ss)
    w, C, ndead = hegv_two_trsm_deflate(Hs, Ss, nb)
    if ndead:
        events.append(f"basis_deflated_{ndead}")
    Xn = rotate(V, C)
    Pn = rotate(V[nb:], C[nb:])
    return State(Xn, apply_h(cell, Xn), w.copy(), Pn, None, st.iteration + 1, st.events + events)


def tpa_preconditioner(cell: OracleCell):
    def apply(R: np.ndarray, st: State) -> np.ndarray:
        E = band_kinetic_energy(st.X, cell.n, cell.L, cell.k)
        return tpa_apply(R, E, cell.n, cell.L, cell.k)

    return apply


def run(
    cell: OracleCell,
    X0: np.ndarray,
    ntrack: int,
    tol: float = 1e-8,
    maxit: int = 200,
    precond: Optional[Callable] = None,
    callback: Optional[Callable] = None,
    lock_factor: float = 0.1,
):
    """Iterate until the largest tracked residual norm is at most tol.

    Bands whose residual is at most ``lock_factor * tol`` are soft-locked.
    Returns (state, history) where history holds (theta, residual norms) of
    the block at the start of every iteration.
    """
    st = initial_state(cell, X0)
    hist = []
    for _ in range(maxit + 1):
        _, res = residual(st)
        hist.append((st.theta.copy(), res.copy()))
        if callback is not None:
            callback(st, res)
        if np.max(res[:ntrack]) <= tol:
            return st, hist
        st = step(cell, st, precond, lock_factor * tol)
    return st, hist
