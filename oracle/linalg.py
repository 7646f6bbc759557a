"""Oracle dense linear algebra for the LOBPCG subspace problem, plain FP64.

Part of the CPU oracle (test infrastructure only).

The subspace problem H X = lambda S X (paragraph before Eq. 1) is reduced
with the Cholesky factor S = L L^H to K Z = lambda Z, K = L^-1 H L^-H,
Z = L^H X (Eq. 1).  K is formed by two triangular solves (paragraph after
Eq. 1): Y = L^-1 H and then K = L^-1 Y^H, which equals L^-1 H L^-H because
H is Hermitian.  The standard problem is solved here by cyclic complex
Jacobi rotations (Golub and Van Loan, "Matrix Computations", the symmetric
Jacobi method and its parallel round-robin ordering), and X = L^-H Z.

Every routine is an explicit loop over rows or columns, or over rounds of
disjoint Jacobi rotations; no LAPACK routine is called.
"""
from __future__ import annotations

import math

import numpy as np

CHOL_REL_TOL = 1e-14


def cholesky_lower(S: np.ndarray, rel_tol: float = CHOL_REL_TOL):
    """S = L L^H by the column-by-column (Cholesky-Crout) recurrence.

    Returns (L, info).  info = 0 on success; info = k (1-based) when the k-th
    pivot d_k = S_kk - sum_j |L_kj|^2 is not above rel_tol * max_i S_ii, in
    which case L is only valid in its first k-1 columns.
    """
    S = np.asarray(S, dtype=np.complex128)
    n = S.shape[0]
    L = np.zeros_like(S)
    dmax = float(np.max(np.real(np.diag(S)))) if n else 0.0
    for k in range(n):
        d = float(np.real(S[k, k]) - np.sum(np.abs(L[k, :k]) ** 2))
        if not (d > rel_tol * dmax):
            return L, k + 1
        L[k, k] = math.sqrt(d)
        # column below the pivot
        L[k + 1:, k] = (S[k + 1:, k] - L[k + 1:, :k] @ np.conj(L[k, :k])) / L[k, k]
    return L, 0


def cholesky_lower_deflate(S: np.ndarray, rel_tol: float = CHOL_REL_TOL):
    """Cholesky with deflation of dependent columns, S ~ L L^H.

    The Crout recurrence of ``cholesky_lower``, except that a column whose
    pivot d_k = S_kk - sum_j |L_kj|^2 is not above rel_tol * max_i S_ii is
    declared dead instead of stopping: L_kk = 1 and L_ik = 0 below it, so it
    takes no part in the later columns.  The live columns then hold exactly
    the Cholesky factor of S restricted to the live indices (a greedy choice
    from the left of a maximal well-conditioned set of basis vectors).
    Returns (L, dead) with dead a boolean mask.
    """
    S = np.asarray(S, dtype=np.complex128)
    n = S.shape[0]
    L = np.zeros_like(S)
    dead = np.zeros(n, dtype=bool)
    dmax = float(np.max(np.real(np.diag(S)))) if n else 0.0
    for k in range(n):
        d = float(np.real(S[k, k]) - np.sum(np.abs(L[k, :k]) ** 2))
        if not (d > rel_tol * dmax):
            dead[k] = True
            L[k, k] = 1.0
            continue
        L[k, k] = math.sqrt(d)
        L[k + 1:, k] = (S[k + 1:, k] - L[k + 1:, :k] @ np.conj(L[k, :k])) / L[k, k]
    return L, dead


def solve_lower(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Y with L Y = B, forward substitution row by row."""
    n = L.shape[0]
    Y = np.zeros_like(B, dtype=np.complex128)
    for i in range(n):
        Y[i] = (B[i] - L[i, :i] @ Y[:i]) / L[i, i]
    return Y


def solve_lower_conj_t(L: np.ndarray, B: np.ndarray) -> np.ndarray:
    """X with L^H X = B, backward substitution row by row."""
    n = L.shape[0]
    X = np.zeros_like(B, dtype=np.complex128)
    LH = np.conj(L.T)
    for i in range(n - 1, -1, -1):
        X[i] = (B[i] - LH[i, i + 1:] @ X[i + 1:]) / LH[i, i]
    return X


def _round_robin(m: int):
    """Rounds of disjoint pairs covering every (p, q) once (m even)."""
    players = list(range(m))
    rounds = []
    for _ in range(m - 1):
        pairs = [(players[i], players[m - 1 - i]) for i in range(m // 2)]
        rounds.append([(min(p, q), max(p, q)) for p, q in pairs])
        players = [players[0]] + [players[-1]] + players[1:-1]
    return rounds


def jacobi_eigh(K: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """Eigen-decomposition of a Hermitian K by cyclic complex Jacobi.

    Each rotation annihilates one off-diagonal pair (p, q): with
    K_pq = |b| e^{i phi}, the unitary J = diag(1, e^{-i phi}) R(theta) turns the
    2x2 block real and then diagonal, tan(theta) = t the smaller root of
    t^2 + 2 tau t - 1 = 0, tau = (K_qq - K_pp) / (2 |b|).  Rotations are applied
    in round-robin rounds of disjoint pairs until the off-diagonal Frobenius
    norm is at most tol * ||K||_F.  Returns (w, Z) sorted ascending.
    """
    A = np.array(K, dtype=np.complex128)
    n = A.shape[0]
    Z = np.eye(n, dtype=np.complex128)
    if n == 1:
        return np.real(np.diag(A)).copy(), Z
    m = n + (n % 2)
    if m != n:  # pad with a decoupled dummy index
        A2 = np.zeros((m, m), dtype=np.complex128)
        A2[:n, :n] = A
        Z2 = np.eye(m, dtype=np.complex128)
        A, Z = A2, Z2
    rounds = _round_robin(m)
    fro = np.linalg.norm(A)
    for _ in range(max_sweeps):
        off = np.linalg.norm(A - np.diag(np.diag(A)))
        if off <= tol * fro or off == 0.0:
            break
        for pairs in rounds:
            P = np.array([p for p, _ in pairs])
            Q = np.array([q for _, q in pairs])
            b = A[P, Q]
            absb = np.abs(b)
            act = absb > 0.0
            a_pp = np.real(A[P, P])
            a_qq = np.real(A[Q, Q])
            safe = np.where(act, absb, 1.0)
            diff = a_qq - a_pp
            # |tau| beyond 1e100: t = 1/(2 tau) to full precision, no overflow
            huge = np.abs(diff) > 1e100 * safe
            tau = np.divide(diff, 2.0 * safe, out=np.ones_like(diff), where=~huge)
            sgn = np.where(tau >= 0.0, 1.0, -1.0)
            t = sgn / (np.abs(tau) + np.sqrt(1.0 + tau * tau))
            t = np.where(huge, np.divide(safe, diff, out=np.zeros_like(diff), where=huge), t)
            c = 1.0 / np.sqrt(1.0 + t * t)
            s = t * c
            ph = np.where(act, b / safe, 1.0)  # e^{i phi}
            c = np.where(act, c, 1.0)
            s = np.where(act, s, 0.0)
            # J = [[c, s], [-s e^{-i phi}, c e^{-i phi}]] on (p, q)
            j00, j01 = c, s
            j10, j11 = -s * np.conj(ph), c * np.conj(ph)
            # columns: A <- A J
            cp, cq = A[:, P].copy(), A[:, Q].copy()
            A[:, P] = cp * j00 + cq * j10
            A[:, Q] = cp * j01 + cq * j11
            zp, zq = Z[:, P].copy(), Z[:, Q].copy()
            Z[:, P] = zp * j00 + zq * j10
            Z[:, Q] = zp * j01 + zq * j11
            # rows: A <- J^H A
            rp, rq = A[P, :].copy(), A[Q, :].copy()
            A[P, :] = np.conj(j00)[:, None] * rp + np.conj(j10)[:, None] * rq
            A[Q, :] = np.conj(j01)[:, None] * rp + np.conj(j11)[:, None] * rq
            A[P, Q] = 0.0
            A[Q, P] = 0.0
            A[P, P] = np.real(A[P, P])
            A[Q, Q] = np.real(A[Q, Q])
    w = np.real(np.diag(A))[:n]
    Z = Z[:n, :n]
    order = np.argsort(w, kind="stable")
    return w[order], Z[:, order]


def hegv_two_trsm(H: np.ndarray, S: np.ndarray, nev: int):
    """Lowest nev eigenpairs of H C = S C diag(w), C^H S C = I.

    Steps: L = chol(S); Y = L^-1 H; K = L^-1 Y^H; K <- (K + K^H)/2;
    (w, Z) = Jacobi(K); C = L^-H Z[:, :nev].  Returns (w[:nev], C, info) with
    info = n + k when the leading minor k of S is not positive definite.
    """
    n = H.shape[0]
    L, info = cholesky_lower(S)
    if info:
        return None, None, n + info
    Y = solve_lower(L, H)
    K = solve_lower(L, np.conj(Y.T))
    K = 0.5 * (K + np.conj(K.T))
    w, Z = jacobi_eigh(K)
    C = solve_lower_conj_t(L, Z[:, :nev])
    return w[:nev], C, 0


def hegv_two_trsm_deflate(H: np.ndarray, S: np.ndarray, nev: int):
    """The reduction of ``hegv_two_trsm`` on a possibly singular S.

    Columns that ``cholesky_lower_deflate`` declares dead are dropped from the
    basis: the pencil restricted to the live indices is solved exactly as in
    ``hegv_two_trsm`` (its Cholesky factor is the live part of L), and the
    coefficients of the dead basis vectors are zero.  Needs at least nev live
    columns.  Returns (w[:nev], C, ndead).
    """
    n = H.shape[0]
    _, dead = cholesky_lower_deflate(S)
    live = np.nonzero(~dead)[0]
    if len(live) < nev:
        raise np.linalg.LinAlgError("fewer independent basis vectors than wanted eigenpairs")
    w, Cl, info = hegv_two_trsm(H[np.ix_(live, live)], S[np.ix_(live, live)], nev)
    if info:
        raise np.linalg.LinAlgError("live block not positive definite")  # unreachable: same pivots
    C = np.zeros((n, nev), dtype=np.complex128)
    C[live] = Cl
    return w, C, int(np.sum(dead))
