"""Oracle Teter-Payne-Allan preconditioner, plain FP64.

Part of the CPU oracle (test infrastructure only).

The paper's method is *preconditioned* LOBPCG but it names no
preconditioner.  This is the kinetic-energy preconditioner of Teter, Payne
and Allan (Phys. Rev. B 40, 12255 (1989)): in reciprocal space each residual
coefficient is multiplied by

    K(x) = (27 + 18x + 12x^2 + 8x^3) / (27 + 18x + 12x^2 + 8x^3 + 16x^4),

with x = (|G|^2/2) / E_i and E_i = <x_i|T|x_i> the kinetic energy of the
band's current Ritz vector (the original TPA choice).
"""
from __future__ import annotations

import numpy as np

from .hamiltonian import apply_t, dft3, kinetic_diag, kinetic_diag_k


def tpa_polynomial(x: np.ndarray) -> np.ndarray:
    num = 27.0 + 18.0 * x + 12.0 * x ** 2 + 8.0 * x ** 3
    return num / (num + 16.0 * x ** 4)


def band_kinetic_energy(X: np.ndarray, n: int, L: float, k=None) -> np.ndarray:
    """E_i = <x_i | T | x_i> for the rows x_i of X (nb, Ng); T = T_k with a
    Bloch vector k."""
    TX = apply_t(X, n, L, k)
    return np.real(np.einsum("ij,ij->i", np.conj(X), TX))


def tpa_apply(R: np.ndarray, E: np.ndarray, n: int, L: float, k=None) -> np.ndarray:
    """w_i = IDFT( K(T(G)/E_i) * DFT(r_i) ) for the rows r_i of R (nb, Ng),
    T(G) = |G + k|^2 / 2 with a Bloch vector k."""
    nb = R.shape[0]
    rh = dft3(R.reshape(nb, n, n, n), n)
    T = kinetic_diag(n, L) if k is None else kinetic_diag_k(n, L, k)
    x = T[None] / E[:, None, None, None]
    wh = rh * tpa_polynomial(x)
    return dft3(wh, n, inverse=True).reshape(nb, n ** 3)
