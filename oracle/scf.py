"""Oracle self-consistent field loop around the eigensolve, plain FP64.

Part of the CPU oracle (test infrastructure only).

The paper's SCF iteration repeats the eigensolve inside an outer loop whose
other steps (density, potential, mixing) are the "Others" of its cost
breakdown (SCF task list and the Fig. 1 discussion).  The readings here:

* Occupied orbitals x_i (unit Euclidean norm on the grid) with occupations
  f_i (2 for a closed shell) give electrons per grid point
  n(r) = sum_i f_i |x_i(r)|^2; the density per volume is rho = n / dV with
  dV = L^3 / Ng, and sum_r n(r) = sum_i f_i.
* Hartree potential by the periodic Poisson equation, lap V_H = -4 pi rho,
  in Fourier space: V_H(G) = 4 pi rho(G) / |G|^2, V_H(G = 0) = 0 (a uniform
  neutralising background).  Transforms: the oracle's separable naive DFT.
* Local density approximation: Slater exchange
  e_x = -(3/4) (3 rho / pi)^(1/3), v_x = (4/3) e_x, and the Perdew-Zunger
  parametrisation of the Ceperley-Alder correlation energy (Phys. Rev. B 23,
  5048 (1981)), r_s = (3 / (4 pi rho))^(1/3):
    r_s >= 1: e_c = g / (1 + b1 sqrt(r_s) + b2 r_s), g = -0.1423,
              b1 = 1.0529, b2 = 0.3334;
    r_s <  1: e_c = A ln r_s + B + C r_s ln r_s + D r_s, A = 0.0311,
              B = -0.048, C = 0.0020, D = -0.0116;
  v_c = e_c - (r_s / 3) d e_c / d r_s.  Densities below 1e-30 bohr^-3 get
  zero energy and potential.
* V_eff = V_ion + V_H + V_xc; linear mixing of the input density,
  n_in <- (1 - alpha) n_in + alpha n_out, until ||n_out - n_in||_2 is below
  a tolerance.
* Reported energy (electronic, without ion-ion terms):
  E = sum_i f_i theta_i - (1/2) sum_r V_H n - sum_r v_xc n + sum_r e_xc n.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Callable

import numpy as np

from .hamiltonian import dft3, kinetic_diag, from_arrays, OracleCell

PZ_G, PZ_B1, PZ_B2 = -0.1423, 1.0529, 0.3334
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116
RHO_MIN = 1e-30


def density(X: np.ndarray, occ: np.ndarray) -> np.ndarray:
    """Electrons per grid point, n(r) = sum_i f_i |x_i(r)|^2 (X band-major)."""
    return np.einsum("i,ir->r", np.asarray(occ, np.float64), np.abs(X) ** 2)


def hartree(n: np.ndarray, ngrid: int, L: float) -> np.ndarray:
    """V_H on the grid from electrons per grid point n (Ng reals)."""
    dV = L ** 3 / ngrid ** 3
    rho = (n / dV).astype(np.complex128).reshape(1, ngrid, ngrid, ngrid)
    rho_g = dft3(rho, ngrid)
    g2 = 2.0 * kinetic_diag(ngrid, L)  # |G|^2
    fac = np.where(g2 > 0.0, 4.0 * math.pi / np.where(g2 > 0.0, g2, 1.0), 0.0)
    v = dft3(fac[None] * rho_g, ngrid, inverse=True)
    return np.real(v).reshape(ngrid ** 3)


def lda_xc(rho: np.ndarray):
    """(e_xc, v_xc) per the LDA above, for densities per volume rho."""
    rho = np.asarray(rho, np.float64)
    live = rho > RHO_MIN
    r = np.where(live, rho, 1.0)
    ex = -0.75 * np.cbrt(3.0 * r / math.pi)
    vx = 4.0 / 3.0 * ex
    rs = np.cbrt(3.0 / (4.0 * math.pi * r))
    hi = rs >= 1.0
    sq = np.sqrt(rs)
    den = 1.0 + PZ_B1 * sq + PZ_B2 * rs
    ec_hi = PZ_G / den
    vc_hi = ec_hi * (1.0 + 7.0 / 6.0 * PZ_B1 * sq + 4.0 / 3.0 * PZ_B2 * rs) / den
    lnr = np.log(rs)
    ec_lo = PZ_A * lnr + PZ_B + PZ_C * rs * lnr + PZ_D * rs
    vc_lo = PZ_A * lnr + (PZ_B - PZ_A / 3.0) + 2.0 / 3.0 * PZ_C * rs * lnr + (2.0 * PZ_D - PZ_C) / 3.0 * rs
    ec = np.where(hi, ec_hi, ec_lo)
    vc = np.where(hi, vc_hi, vc_lo)
    exc = np.where(live, ex + ec, 0.0)
    vxc = np.where(live, vx + vc, 0.0)
    return exc, vxc


def potential(n: np.ndarray, v_ion: np.ndarray, ngrid: int, L: float):
    """V_eff = V_ion + V_H[n] + V_xc[n]; also the sums over the grid
    (sum V_H n, sum v_xc n, sum e_xc n, sum n)."""
    dV = L ** 3 / ngrid ** 3
    vh = hartree(n, ngrid, L)
    exc, vxc = lda_xc(n / dV)
    terms = np.array([np.sum(vh * n), np.sum(vxc * n), np.sum(exc * n), np.sum(n)])
    return v_ion + vh + vxc, terms


def mix(n_in: np.ndarray, n_out: np.ndarray, alpha: float):
    """Linear mixing; returns (next input density, ||n_out - n_in||_2)."""
    return (1.0 - alpha) * n_in + alpha * n_out, float(np.linalg.norm(n_out - n_in))


def energy(theta: np.ndarray, occ: np.ndarray, terms: np.ndarray) -> float:
    """Electronic energy from the band energies and the grid sums of the
    potential that produced them (double counting removed)."""
    return float(np.sum(occ * theta) - 0.5 * terms[0] - terms[1] + terms[2])


@dataclass
class ScfResult:
    n: np.ndarray
    theta: np.ndarray
    X: np.ndarray
    energy: float
    iterations: int
    history: list = field(default_factory=list)


def run(cell: OracleCell, nocc: int, eigensolve: Callable, X0: np.ndarray, alpha: float = 0.3, tol: float = 1e-7,
        maxit: int = 60) -> ScfResult:
    """The SCF loop with a supplied eigensolver
    eigensolve(cell_with_v_eff, X_start) -> (theta, X): the lowest bands of
    H = T + V_eff + V_NL, band-major, orthonormal.  n_in starts as the
    density of the eigensolve in V_ion alone."""
    occ = np.full(nocc, 2.0)
    v_ion = cell.V.copy()
    theta, X = eigensolve(cell, X0)
    n_in = density(X[:nocc], occ)
    hist = []
    for it in range(1, maxit + 1):
        v_eff, terms = potential(n_in, v_ion, cell.n, cell.L)
        c = from_arrays(cell.n, cell.L, v_eff, cell.proj_supp, cell.proj_val, cell.D)
        theta, X = eigensolve(c, X)
        n_out = density(X[:nocc], occ)
        n_next, resid = mix(n_in, n_out, alpha)
        e = energy(theta[:nocc], occ, terms)
        hist.append((resid, e))
        if resid <= tol:
            return ScfResult(n_out, theta, X, e, it, hist)
        n_in = n_next
    return ScfResult(n_out, theta, X, e, maxit, hist)
