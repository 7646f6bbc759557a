"""Oracle Hamiltonian: H psi = T psi + V_loc psi + V_NL psi, in plain FP64.

Part of the CPU oracle (test infrastructure only).

Conventions (Hartree atomic units):
* grid point (i, j, k) at (i, j, k) * L / n; linear index (i*n + j)*n + k;
* forward transform sum_r exp(-i G.r) f(r), inverse with exp(+i G.r) / n
  per axis; G = 2 pi m / L with the integer m wrapped into [-n/2, n/2);
* kinetic energy of a plane wave |G|^2 / 2.

The SCF task list of the paper names the Laplacian through FFTs and the
nonlocal pseudopotential operator as two of its four cost centres; the local
potential completes H.  This module applies the transform as a *naive*
per-axis DFT (an n x n matrix contracted along each axis), which is slow but
has nothing in common with a fast transform.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

DIAMOND = [
    (0.0, 0.0, 0.0), (0.0, 0.5, 0.5), (0.5, 0.0, 0.5), (0.5, 0.5, 0.0),
    (0.25, 0.25, 0.25), (0.25, 0.75, 0.75), (0.75, 0.25, 0.75), (0.75, 0.75, 0.25),
]
BCC = [(0.0, 0.0, 0.0), (0.5, 0.5, 0.5)]


def dft_matrix(n: int, sign: int) -> np.ndarray:
    """F[k, j] = exp(sign * 2 pi i j k / n)."""
    j = np.arange(n)
    # reduce jk mod n in integers first so the phase is exact for large n
    return np.exp(sign * 2j * math.pi * ((np.outer(j, j) % n) / n))


def _along_axis(a: np.ndarray, F: np.ndarray, axis: int) -> np.ndarray:
    out = np.tensordot(a, F, axes=([axis], [1]))  # new axis appended last
    return np.moveaxis(out, -1, axis)


def dft3(psi: np.ndarray, n: int, inverse: bool = False) -> np.ndarray:
    """Separable 3D DFT of a (nb, n, n, n) block by naive per-axis matrices."""
    F = dft_matrix(n, +1 if inverse else -1)
    out = psi
    for ax in (1, 2, 3):
        out = _along_axis(out, F, ax)
    if inverse:
        out = out / float(n) ** 3
    return out


def wrapped_m(n: int) -> np.ndarray:
    k = np.arange(n)
    return np.where(2 * k < n, k, k - n)


def kinetic_diag(n: int, L: float) -> np.ndarray:
    """|G|^2 / 2 on the (n, n, n) reciprocal grid."""
    m = wrapped_m(n).astype(np.float64)
    g = 2.0 * math.pi / L * m
    g2 = g[:, None, None] ** 2 + g[None, :, None] ** 2 + g[None, None, :] ** 2
    return 0.5 * g2


def kinetic_diag_k(n: int, L: float, k) -> np.ndarray:
    """|G + k|^2 / 2 on the (n, n, n) reciprocal grid (k Cartesian, 1/bohr)."""
    m = wrapped_m(n).astype(np.float64)
    g = 2.0 * math.pi / L * m
    gx, gy, gz = g + k[0], g + k[1], g + k[2]
    return 0.5 * (gx[:, None, None] ** 2 + gy[None, :, None] ** 2 + gz[None, None, :] ** 2)


def apply_t(psi: np.ndarray, n: int, L: float, k=None) -> np.ndarray:
    """T psi for psi of shape (nb, Ng); with a Bloch vector k, the kinetic
    operator of the periodic part u of psi = exp(i k.r) u, |G + k|^2 / 2."""
    nb = psi.shape[0]
    p = psi.reshape(nb, n, n, n)
    ph = dft3(p, n)
    t = kinetic_diag(n, L) if k is None else kinetic_diag_k(n, L, k)
    ph = ph * t[None]
    return dft3(ph, n, inverse=True).reshape(nb, n ** 3)


# --------------------------------------------------------------------------
# The oracle's own geometry: potential and projectors recomputed from the
# cell description by brute force over every grid point and lattice image.
# --------------------------------------------------------------------------


@dataclass
class OracleCell:
    n: int
    L: float
    V: np.ndarray  # (Ng,)
    proj_supp: list  # per projector: int array of grid indices
    proj_val: list  # per projector: float array of b values
    D: np.ndarray  # (nproj,)
    # Bloch vector (Cartesian, 1/bohr) and, per projector, the displacement
    # of each support point from the atom (nearest image, bohr); both None
    # at the Gamma point
    k: np.ndarray = None
    proj_disp: list = None

    @property
    def Ng(self) -> int:
        return self.n ** 3


def oracle_positions(cfg) -> np.ndarray:
    if cfg.lattice == "custom":
        return np.array(cfg.positions, dtype=np.float64).reshape(-1, 3) * cfg.L
    basis = DIAMOND if cfg.lattice == "diamond" else BCC
    pos = []
    for i in range(cfg.nsc):
        for j in range(cfg.nsc):
            for k in range(cfg.nsc):
                for b in basis:
                    pos.append([(i + b[0]) * cfg.a, (j + b[1]) * cfg.a, (k + b[2]) * cfg.a])
    return np.array(pos, dtype=np.float64)


def grid_points(n: int, L: float) -> np.ndarray:
    h = L / n
    idx = np.arange(n) * h
    X, Y, Z = np.meshgrid(idx, idx, idx, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)


def oracle_potential(cfg, pos: np.ndarray) -> np.ndarray:
    """A sum_a sum_T exp(-|r - R_a - T|^2/(2 s^2)) over images within 10 s."""
    n, L, s = cfg.n, cfg.L, cfg.v_sigma
    cut = 10.0 * s
    r = grid_points(n, L)
    V = np.zeros(n ** 3)
    S = int(math.ceil(cut / L)) + 1
    for R in pos:
        for tx in range(-S, S + 1):
            for ty in range(-S, S + 1):
                for tz in range(-S, S + 1):
                    c = R + L * np.array([tx, ty, tz], dtype=np.float64)
                    # skip images whose nearest approach to the cell is beyond the cut
                    near = np.clip(c, 0.0, L)
                    if np.linalg.norm(c - near) > cut:
                        continue
                    d = r - c
                    d2 = np.einsum("ij,ij->i", d, d)
                    m = d2 <= cut * cut
                    V[m] += np.exp(-d2[m] / (2.0 * s * s))
    return cfg.v_depth * V


def _real_solid_harmonics(l: int, x, y, z):
    if l == 0:
        return [np.ones_like(x)]
    if l == 1:
        return [x, y, z]
    r2 = x * x + y * y + z * z
    return [x * y, y * z, z * x, (x * x - y * y) / 2.0, (3.0 * z * z - r2) / (2.0 * math.sqrt(3.0))]


def oracle_projectors(cfg, pos: np.ndarray, with_disp: bool = False):
    """Per projector: (support indices ascending, normalised values), and
    with ``with_disp`` the support points' displacements from the atom."""
    if cfg.lmax < 0:
        return ([], [], []) if with_disp else ([], [])
    n, L = cfg.n, cfg.L
    rcut = cfg.rcut_factor * cfg.rc
    r = grid_points(n, L)
    supp, vals, disp = [], [], []
    for R in pos:
        d = r - R
        d = d - L * np.floor(d / L + 0.5)  # minimum image
        d2 = np.einsum("ij,ij->i", d, d)
        idx = np.nonzero(d2 < rcut * rcut)[0]
        x, y, z = d[idx, 0], d[idx, 1], d[idx, 2]
        g = np.exp(-(x * x + y * y + z * z) / (2.0 * cfg.rc ** 2))
        for l in range(cfg.lmax + 1):
            for poly in _real_solid_harmonics(l, x, y, z):
                b = poly * g
                b = b / math.sqrt(float(np.sum(b * b)))
                supp.append(idx)
                vals.append(b)
                disp.append(d[idx])
    return (supp, vals, disp) if with_disp else (supp, vals)


def oracle_cell(cfg, D: np.ndarray) -> OracleCell:
    """Rebuild V and the projectors from the description; D is an input draw."""
    pos = oracle_positions(cfg)
    V = oracle_potential(cfg, pos)
    supp, vals = oracle_projectors(cfg, pos)
    if len(supp) != len(D):
        raise ValueError("projector count differs from the coupling constants")
    return OracleCell(cfg.n, cfg.L, V, supp, vals, np.asarray(D, dtype=np.float64))


def from_arrays(n: int, L: float, V: np.ndarray, supp: list, vals: list, D, k=None, disp=None) -> OracleCell:
    return OracleCell(n, L, np.asarray(V, np.float64), list(supp), list(vals), np.asarray(D, np.float64),
                      None if k is None else np.asarray(k, np.float64), None if disp is None else list(disp))


def _atom_groups(cell: OracleCell):
    """Consecutive projectors that share one support list (one atom)."""
    groups = []
    p = 0
    while p < len(cell.proj_supp):
        q = p + 1
        while q < len(cell.proj_supp) and (
            cell.proj_supp[q] is cell.proj_supp[p]
            or (len(cell.proj_supp[q]) == len(cell.proj_supp[p])
                and np.array_equal(cell.proj_supp[q], cell.proj_supp[p]))):
            q += 1
        groups.append((p, q))
        p = q
    return groups


def apply_nl(cell: OracleCell, psi: np.ndarray) -> np.ndarray:
    """sum over projectors p of b_p D_p (b_p^H psi).

    Projectors of one atom share a support, so their terms are formed
    together: c = psi_S B^H, then psi_S += (c * D) B with B the rows b_p.

    With a Bloch vector k the operator acts on the periodic part u of
    psi = exp(i k.r) u: the projector seen by u at a support point with
    displacement d from its atom is b(d) exp(-i k.d) (the orbital at the
    image of the point nearest the atom carries exp(i k.(R + d)), and
    H u = exp(-i k.r) H psi; the common factor exp(i k.R) cancels)."""
    out = np.zeros_like(psi)
    for p, q in _atom_groups(cell):
        idx = cell.proj_supp[p]
        B = np.array(cell.proj_val[p:q], dtype=np.complex128)  # (np_a, |S|)
        if cell.k is not None:
            B = B * np.exp(-1j * (cell.proj_disp[p] @ cell.k))[None, :]
        c = psi[:, idx] @ np.conj(B).T  # (nb, np_a)
        out[:, idx] += (c * cell.D[p:q]) @ B
    return out


def project(cell: OracleCell, psi: np.ndarray) -> np.ndarray:
    """Projector coefficients c[p, band] = sum_r b_p(r) psi_band(r)."""
    return np.array([psi[:, idx] @ b for idx, b in zip(cell.proj_supp, cell.proj_val)])


def apply_h(cell: OracleCell, psi: np.ndarray) -> np.ndarray:
    """H psi for psi of shape (nb, Ng), complex128."""
    psi = np.asarray(psi, dtype=np.complex128)
    out = apply_t(psi, cell.n, cell.L, cell.k)
    out = out + cell.V[None, :] * psi
    if cell.proj_supp:
        out = out + apply_nl(cell, psi)
    return out
