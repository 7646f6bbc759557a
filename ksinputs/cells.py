"""Synthetic diamond-like and bcc-metal cells for the Kohn-Sham eigensolve.

The paper benchmarks a 216-atom diamond 3x3x3 supercell and a 128-atom bcc
tungsten 4x4x4 supercell with ONCV pseudopotentials (benchmark-target
paragraph).  Those pseudopotential files are not available, so these cells
keep the supercell shapes and band counts and replace the physics by:

* a local potential that is a periodic sum of Gaussians,
      V(r) = A * sum_a sum_T exp(-|r - R_a - T|^2 / (2 sigma^2)),
  where T runs over lattice translations and an image contributes while
  |r - R_a - T| <= 10 sigma;
* separable Kleinman-Bylander projectors b_lm(r) = |r|^l exp(-|r|^2/(2 rc^2))
  Y_lm(r/|r|) written with real solid harmonics, supported on the grid points
  whose minimum-image distance to the atom is below 4 rc, and normalised so
  that sum_r b(r)^2 = 1 on the grid;
* one coupling constant D per (atom, l), uniform in [-1, 1] Ha, shared by the
  2l+1 projectors of that shell.

Random numbers come from ``numpy.random.default_rng`` (PCG64): the cell (the
D values, atoms in order and l ascending) uses seed 0, the initial orbital
block uses seed 1 and is (N(0,1) + i N(0,1))/sqrt(2), the real part drawn
first, with shape (nb, Ng).

Grid point (i, j, k) sits at (i, j, k) * L / n from the cell origin and has
linear index (i*n + j)*n + k, so an orbital block is stored band-major with
z fastest.
"""
from __future__ import annotations

import dataclasses
import math
from dataclasses import dataclass
from typing import Optional, Sequence

import numpy as np

DIAMOND_BASIS = np.array(
    [
        [0.0, 0.0, 0.0],
        [0.0, 0.5, 0.5],
        [0.5, 0.0, 0.5],
        [0.5, 0.5, 0.0],
        [0.25, 0.25, 0.25],
        [0.25, 0.75, 0.75],
        [0.75, 0.25, 0.75],
        [0.75, 0.75, 0.25],
    ]
)
BCC_BASIS = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.5]])


@dataclass(frozen=True)
class CellConfig:
    """One problem instance: geometry, grid, bands, potential, projectors."""

    name: str
    lattice: str  # "diamond", "bcc" or "custom"
    a: float  # conventional lattice constant (bohr); for "custom" the cell edge L
    nsc: int  # supercell repeats per axis
    n: int  # grid points per axis
    nb: int  # bands in the block
    ntrack: int  # occupied bands tracked for convergence
    v_depth: float  # A (Ha)
    v_sigma: float  # sigma (bohr)
    lmax: int  # -1: no nonlocal term; 0: s; 1: s+p; 2: s+p+d
    rc: float  # projector Gaussian radius (bohr)
    precision: str  # "fp64" or "mixed"
    res_tol: float = 1e-8
    positions: Optional[tuple] = None  # custom fractional positions
    rcut_factor: float = 4.0

    @property
    def L(self) -> float:
        return self.a * self.nsc

    @property
    def Ng(self) -> int:
        return self.n ** 3

    @property
    def h(self) -> float:
        return self.L / self.n

    @property
    def nproj_per_atom(self) -> int:
        return 0 if self.lmax < 0 else (self.lmax + 1) ** 2


def diamond_sites(nsc: int, a: float) -> np.ndarray:
    """Atom positions (bohr): supercell images lexicographic, then basis."""
    out = []
    for i in range(nsc):
        for j in range(nsc):
            for k in range(nsc):
                for b in DIAMOND_BASIS:
                    out.append((np.array([i, j, k]) + b) * a)
    return np.array(out, dtype=np.float64)


def bcc_sites(nsc: int, a: float) -> np.ndarray:
    out = []
    for i in range(nsc):
        for j in range(nsc):
            for k in range(nsc):
                for b in BCC_BASIS:
                    out.append((np.array([i, j, k]) + b) * a)
    return np.array(out, dtype=np.float64)


# The five workloads.  C1..C4 are eigensolve cells; C5 (the learned
# preconditioner) trains on C1 and C2 and is applied on C2 and C3.
CONFIGS = {
    "C1": CellConfig("C1", "diamond", 6.74, 1, 16, 16, 16, -2.0, 0.8, -1, 1.0, "fp64"),
    "C2": CellConfig("C2", "diamond", 6.74, 2, 48, 160, 128, -2.0, 0.8, 1, 1.0, "fp64"),
    "C3": CellConfig("C3", "diamond", 6.74, 3, 96, 480, 432, -2.0, 0.8, 1, 1.0, "mixed", 1e-6),
    "C4": CellConfig("C4", "bcc", 5.98, 4, 112, 960, 896, -4.0, 0.6, 2, 1.2, "mixed", 1e-6),
}


def config(name: str, **overrides) -> CellConfig:
    cfg = CONFIGS[name]
    return dataclasses.replace(cfg, **overrides) if overrides else cfg


def custom_config(
    name: str,
    L: float,
    n: int,
    frac_positions: Sequence[Sequence[float]],
    nb: int,
    v_depth: float = -2.0,
    v_sigma: float = 0.8,
    lmax: int = -1,
    rc: float = 1.0,
    precision: str = "fp64",
    ntrack: Optional[int] = None,
    res_tol: float = 1e-8,
    rcut_factor: float = 4.0,
) -> CellConfig:
    """A small cubic cell of edge L with explicit fractional positions."""
    pos = tuple(tuple(float(c) for c in p) for p in frac_positions)
    return CellConfig(
        name, "custom", L, 1, n, nb, nb if ntrack is None else ntrack,
        v_depth, v_sigma, lmax, rc, precision, res_tol, pos, rcut_factor,
    )


@dataclass
class Cell:
    cfg: CellConfig
    L: float
    n: int
    h: float
    positions: np.ndarray  # (natoms, 3) bohr
    V: np.ndarray  # (Ng,) float64
    # projector set, CSR by atom
    atom_supp_ptr: np.ndarray  # (natoms+1,) int32
    supp_idx: np.ndarray  # (nsupp,) int32, ascending within an atom
    atom_proj_ptr: np.ndarray  # (natoms+1,) int32
    beta: np.ndarray  # float64, atom-major, then projector, then support point
    D: np.ndarray  # (nproj,) float64
    proj_atom: np.ndarray  # (nproj,) int32
    proj_l: np.ndarray  # (nproj,) int32
    beta_ptr: np.ndarray  # (natoms+1,) int64 offsets of each atom's beta slab
    # (nsupp, 3) float64: displacement of each support point from its atom
    # (the image of the point nearest the atom), in bohr
    supp_disp: np.ndarray = None

    @property
    def Ng(self) -> int:
        return self.n ** 3

    @property
    def natoms(self) -> int:
        return len(self.positions)

    @property
    def nproj(self) -> int:
        return len(self.D)


def atom_positions(cfg: CellConfig) -> np.ndarray:
    if cfg.lattice == "diamond":
        return diamond_sites(cfg.nsc, cfg.a)
    if cfg.lattice == "bcc":
        return bcc_sites(cfg.nsc, cfg.a)
    if cfg.lattice == "custom":
        return np.array(cfg.positions, dtype=np.float64).reshape(-1, 3) * cfg.L
    raise ValueError(cfg.lattice)


def _gaussian_potential(cfg: CellConfig, pos: np.ndarray) -> np.ndarray:
    n, h, L = cfg.n, cfg.h, cfg.L
    cut = 10.0 * cfg.v_sigma
    V = np.zeros(cfg.Ng, dtype=np.float64)
    inv2s2 = 1.0 / (2.0 * cfg.v_sigma ** 2)
    for R in pos:
        # every unwrapped index i along an axis is one (grid point, image) pair
        rng_axes = []
        for ax in range(3):
            lo = math.ceil((R[ax] - cut) / h)
            hi = math.floor((R[ax] + cut) / h)
            idx = np.arange(lo, hi + 1)
            rng_axes.append((idx, idx * h - R[ax]))
        (ix, dx), (iy, dy), (iz, dz) = rng_axes
        d2 = dx[:, None, None] ** 2 + dy[None, :, None] ** 2 + dz[None, None, :] ** 2
        mask = d2 <= cut * cut
        val = np.where(mask, np.exp(-d2 * inv2s2), 0.0)
        lin = ((ix[:, None, None] % n) * n + (iy[None, :, None] % n)) * n + (iz[None, None, :] % n)
        np.add.at(V, lin[mask], val[mask])
    return cfg.v_depth * V


def _solid_harmonics(l: int, x, y, z):
    """Real solid harmonics r^l Y_lm up to normalisation, fixed m order."""
    if l == 0:
        return [np.ones_like(x)]
    if l == 1:
        return [x, y, z]
    if l == 2:
        r2 = x * x + y * y + z * z
        return [x * y, y * z, z * x, 0.5 * (x * x - y * y), (3.0 * z * z - r2) / (2.0 * math.sqrt(3.0))]
    raise ValueError(l)


def _projectors(cfg: CellConfig, pos: np.ndarray, rng: np.random.Generator):
    natoms = len(pos)
    n, h, L = cfg.n, cfg.h, cfg.L
    rcut = cfg.rcut_factor * cfg.rc
    if cfg.lmax < 0:
        z32 = np.zeros(natoms + 1, dtype=np.int32)
        return (z32, np.zeros(0, np.int32), z32.copy(), np.zeros(0), np.zeros(0),
                np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(natoms + 1, np.int64), np.zeros((0, 3)))
    if 2.0 * rcut >= L:
        raise ValueError("projector support must be smaller than half the cell")
    supp_ptr = [0]
    supp_all = []
    disp_all = []
    beta_all = []
    beta_ptr = [0]
    proj_ptr = [0]
    D = []
    proj_atom = []
    proj_l = []
    inv2rc2 = 1.0 / (2.0 * cfg.rc ** 2)
    for a, R in enumerate(pos):
        axes = []
        for ax in range(3):
            lo = math.ceil((R[ax] - rcut) / h)
            hi = math.floor((R[ax] + rcut) / h)
            idx = np.arange(lo, hi + 1)
            axes.append((idx % n, idx * h - R[ax]))
        (ix, dx), (iy, dy), (iz, dz) = axes
        DX, DY, DZ = np.meshgrid(dx, dy, dz, indexing="ij")
        IX, IY, IZ = np.meshgrid(ix, iy, iz, indexing="ij")
        d2 = DX ** 2 + DY ** 2 + DZ ** 2
        mask = d2 < rcut * rcut
        lin = ((IX * n + IY) * n + IZ)[mask]
        order = np.argsort(lin, kind="stable")
        lin = lin[order]
        if len(np.unique(lin)) != len(lin):
            raise ValueError("support overlaps its own image")
        x, y, z = DX[mask][order], DY[mask][order], DZ[mask][order]
        g = np.exp(-(x * x + y * y + z * z) * inv2rc2)
        supp_all.append(lin.astype(np.int32))
        disp_all.append(np.stack([x, y, z], axis=1))
        supp_ptr.append(supp_ptr[-1] + len(lin))
        npa = 0
        for l in range(cfg.lmax + 1):
            dval = rng.uniform(-1.0, 1.0)
            for poly in _solid_harmonics(l, x, y, z):
                b = poly * g
                b = b / math.sqrt(float(np.dot(b, b)))
                beta_all.append(b)
                D.append(dval)
                proj_atom.append(a)
                proj_l.append(l)
                npa += 1
        proj_ptr.append(proj_ptr[-1] + npa)
        beta_ptr.append(beta_ptr[-1] + npa * len(lin))
    return (
        np.array(supp_ptr, dtype=np.int32),
        np.concatenate(supp_all).astype(np.int32),
        np.array(proj_ptr, dtype=np.int32),
        np.concatenate(beta_all).astype(np.float64),
        np.array(D, dtype=np.float64),
        np.array(proj_atom, dtype=np.int32),
        np.array(proj_l, dtype=np.int32),
        np.array(beta_ptr, dtype=np.int64),
        np.concatenate(disp_all).astype(np.float64),
    )


def make_cell(cfg: CellConfig, seed: int = 0) -> Cell:
    pos = atom_positions(cfg)
    V = _gaussian_potential(cfg, pos)
    rng = np.random.default_rng(seed)
    (sp, si, pp, beta, D, pa, pl, bp, disp) = _projectors(cfg, pos, rng)
    return Cell(cfg, cfg.L, cfg.n, cfg.h, pos, V, sp, si, pp, beta, D, pa, pl, bp, disp)


def make_x0(cfg: CellConfig, seed: int = 1, nb: Optional[int] = None) -> np.ndarray:
    """Initial block, complex128 of shape (nb, Ng)."""
    nb = cfg.nb if nb is None else nb
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((nb, cfg.Ng))
    im = rng.standard_normal((nb, cfg.Ng))
    return (re + 1j * im) / math.sqrt(2.0)
