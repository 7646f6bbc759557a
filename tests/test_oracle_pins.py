"""Pins of the CPU oracle against closed forms, library routines, invariants
and brute force.  None of these calls the HIP library."""
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.ndimage

import ksinputs as ki
from oracle import cg as ocg
from oracle import cnn as ocnn
from oracle import hamiltonian as oh
from oracle import linalg as ola
from oracle import lobpcg as olob
from oracle import precond as opc

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def tiny_cfg(n=10, L=7.0, lmax=1, positions=((0.1, 0.2, 0.3), (0.6, 0.55, 0.45)), nb=6, **kw):
    return ki.custom_config("tiny", L, n, positions, nb, lmax=lmax, rc=0.61, **kw)


def dense_h_from_generator(cell):
    """Dense H built independently of the oracle: numpy.fft for T, the
    generator's own potential and projector tables."""
    n, L = cell.n, cell.L
    Ng = n ** 3
    Tk = oh.kinetic_diag(n, L)  # closed form |G|^2/2 (also pinned below)
    eye = np.eye(Ng)
    T = np.array([np.fft.ifftn(np.fft.fftn(eye[i].reshape(n, n, n)) * Tk).ravel() for i in range(Ng)]).T
    H = T + np.diag(cell.V)
    for a in range(cell.natoms):
        s0, s1 = cell.atom_supp_ptr[a], cell.atom_supp_ptr[a + 1]
        idx = cell.supp_idx[s0:s1]
        ns = s1 - s0
        for j in range(cell.atom_proj_ptr[a], cell.atom_proj_ptr[a + 1]):
            jj = j - cell.atom_proj_ptr[a]
            b = np.zeros(Ng)
            b[idx] = cell.beta[cell.beta_ptr[a] + jj * ns: cell.beta_ptr[a] + (jj + 1) * ns]
            H += cell.D[j] * np.outer(b, b)
    return 0.5 * (H + H.conj().T)


# ---------------------------------------------------------------- P3, P2, P1


@pytest.mark.parametrize("n", [5, 8, 12, 16])
def test_naive_dft_matches_numpy_fft(n):
    rng = np.random.default_rng(n)
    a = rng.standard_normal((2, n, n, n)) + 1j * rng.standard_normal((2, n, n, n))
    f = oh.dft3(a, n)
    ref = np.fft.fftn(a, axes=(1, 2, 3))
    assert np.abs(f - ref).max() <= 1e-13 * np.abs(ref).max()
    b = oh.dft3(f, n, inverse=True)
    assert np.abs(b - a).max() <= 1e-13 * np.abs(a).max()


@pytest.mark.parametrize("n,L", [(8, 6.74), (9, 5.0), (16, 6.74)])
def test_plane_wave_is_kinetic_eigenvector(n, L):
    x = np.arange(n) * L / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    for m in [(0, 0, 0), (1, 0, 0), (1, -2, 3), (n // 2, 1, -1), (-(n // 2), 0, 2)]:
        g = [2 * math.pi / L * mi for mi in m]
        pw = np.exp(1j * (g[0] * X + g[1] * Y + g[2] * Z)).ravel()[None]
        mw = [((mi + n // 2) % n) - n // 2 if n % 2 == 0 else ((mi + (n - 1) // 2) % n) - (n - 1) // 2 for mi in m]
        expect = 0.5 * sum((2 * math.pi / L * mi) ** 2 for mi in mw)
        tpw = oh.apply_t(pw, n, L)
        assert np.abs(tpw - expect * pw).max() <= 1e-11 * max(1.0, expect)


def test_free_electron_spectrum_closed_form():
    # V = 0, no projectors: eigenvalues are (1/2)(2 pi/L)^2 |m|^2
    L, n = 6.74, 16
    q = 0.5 * (2 * math.pi / L) ** 2
    assert abs(q - 0.43452) < 5e-6
    levels = np.array([0, 1, 2, 3, 4, 5]) * q
    mult = [1, 6, 12, 8, 6, 24]
    expect = np.repeat(levels, mult)
    oc = oh.OracleCell(n, L, np.zeros(n ** 3), [], [], np.zeros(0))
    cfg = ki.custom_config("fe", L, n, [(0, 0, 0)], 19)
    X0 = ki.make_x0(cfg)
    st, _ = olob.run(oc, X0, 19, tol=1e-9, maxit=300, precond=olob.tpa_preconditioner(oc))
    assert np.abs(st.theta - expect[:19]).max() <= 1e-10


# ---------------------------------------------------------------- geometry


def test_oracle_recomputes_generator_potential_and_projectors():
    cfg = ki.config("C2")
    cell = ki.make_cell(cfg)
    oc = oh.oracle_cell(cfg, cell.D)
    assert np.abs(oc.V - cell.V).max() <= 1e-12
    for a in range(cell.natoms):
        s0, s1 = cell.atom_supp_ptr[a], cell.atom_supp_ptr[a + 1]
        ns = s1 - s0
        for j in range(cell.atom_proj_ptr[a], cell.atom_proj_ptr[a + 1]):
            jj = j - cell.atom_proj_ptr[a]
            np.testing.assert_array_equal(oc.proj_supp[j], cell.supp_idx[s0:s1])
            b = cell.beta[cell.beta_ptr[a] + jj * ns: cell.beta_ptr[a] + (jj + 1) * ns]
            assert np.abs(oc.proj_val[j] - b).max() <= 1e-12
    # the displacements the Bloch phases use: the oracle's own minimum image
    _, _, disp = oh.oracle_projectors(cfg, oh.oracle_positions(cfg), with_disp=True)
    for a in range(cell.natoms):
        s0, s1 = cell.atom_supp_ptr[a], cell.atom_supp_ptr[a + 1]
        assert np.abs(disp[cell.atom_proj_ptr[a]] - cell.supp_disp[s0:s1]).max() <= 1e-12


# ---------------------------------------------------------------- Bloch vectors (k-points)


def _dense_h(oc):
    Ng = oc.n ** 3
    return oh.apply_h(oc, np.eye(Ng, dtype=np.complex128)).T


def _tiny_cfg(n, L, lmax, rc=0.35, pos=((1.3, 0.7, 2.1),)):
    from types import SimpleNamespace

    return SimpleNamespace(n=n, L=L, v_sigma=0.6, v_depth=-2.0, rcut_factor=4.0, rc=rc, lmax=lmax,
                           lattice="custom", positions=[x / L for p in pos for x in p], a=L, nsc=1)


def _tiny_cell(cfg, D, k=None):
    pos = np.array(cfg.positions, dtype=np.float64).reshape(-1, 3) * cfg.L
    V = oh.oracle_potential(cfg, pos)
    supp, vals, disp = oh.oracle_projectors(cfg, pos, with_disp=True)
    return oh.from_arrays(cfg.n, cfg.L, V, supp, vals, D, k=k, disp=disp)


def test_free_electrons_at_a_bloch_vector_have_the_shifted_spectrum():
    """V = 0, no projectors: H_k is diagonal in G with |G + k|^2 / 2 over the
    grid's wave vectors (closed form), and Hermitian."""
    n, L = 6, 5.0
    k = np.array([0.31, -0.17, 0.05])
    oc = oh.from_arrays(n, L, np.zeros(n ** 3), [], [], [], k=k)
    H = _dense_h(oc)
    assert np.abs(H - H.conj().T).max() <= 1e-12
    m = oh.wrapped_m(n)
    g = 2 * math.pi / L * m
    ref = np.sort((0.5 * ((g[:, None, None] + k[0]) ** 2 + (g[None, :, None] + k[1]) ** 2
                          + (g[None, None, :] + k[2]) ** 2)).ravel())
    assert np.abs(np.linalg.eigvalsh(H) - ref).max() <= 1e-10


def test_supercell_at_gamma_is_the_union_of_the_cell_at_eight_bloch_vectors():
    """Bloch's theorem on the grid: the 2x2x2 supercell (8^3 grid, L = 8) at
    k = 0 has exactly the eigenvalues of the primitive cell (4^3, L = 4, one
    atom with a Gaussian well and s+p projectors) at the eight vectors
    k = (pi / L)(n1, n2, n3), n_i in {0, 1}: the kinetic sets |G + k|^2 / 2
    tile the supercell's wave vectors and the projector phases exp(-i k.d)
    carry the images.  A wrong sign or a dropped phase breaks it."""
    L = 4.0
    cfg = _tiny_cfg(4, L, 1)
    rng = np.random.default_rng(21)
    D = rng.uniform(-1, 1, 4)
    ev = []
    for n1 in (0, 1):
        for n2 in (0, 1):
            for n3 in (0, 1):
                k = math.pi / L * np.array([n1, n2, n3], dtype=np.float64)
                H = _dense_h(_tiny_cell(cfg, D, k))
                assert np.abs(H - H.conj().T).max() <= 1e-12
                ev.append(np.linalg.eigvalsh(H))
    ev = np.sort(np.concatenate(ev))
    R = np.array([1.3, 0.7, 2.1])
    pos = [tuple(R + L * np.array([i, j, q])) for i in (0, 1) for j in (0, 1) for q in (0, 1)]
    scfg = _tiny_cfg(8, 2 * L, 1, pos=pos)
    sup = _tiny_cell(scfg, np.tile(D, 8))
    es = np.linalg.eigvalsh(_dense_h(sup))
    assert np.abs(es - ev).max() <= 1e-10


def test_spectrum_at_minus_k_equals_spectrum_at_k():
    """A real potential and real projector radial parts give
    H_{-k} = conj(H_k): the same eigenvalues at k and -k, different from the
    Gamma point's."""
    cfg = _tiny_cfg(5, 4.5, 1)
    D = np.array([0.7, -0.4, -0.4, -0.4])
    k = np.array([0.4, 0.1, -0.25])
    Hp = _dense_h(_tiny_cell(cfg, D, k))
    Hm = _dense_h(_tiny_cell(cfg, D, -k))
    assert np.abs(Hm - np.conj(Hp)).max() <= 1e-12
    ep, em = np.linalg.eigvalsh(Hp), np.linalg.eigvalsh(Hm)
    e0 = np.linalg.eigvalsh(_dense_h(_tiny_cell(cfg, D)))
    assert np.abs(ep - em).max() <= 1e-10
    assert np.abs(ep - e0).max() > 1e-3


def test_oracle_lobpcg_at_a_bloch_vector_matches_dense_eigh():
    """The oracle's LOBPCG (TPA on |G + k|^2 / 2) at k on a 6^3 cell with s+p
    projectors: lowest eigenvalues against a dense eigensolve of H_k."""
    cfg = _tiny_cfg(6, 5.0, 1, rc=0.4)
    D = np.array([0.9, -0.5, -0.5, -0.5])
    k = np.array([0.2, -0.35, 0.1])
    oc = _tiny_cell(cfg, D, k)
    ref = np.linalg.eigvalsh(_dense_h(oc))
    rng = np.random.default_rng(5)
    X0 = rng.standard_normal((8, 216)) + 1j * rng.standard_normal((8, 216))
    st, _ = olob.run(oc, X0, 6, 1e-9, 300, olob.tpa_preconditioner(oc))
    assert np.abs(st.theta[:6] - ref[:6]).max() <= 1e-10


def test_config_sizes_match_derived_table():
    c2, c3, c4 = ki.config("C2"), ki.config("C3"), ki.config("C4")
    assert c2.Ng == 110592 and c3.Ng == 884736 and c4.Ng == 1404928
    assert abs(c3.L - 20.22) < 1e-9 and abs(c4.L - 23.92) < 1e-9
    cell = ki.make_cell(c2)
    assert cell.natoms == 64 and cell.nproj == 256
    per_atom = np.diff(cell.atom_supp_ptr)
    assert 11500 < per_atom.mean() < 12700  # about 12.1k points inside 4 bohr


# ---------------------------------------------------------------- P8, P9


def random_hpd(n, rng, cond=1e3):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    s = np.logspace(0, -math.log10(cond), n)
    return (Q * s) @ Q.conj().T


@pytest.mark.parametrize("n", [1, 2, 5, 17, 48])
def test_cholesky_and_triangular_solves_match_library(n):
    rng = np.random.default_rng(n)
    S = random_hpd(n, rng)
    L, info = ola.cholesky_lower(S)
    assert info == 0
    assert np.abs(L - np.linalg.cholesky(S)).max() <= 1e-12
    B = rng.standard_normal((n, 3)) + 1j * rng.standard_normal((n, 3))
    Y = ola.solve_lower(L, B)
    assert np.abs(Y - scipy.linalg.solve_triangular(L, B, lower=True)).max() <= 1e-10 * np.abs(Y).max()
    Xs = ola.solve_lower_conj_t(L, B)
    ref = scipy.linalg.solve_triangular(L, B, lower=True, trans="C")
    assert np.abs(Xs - ref).max() <= 1e-10 * np.abs(ref).max()


def test_cholesky_reports_failing_minor():
    S = np.diag([1.0, 2.0, -1.0, 3.0]).astype(complex)
    _, info = ola.cholesky_lower(S)
    assert info == 3
    rng = np.random.default_rng(0)
    A = rng.standard_normal((6, 4)) + 1j * rng.standard_normal((6, 4))
    A = np.concatenate([A, A[:, 1:2]], axis=1)  # duplicated column
    _, info = ola.cholesky_lower(A.conj().T @ A)
    assert info == 5


@pytest.mark.parametrize("n", [1, 2, 3, 16, 47, 64])
def test_jacobi_matches_numpy_eigh(n):
    rng = np.random.default_rng(100 + n)
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    A = A + A.conj().T
    w, Z = ola.jacobi_eigh(A)
    ref = np.linalg.eigvalsh(A)
    assert np.abs(w - ref).max() <= 1e-13 * np.abs(ref).max() * max(1, n)
    assert np.abs(Z.conj().T @ Z - np.eye(n)).max() <= 1e-13 * max(1, n)
    assert np.abs(A @ Z - Z * w).max() <= 1e-12 * np.abs(ref).max() * max(1, n)


def test_jacobi_diagonal_input_unchanged():
    d = np.array([3.0, -1.0, 2.0, 0.5])
    w, Z = ola.jacobi_eigh(np.diag(d).astype(complex))
    np.testing.assert_array_equal(w, np.sort(d))
    assert np.abs(np.abs(Z) - np.abs(Z).round()).max() == 0.0


@pytest.mark.parametrize("n,nev", [(12, 4), (48, 16), (90, 30)])
def test_two_trsm_reduction_matches_generalised_library_solve(n, nev):
    rng = np.random.default_rng(7 * n)
    S = random_hpd(n, rng, cond=1e4)
    Hm = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Hm = Hm + Hm.conj().T
    w, C, info = ola.hegv_two_trsm(Hm, S, nev)
    assert info == 0
    ref = scipy.linalg.eigh(Hm, S, eigvals_only=True)[:nev]
    assert np.abs(w - ref).max() <= 1e-12 * np.abs(ref).max() * 10
    assert np.abs(C.conj().T @ S @ C - np.eye(nev)).max() <= 1e-10
    assert np.abs(Hm @ C - S @ C * w).max() <= 1e-9 * np.abs(Hm).max()


def test_two_trsm_reports_indefinite_overlap():
    n = 6
    S = np.eye(n, dtype=complex)
    S[3, 3] = -1.0
    _, _, info = ola.hegv_two_trsm(np.eye(n, dtype=complex), S, 2)
    assert info == n + 4


# ---------------------------------------------------------------- P5, P6, P7, P4, P11


@pytest.fixture(scope="module")
def tiny():
    cfg = tiny_cfg()
    cell = ki.make_cell(cfg)
    oc = oh.oracle_cell(cfg, cell.D)
    return cfg, cell, oc


def test_hamiltonian_is_hermitian(tiny):
    cfg, cell, oc = tiny
    rng = np.random.default_rng(3)
    a = rng.standard_normal((2, cfg.Ng)) + 1j * rng.standard_normal((2, cfg.Ng))
    Ha = oh.apply_h(oc, a)
    lhs = np.vdot(a[0], Ha[1])
    rhs = np.vdot(Ha[0], a[1])
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


@pytest.mark.parametrize("n,lmax,npos", [(8, 1, 1), (10, 1, 2), (12, 2, 2)])
def test_lobpcg_matches_brute_force_dense_eigh(n, lmax, npos):
    pos = ((0.1, 0.2, 0.3), (0.6, 0.55, 0.45))[:npos]
    L = 7.0 if n < 12 else 8.0
    cfg = tiny_cfg(n=n, L=L, lmax=lmax, positions=pos, nb=8)
    cell = ki.make_cell(cfg)
    Hd = dense_h_from_generator(cell)
    ref = np.linalg.eigvalsh(Hd)
    oc = oh.oracle_cell(cfg, cell.D)
    # oracle H-apply equals the dense matrix on random vectors
    rng = np.random.default_rng(n)
    v = rng.standard_normal((3, cfg.Ng)) + 1j * rng.standard_normal((3, cfg.Ng))
    assert np.abs(oh.apply_h(oc, v) - (Hd @ v.T).T).max() <= 1e-11 * np.abs(Hd).max()
    st, hist = olob.run(oc, ki.make_x0(cfg), 8, tol=1e-9, maxit=400, precond=olob.tpa_preconditioner(oc))
    assert hist[-1][1][:8].max() <= 1e-9
    assert np.abs(st.theta - ref[:8]).max() <= 1e-10
    # S-orthonormality of the final block (S = I)
    G = np.conj(st.X) @ st.X.T
    assert np.abs(G - np.eye(8)).max() <= 1e-12


def test_constant_potential_shift_and_zero_coupling(tiny):
    cfg, cell, oc = tiny
    X0 = ki.make_x0(cfg)
    pc = olob.tpa_preconditioner
    st0, _ = olob.run(oc, X0, 6, 1e-9, 300, pc(oc))
    oc_shift = oh.OracleCell(oc.n, oc.L, oc.V + 0.37, oc.proj_supp, oc.proj_val, oc.D)
    st1, _ = olob.run(oc_shift, X0, 6, 1e-9, 300, pc(oc_shift))
    assert np.abs(st1.theta - st0.theta - 0.37).max() <= 1e-10
    # D = 0 reduces to the local-only problem
    oc_d0 = oh.OracleCell(oc.n, oc.L, oc.V, oc.proj_supp, oc.proj_val, np.zeros_like(oc.D))
    oc_loc = oh.OracleCell(oc.n, oc.L, oc.V, [], [], np.zeros(0))
    a, _ = olob.run(oc_d0, X0, 6, 1e-9, 300, pc(oc_d0))
    b, _ = olob.run(oc_loc, X0, 6, 1e-9, 300, pc(oc_loc))
    assert np.abs(a.theta - b.theta).max() <= 1e-10


def test_translation_and_permutation_invariance():
    base = ((0.1, 0.2, 0.3), (0.6, 0.55, 0.45))
    n, L = 10, 7.0
    cfg = tiny_cfg(n=n, L=L, positions=base)
    cell = ki.make_cell(cfg)
    ref = np.linalg.eigvalsh(dense_h_from_generator(cell))[:10]
    # translate every atom by a whole grid vector (2, -1, 3) * h
    sh = np.array([2, -1, 3]) / n
    moved = tuple(tuple((np.array(p) + sh) % 1.0) for p in base)
    cfg2 = tiny_cfg(n=n, L=L, positions=moved)
    cell2 = ki.make_cell(cfg2)
    cell2.D[:] = cell.D
    w2 = np.linalg.eigvalsh(dense_h_from_generator(cell2))[:10]
    assert np.abs(w2 - ref).max() <= 1e-11
    # permute the atoms together with their couplings
    cfg3 = tiny_cfg(n=n, L=L, positions=base[::-1])
    cell3 = ki.make_cell(cfg3)
    npa = cell.nproj // 2
    cell3.D[:npa], cell3.D[npa:] = cell.D[npa:], cell.D[:npa]
    w3 = np.linalg.eigvalsh(dense_h_from_generator(cell3))[:10]
    assert np.abs(w3 - ref).max() <= 1e-11


# ---------------------------------------------------------------- P10


def test_rank_one_projector_interlaces_and_solves_secular_equation():
    cfg = tiny_cfg(n=8, L=7.0, lmax=0, positions=((0.3, 0.4, 0.5),), nb=6)
    cell = ki.make_cell(cfg)
    cell.D[:] = 0.8
    oc = oh.oracle_cell(cfg, cell.D)
    oc_loc = oh.OracleCell(oc.n, oc.L, oc.V, [], [], np.zeros(0))
    # local spectrum by brute force (dense from numpy.fft)
    Hd = dense_h_from_generator(cell)
    b = np.zeros(cfg.Ng)
    b[oc.proj_supp[0]] = oc.proj_val[0]
    H0 = Hd - 0.8 * np.outer(b, b)
    lam0, phi = np.linalg.eigh(H0)
    lam, _ = np.linalg.eigh(Hd)
    # interlacing for a positive rank-one update
    assert np.all(lam[:-1] >= lam0[:-1] - 1e-12) and np.all(lam[:-1] <= lam0[1:] + 1e-12)
    # oracle LOBPCG reproduces the updated values
    st, _ = olob.run(oc, ki.make_x0(cfg), 6, 1e-9, 300, olob.tpa_preconditioner(oc))
    assert np.abs(st.theta - lam[:6]).max() <= 1e-10
    # every eigenvalue with nonzero weight solves 1 + D sum |<phi|b>|^2/(lam_k - lam) = 0
    wgt = np.abs(phi.T @ b) ** 2
    for x in st.theta[:3]:
        sec = 1.0 + 0.8 * np.sum(wgt / (lam0 - x))
        assert abs(sec) <= 1e-6 * np.sum(wgt / np.abs(lam0 - x))
    del oc_loc


# ---------------------------------------------------------------- P12


def test_residual_bounds_certify_eigenvalues(tiny):
    cfg, cell, oc = tiny
    ref = np.linalg.eigvalsh(dense_h_from_generator(cell))
    st, _ = olob.run(oc, ki.make_x0(cfg), 6, 1e-4, 300, olob.tpa_preconditioner(oc))
    R, res = olob.residual(st)
    for i in range(6):
        # Krylov-Weinstein: some eigenvalue within ||r|| of theta
        assert np.min(np.abs(ref - st.theta[i])) <= res[i] * (1 + 1e-9)
    # Kato-Temple for the lowest (gap to the second level)
    gap = ref[1] - st.theta[0]
    assert st.theta[0] - ref[0] <= res[0] ** 2 / gap * (1 + 1e-6) + 1e-14


# ---------------------------------------------------------------- P14


def test_tpa_on_plane_wave_is_the_polynomial():
    n, L = 12, 6.0
    x = np.arange(n) * L / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    m = (2, -1, 3)
    g = [2 * math.pi / L * mi for mi in m]
    pw = np.exp(1j * (g[0] * X + g[1] * Y + g[2] * Z)).ravel()[None]
    E = np.array([1.7])
    w = opc.tpa_apply(pw, E, n, L)
    xg = 0.5 * sum(gi * gi for gi in g) / E[0]
    k = (27 + 18 * xg + 12 * xg ** 2 + 8 * xg ** 3) / (27 + 18 * xg + 12 * xg ** 2 + 8 * xg ** 3 + 16 * xg ** 4)
    assert np.abs(w - k * pw).max() <= 1e-12
    assert opc.tpa_polynomial(np.array([0.0]))[0] == 1.0


def test_band_kinetic_energy_of_plane_wave():
    n, L = 8, 5.0
    x = np.arange(n) * L / n
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    g = 2 * math.pi / L
    pw = (np.exp(1j * g * (X + 2 * Y)).ravel() / math.sqrt(n ** 3))[None]
    E = opc.band_kinetic_energy(pw, n, L)
    assert abs(E[0] - 0.5 * g * g * 5) <= 1e-12


# ---------------------------------------------------------------- P15


def test_conv_matches_scipy_correlate_wrap():
    rng = np.random.default_rng(5)
    n = 6
    inp = rng.standard_normal((3, n, n, n))
    w = rng.standard_normal((4, 3, 3, 3, 3))
    b = rng.standard_normal(4)
    out = ocnn.conv3d(inp, w, b)
    for o in range(4):
        ref = np.full((n, n, n), b[o])
        for i in range(3):
            ref += scipy.ndimage.correlate(inp[i], w[o, i], mode="wrap")
        assert np.abs(out[o] - ref).max() <= 1e-12


def test_cnn_backward_matches_finite_differences():
    rng = np.random.default_rng(6)
    n = 5
    params = ocnn.init_params(2, channels=(3, 4, 4, 2))
    x = rng.standard_normal((3, n, n, n))
    t = rng.standard_normal((2, n, n, n))

    def loss_of(ps, xx):
        y, _ = ocnn.forward(ps, xx)
        return ocnn.normalised_loss(y, t)[0]

    y, cache = ocnn.forward(params, x)
    _, gy = ocnn.normalised_loss(y, t)
    grads, gx = ocnn.backward(params, cache, gy)
    eps = 1e-6
    for k, idx in [(0, (1, 2, 0, 1, 2)), (1, (3, 0, 2, 2, 1)), (2, (1, 3, 0, 0, 0))]:
        w = params[k][0]
        wp = w.copy(); wp[idx] += eps
        wm = w.copy(); wm[idx] -= eps
        pp = list(params); pp[k] = (wp, params[k][1])
        pm = list(params); pm[k] = (wm, params[k][1])
        fd = (loss_of(pp, x) - loss_of(pm, x)) / (2 * eps)
        assert abs(fd - grads[k][0][idx]) <= 1e-6 * max(1e-3, abs(fd))
    for k in range(3):
        bp = params[k][1].copy(); bp[1] += eps
        bm = params[k][1].copy(); bm[1] -= eps
        pp = list(params); pp[k] = (params[k][0], bp)
        pm = list(params); pm[k] = (params[k][0], bm)
        fd = (loss_of(pp, x) - loss_of(pm, x)) / (2 * eps)
        assert abs(fd - grads[k][1][1]) <= 1e-6 * max(1e-3, abs(fd))
    xp = x.copy(); xp[0, 1, 2, 3] += eps
    xm = x.copy(); xm[0, 1, 2, 3] -= eps
    fd = (loss_of(params, xp) - loss_of(params, xm)) / (2 * eps)
    assert abs(fd - gx[0, 1, 2, 3]) <= 1e-6 * max(1e-3, abs(fd))


def test_residual_network_with_zero_last_layer_is_identity_on_its_input():
    # a zero last layer makes the residual variant return its first two
    # input channels exactly (it then reproduces the unlearned direction)
    rng = np.random.default_rng(8)
    n = 5
    params = ocnn.init_params(2, channels=(3, 4, 4, 2))
    params[2] = (np.zeros_like(params[2][0]), np.zeros_like(params[2][1]))
    x = rng.standard_normal((3, n, n, n))
    out, _ = ocnn.forward_residual(params, x)
    assert np.array_equal(out, x[:2])
    # and with any weights it differs from the plain network by x[:2]
    p2 = ocnn.init_params(3, channels=(3, 4, 4, 2))
    a, _ = ocnn.forward(p2, x)
    b, _ = ocnn.forward_residual(p2, x)
    assert np.abs((b - a) - x[:2]).max() <= 1e-12


def test_adam_first_step_is_lr_times_sign():
    p = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    p1, _, _ = ocnn.adam_update(p, g, np.zeros(3), np.zeros(3), 1, lr=1e-3)
    assert np.allclose(p - p1, 1e-3 * np.sign(g), rtol=1e-4)


# ---------------------------------------------------------------- P16


def test_projected_cg_matches_lstsq(tiny):
    cfg, cell, oc = tiny
    Hd = dense_h_from_generator(cell)
    st, _ = olob.run(oc, ki.make_x0(cfg), 6, 1e-9, 300, olob.tpa_preconditioner(oc))
    X = st.X
    i = 2
    theta = st.theta[i]
    rng = np.random.default_rng(11)
    r = rng.standard_normal(cfg.Ng) + 1j * rng.standard_normal(cfg.Ng)
    P = np.eye(cfg.Ng) - X.T @ np.conj(X)
    r = P @ r
    t, its, ok = ocg.projected_cg(lambda v: oh.apply_h(oc, v), X, theta, r, rtol=1e-12, maxit=2000)
    A = P @ (Hd - theta * np.eye(cfg.Ng)) @ P
    ref, *_ = np.linalg.lstsq(A, r, rcond=1e-12)
    ref = P @ ref
    assert ok
    assert np.linalg.norm(t - ref) <= 1e-8 * np.linalg.norm(ref)


def test_bfloat16_rounding_matches_torch_conversion():
    """The oracle's nearest-bfloat16 rounding (ties to even) against torch's
    float32 -> bfloat16 conversion: random magnitudes, exact ties of both
    parities and signs, subnormals, overflow to infinity, zeros and
    infinities; NaN stays NaN."""
    import torch

    rng = np.random.default_rng(11)
    x = (rng.standard_normal(50000) * 10.0 ** rng.integers(-38, 38, 50000)).astype(np.float32)
    hi = rng.integers(0, 1 << 16, 4000, dtype=np.uint64)
    ties = ((hi << 16) | 0x8000).astype(np.uint32).view(np.float32)  # exactly half-way
    tiny = (rng.integers(1, 1 << 23, 2000, dtype=np.uint64)).astype(np.uint32).view(np.float32)  # subnormals
    special = np.array([0.0, -0.0, np.inf, -np.inf, np.finfo(np.float32).max, -np.finfo(np.float32).max,
                        np.float32(1.0) + np.float32(2.0 ** -8), 3.0, -7.5e-39], dtype=np.float32)
    allv = np.concatenate([x, ties, -ties, tiny, special])
    allv = allv[np.isfinite(allv) | np.isinf(allv)]
    ref = torch.from_numpy(allv).to(torch.bfloat16).to(torch.float64).numpy()
    got = ocnn.round_bf16(allv)
    assert np.array_equal(got, ref)
    # representable: the low 16 bits of the binary32 pattern are zero
    assert np.all((got.astype(np.float32).view(np.uint32) & 0xFFFF) == 0)
    assert np.isnan(ocnn.round_bf16(np.array([np.nan], dtype=np.float32))[0])


def test_bfloat16_network_mode_reduces_to_the_exact_network_on_representable_data():
    """The bfloat16 mode of the network rounds the two operands of every
    convolution product.  On one layer whose input, weights and output
    gradient are bfloat16 values already, nothing rounds: forward and
    backward equal the FP64 network (pinned above against scipy and finite
    differences) exactly.  On three layers with generic data the two modes
    differ, by about the bfloat16 unit 2^-8 relative."""
    rng = np.random.default_rng(12)
    n = 5
    w = ocnn.round_bf16(rng.uniform(-0.3, 0.3, (2, 3, 3, 3, 3)))
    b = rng.standard_normal(2)
    x = ocnn.round_bf16(rng.standard_normal((3, n, n, n)))
    g = ocnn.round_bf16(rng.standard_normal((2, n, n, n)))
    one = [(w, b)]
    y0, c0 = ocnn.forward(one, x)
    y1, c1 = ocnn.forward(one, x, bf16=True)
    assert np.array_equal(y0, y1)
    (gr0,), gx0 = ocnn.backward(one, c0, g)
    (gr1,), gx1 = ocnn.backward(one, c1, g, bf16=True)
    assert np.array_equal(gr0[0], gr1[0]) and np.array_equal(gr0[1], gr1[1]) and np.array_equal(gx0, gx1)
    params = ocnn.init_params(2, channels=(3, 4, 4, 2))
    x = rng.standard_normal((3, n, n, n))
    ya, ca = ocnn.forward(params, x)
    yb, cb = ocnn.forward(params, x, bf16=True)
    d = np.abs(ya - yb).max() / np.abs(ya).max()
    assert 1e-5 < d < 3e-2
    ga, _ = ocnn.backward(params, ca, ya)
    gb, _ = ocnn.backward(params, cb, ya, bf16=True)
    for (dwa, dba), (dwb, dbb) in zip(ga, gb):
        dw = np.abs(dwa - dwb).max() / np.abs(dwa).max()
        assert 1e-5 < dw < 3e-2
        assert np.abs(dba - dbb).max() <= 3e-2 * np.abs(dba).max()


# ---------------------------------------------------------------- deflating Cholesky (P8 for a singular overlap)


def _dependent_basis(rng, N=40, m=9, dep=((4, (1, 2)), (7, (0, 4)))):
    """N x m complex basis whose column k (for each (k, (i, j)) in dep) is a
    combination of columns i and j before it."""
    V = rng.standard_normal((N, m)) + 1j * rng.standard_normal((N, m))
    for k, (i, j) in dep:
        V[:, k] = (0.3 - 0.7j) * V[:, i] + 1.9 * V[:, j]
    return V


def test_deflating_cholesky_equals_plain_cholesky_on_positive_definite_input():
    rng = np.random.default_rng(41)
    S = random_hpd(30, rng, cond=1e6)
    L, dead = ola.cholesky_lower_deflate(S)
    assert not dead.any()
    np.testing.assert_allclose(L, np.linalg.cholesky(S), rtol=0, atol=1e-12 * np.abs(S).max())


def test_deflating_cholesky_drops_exactly_the_dependent_columns():
    rng = np.random.default_rng(42)
    V = _dependent_basis(rng)
    S = V.conj().T @ V
    L, dead = ola.cholesky_lower_deflate(S)
    assert np.nonzero(dead)[0].tolist() == [4, 7]
    live = np.nonzero(~dead)[0]
    # the live part is the library Cholesky of the live overlap; dead columns are unit vectors
    ref = np.linalg.cholesky(S[np.ix_(live, live)])
    np.testing.assert_allclose(L[np.ix_(live, live)], ref, rtol=0, atol=1e-11 * np.abs(S).max())
    for k in (4, 7):
        e = np.zeros(S.shape[0]); e[k] = 1.0
        np.testing.assert_array_equal(L[:, k], e)


def test_deflated_reduction_gives_the_ritz_values_of_the_span():
    """Ritz values of a Hermitian A on span(V) do not depend on the basis:
    the deflated two-solve reduction on the dependent basis equals the
    library generalised solve on an independent basis of the same span."""
    rng = np.random.default_rng(43)
    N, nev = 40, 4
    V = _dependent_basis(rng, N=N)
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N))
    A = A + A.conj().T
    Hs, Ss = V.conj().T @ A @ V, V.conj().T @ V
    w, C, ndead = ola.hegv_two_trsm_deflate(Hs, Ss, nev)
    assert ndead == 2
    keep = [0, 1, 2, 3, 5, 6, 8]
    U = V[:, keep]
    ref = scipy.linalg.eigh(U.conj().T @ A @ U, U.conj().T @ U, eigvals_only=True)[:nev]
    assert np.abs(w - ref).max() <= 1e-10 * np.abs(ref).max()
    X = V @ C
    assert np.abs(X.conj().T @ X - np.eye(nev)).max() <= 1e-9
    # Galerkin condition: the residual is orthogonal to the span
    assert np.abs(V.conj().T @ (A @ X - X * w)).max() <= 1e-9 * np.abs(A).max() * np.abs(V).max()
    assert np.abs(C[[4, 7]]).max() == 0.0


def test_orthonormalise_block_zeroes_a_dependent_column_and_keeps_the_span():
    rng = np.random.default_rng(44)
    Vm = _dependent_basis(rng, N=50, m=6, dep=((3, (0, 1)),))
    B = Vm.T.copy()  # band-major: rows are the columns
    Bq, _, ndead = olob.orthonormalise_block(B)
    assert ndead == 1
    assert np.abs(Bq[3]).max() == 0.0
    live = [0, 1, 2, 4, 5]
    G = Bq[live].conj() @ Bq[live].T
    assert np.abs(G - np.eye(5)).max() <= 1e-12
    # same span: projecting the original columns on the new ones loses nothing
    Q = Bq[live].T
    resid = Vm - Q @ (Q.conj().T @ Vm)
    assert np.abs(resid).max() <= 1e-10 * np.abs(Vm).max()


# ---------------------------------------------------------------- Adam beyond the first step; geometry in closed form


def test_adam_constant_gradient_moves_by_lr_sign_at_every_step():
    """With a constant gradient the bias-corrected moments equal g and g^2
    exactly at every t (m_t = (1 - b1^t) g, v_t = (1 - b2^t) g^2), so each
    step is lr * g / (|g| + eps).  A wrong decay or bias correction breaks
    this from t = 2 on."""
    p = np.array([1.0, -2.0, 0.5, 3.0])
    g = np.array([0.3, -4.0, 1e-3, 250.0])
    m = np.zeros(4)
    v = np.zeros(4)
    for t in range(1, 51):
        p1, m, v = ocnn.adam_update(p, g, m, v, t, lr=1e-3)
        assert np.allclose(p - p1, 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=0), t
        p = p1


def test_adam_two_steps_worked_by_hand():
    """g1 = 1 then g2 = -2, lr 0.1, from m = v = 0.  Step 1 moves by -0.1.
    Step 2: m2 = 0.9*0.1 - 0.2 = -0.11, v2 = 0.999*0.001 + 0.004 = 0.004999,
    m2 / (1 - 0.81) = -0.578947..., v2 / (1 - 0.998001) = 2.500750...,
    sqrt = 1.581376..., so the step is +0.1 * 0.578947 / 1.581376 = +0.036610."""
    p0 = np.array([0.0])
    p1, m, v = ocnn.adam_update(p0, np.array([1.0]), np.zeros(1), np.zeros(1), 1, lr=0.1)
    assert abs(p1[0] - (-0.1)) <= 1e-9
    p2, m, v = ocnn.adam_update(p1, np.array([-2.0]), m, v, 2, lr=0.1)
    assert abs(m[0] - (-0.11)) <= 1e-15 and abs(v[0] - 0.004999) <= 1e-15
    assert abs((p2[0] - p1[0]) - 0.036610) <= 2e-6


def test_potential_at_an_atom_on_a_grid_point_is_the_image_shell_sum():
    """One atom on a grid point of a cubic cell, L = 4.1, sigma = 0.8: the
    images within 10 sigma = 8 bohr are the atom itself and the shells
    |T| = L (6), L sqrt(2) (12) and L sqrt(3) (8); |T| = 2L = 8.2 is out.
    So V(R) = A (1 + 6 e^{-L^2/2s^2} + 12 e^{-2L^2/2s^2} + 8 e^{-3L^2/2s^2})."""
    L, s, A, n = 4.1, 0.8, -2.0, 10
    cfg = ki.custom_config("one", L, n, ((0.3, 0.5, 0.7),), 1, v_depth=A, v_sigma=s)
    pos = oh.oracle_positions(cfg)
    V = oh.oracle_potential(cfg, pos)
    q = lambda k: math.exp(-k * L * L / (2 * s * s))  # noqa: E731
    expect = A * (1 + 6 * q(1) + 12 * q(2) + 8 * q(3))
    idx = (3 * n + 5) * n + 7
    assert abs(V[idx] - expect) <= 1e-14 * abs(expect)
    # a neighbouring grid point along z: the same shells seen from dz = h
    h = L / n
    shells = [(0, 0, 0)] + [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1) if (a, b, c) != (0, 0, 0)]
    tot = 0.0
    for a, b, c in shells:
        d2 = (a * L) ** 2 + (b * L) ** 2 + (h - c * L) ** 2
        if d2 <= (10 * s) ** 2:
            tot += math.exp(-d2 / (2 * s * s))
    assert abs(V[idx + 1] - A * tot) <= 1e-14 * abs(A * tot)


def test_projector_values_follow_the_gaussian_and_solid_harmonic_shapes():
    """Atom on a grid point: s values at two support points have the ratio
    exp(-(r1^2 - r2^2)/(2 rc^2)); p_x is odd in x and equals x times the s
    shape up to one constant; d_xy vanishes on the coordinate planes; every
    projector is normalised on the grid; the support is every grid point
    with minimum-image distance below 4 rc (counted by brute force)."""
    L, n, rc = 7.0, 14, 0.55
    cfg = ki.custom_config("one", L, n, ((0.5, 0.5, 0.5),), 1, lmax=2, rc=rc)
    pos = oh.oracle_positions(cfg)
    supp, vals = oh.oracle_projectors(cfg, pos)
    assert len(supp) == 9
    h = L / n
    # brute-force support: integer offsets from the atom's grid point (7, 7, 7)
    offs = [(a, b, c) for a in range(-n // 2, n // 2) for b in range(-n // 2, n // 2) for c in range(-n // 2, n // 2)
            if (a * a + b * b + c * c) * h * h < (4 * rc) ** 2]
    assert len(supp[0]) == len(offs)
    lin = {((7 + a) * n + 7 + b) * n + 7 + c: (a * h, b * h, c * h) for a, b, c in offs}
    assert set(supp[0].tolist()) == set(lin)
    xyz = np.array([lin[i] for i in supp[0].tolist()])
    r2 = np.sum(xyz * xyz, axis=1)
    bs, bx, bxy = vals[0], vals[1], vals[4]
    i0 = int(np.argmin(r2))
    ratio = bs / bs[i0]
    assert np.abs(ratio - np.exp(-(r2 - r2[i0]) / (2 * rc * rc))).max() <= 1e-13
    nz = np.abs(xyz[:, 0]) > 0
    c = bx[nz] / (xyz[nz, 0] * bs[nz])
    assert np.abs(c - c[0]).max() <= 1e-12 * abs(c[0])
    assert np.abs(bx[~nz]).max() == 0.0
    plane = (np.abs(xyz[:, 0]) < 1e-12) | (np.abs(xyz[:, 1]) < 1e-12)
    assert np.abs(bxy[plane]).max() <= 1e-15
    for v in vals:
        assert abs(float(np.sum(v * v)) - 1.0) <= 1e-13


# ---------------------------------------------------------------- SCF pieces
from oracle import scf as oscf  # noqa: E402


def test_hartree_of_a_plane_wave_density_is_four_pi_over_g2():
    """rho = c + a cos(G.r) gives V_H = 4 pi a / |G|^2 cos(G.r) (the constant
    is removed by the neutralising background)."""
    n, L = 10, 6.0
    h = L / n
    idx = np.arange(n) * h
    X, Y, Z = np.meshgrid(idx, idx, idx, indexing="ij")
    G = 2 * math.pi / L * np.array([1, 2, -1])
    ph = G[0] * X + G[1] * Y + G[2] * Z
    c, a = 0.3, 0.05
    dV = h ** 3
    nper = ((c + a * np.cos(ph)) * dV).ravel()
    vh = oscf.hartree(nper, n, L)
    expect = (4 * math.pi * a / float(G @ G) * np.cos(ph)).ravel()
    assert np.abs(vh - expect).max() <= 1e-12 * np.abs(expect).max()


def test_lda_exchange_is_the_electron_gas_constant_and_potentials_are_derivatives():
    """Slater exchange per electron is -0.458165/r_s (the uniform electron
    gas, 3/4 (9/(4 pi^2))^(1/3)); the potentials are the density derivatives
    of rho * e_xc (central differences), on both sides of r_s = 1."""
    rs = np.array([0.3, 0.7, 0.99, 1.01, 2.0, 5.0, 12.0])
    rho = 3.0 / (4.0 * math.pi * rs ** 3)
    exc, vxc = oscf.lda_xc(rho)
    ex = -0.75 * np.cbrt(3.0 * rho / math.pi)
    np.testing.assert_allclose(ex * rs, -0.458165293283143, rtol=1e-12)
    h = 1e-6 * rho
    ep, _ = oscf.lda_xc(rho + h)
    em, _ = oscf.lda_xc(rho - h)
    deriv = ((rho + h) * ep - (rho - h) * em) / (2 * h)
    np.testing.assert_allclose(vxc, deriv, rtol=1e-7)
    e0, v0 = oscf.lda_xc(np.array([0.0, 1e-40]))
    assert np.all(e0 == 0.0) and np.all(v0 == 0.0)


def test_density_counts_the_electrons():
    rng = np.random.default_rng(9)
    A = rng.standard_normal((5, 300)) + 1j * rng.standard_normal((5, 300))
    Q, _ = np.linalg.qr(A.T)
    X = Q.T
    occ = np.array([2.0, 2.0, 2.0, 1.0, 0.5])
    n = oscf.density(X, occ)
    assert abs(n.sum() - occ.sum()) <= 1e-12
    assert np.all(n >= 0)


def _dense_eigensolver(nb):
    def solve(cell, X0):
        Hd = np.stack([oh.apply_h(cell, e[None])[0] for e in np.eye(cell.Ng, dtype=complex)], axis=1)
        w, V = np.linalg.eigh(0.5 * (Hd + Hd.conj().T))
        return w[:nb], V[:, :nb].T.copy()
    return solve


def test_scf_with_lobpcg_reaches_the_fixed_point_of_the_scf_with_dense_eigh():
    """The SCF loop's fixed point does not depend on the eigensolver: with the
    oracle's LOBPCG inside it reaches the density and energy of the same loop
    with a dense library eigensolve (8^3 grid, one atom with s and p
    projectors, 5 occupied bands closing a shell: the bare spectrum has a
    gap of 0.18 Ha above the fifth level)."""
    cfg = ki.custom_config("scf8", 5.0, 8, ((0.3, 0.4, 0.5),), 8, lmax=1, rc=0.5)
    cell = ki.make_cell(cfg)
    oc = oh.oracle_cell(cfg, cell.D)
    nocc = 5
    dense = _dense_eigensolver(cfg.nb)
    ref = oscf.run(oc, nocc, dense, None, alpha=0.3, tol=1e-9, maxit=80)

    def lob(cell_v, X0):
        X0 = ki.make_x0(cfg) if X0 is None else X0
        st, _ = olob.run(cell_v, X0, cfg.nb, 1e-10, 300, olob.tpa_preconditioner(cell_v))
        return st.theta, st.X

    got = oscf.run(oc, nocc, lob, None, alpha=0.3, tol=1e-9, maxit=80)
    assert ref.iterations < 80 and got.iterations < 80
    assert np.abs(got.n - ref.n).max() <= 1e-8
    assert abs(got.energy - ref.energy) <= 1e-9
    assert np.abs(got.theta[:nocc] - ref.theta[:nocc]).max() <= 1e-9
