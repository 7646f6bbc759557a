"""Parity of the HIP path (through the C ABI) with the CPU oracle."""
import math
import sys

import numpy as np
import pytest

import ksinputs as ki
from oracle import hamiltonian as oh
from oracle import linalg as ola
from oracle import lobpcg as olob
from oracle import precond as opc

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def tiny_cfg(n=10, L=7.0, lmax=1, positions=((0.1, 0.2, 0.3), (0.6, 0.55, 0.45)), nb=6):
    return ki.custom_config("tiny", L, n, positions, nb, lmax=lmax, rc=0.61)


CELLS = {
    "C1": lambda: ki.config("C1"),
    "tiny10_sp": lambda: tiny_cfg(),
    "tiny12_spd": lambda: tiny_cfg(n=12, L=8.0, lmax=2),
    "odd14": lambda: ki.custom_config("odd14", 7.5, 14, ((0.2, 0.3, 0.4),), 5, lmax=1, rc=0.6),
    "C2": lambda: ki.config("C2"),
    # planes above 4096 points take the 1024-thread plane passes
    "big72": lambda: ki.custom_config("big72", 10.0, 72, ((0.1, 0.2, 0.3), (0.6, 0.55, 0.45)), 3, lmax=1,
                                      rc=0.61),
    "big70": lambda: ki.custom_config("big70", 9.5, 70, ((0.15, 0.25, 0.35),), 3, lmax=2, rc=0.63),
    # the 216-atom and 128-atom cells' grids (radices 16 x 6 and 16 x 7)
    "big96": lambda: ki.custom_config("big96", 12.0, 96, ((0.3, 0.45, 0.2),), 2, lmax=1, rc=0.62),
    "big112": lambda: ki.custom_config("big112", 14.0, 112, ((0.6, 0.35, 0.15),), 1, lmax=2, rc=0.64),
    # FP64 planes beyond a CU's LDS: the split row / column passes
    "big100": lambda: ki.custom_config("big100", 12.5, 100, ((0.3, 0.45, 0.2),), 2, lmax=1, rc=0.62),
}


def make_plan(ks, cell, nb, precision=0):
    from paper_2512_04447_amd import binding as b

    proj = b.ProjectorArrays.from_cell(cell) if cell.nproj else None
    return b.Plan(cell.n, cell.L, proj, nb, precision)


def to_dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


@pytest.mark.parametrize("name,nb,prec", [("C1", 16, 0), ("tiny10_sp", 5, 0), ("tiny12_spd", 7, 0), ("odd14", 3, 0),
                                          ("C2", 20, 0), ("big72", 3, 0), ("big70", 2, 0), ("big72", 3, 1),
                                          ("big70", 2, 1), ("big96", 2, 0), ("big96", 2, 1), ("big112", 1, 1),
                                          ("big112", 1, 0), ("big100", 2, 0)])
def test_apply_h_matches_oracle(ks, name, nb, prec):
    """FP64 plans to 1e-12 and FP32 plans (prec 1) to 2e-6 of max |H psi|."""
    import torch

    cfg = CELLS[name]()
    cell = ki.make_cell(cfg)
    _say("apply_h", name, cfg.n, nb)
    oc = oh.from_arrays(cell.n, cell.L, cell.V,
                        [cell.supp_idx[cell.atom_supp_ptr[a]:cell.atom_supp_ptr[a + 1]]
                         for a in range(cell.natoms) for _ in range(cell.atom_proj_ptr[a + 1] - cell.atom_proj_ptr[a])],
                        [cell.beta[cell.beta_ptr[a] + j * (cell.atom_supp_ptr[a + 1] - cell.atom_supp_ptr[a]):
                                   cell.beta_ptr[a] + (j + 1) * (cell.atom_supp_ptr[a + 1] - cell.atom_supp_ptr[a])]
                         for a in range(cell.natoms) for j in range(cell.atom_proj_ptr[a + 1] - cell.atom_proj_ptr[a])],
                        cell.D)
    rng = np.random.default_rng(42)
    psi = rng.standard_normal((nb, cfg.Ng)) + 1j * rng.standard_normal((nb, cfg.Ng))
    ref = oh.apply_h(oc, psi)
    from paper_2512_04447_amd import binding as b

    plan = make_plan(ks, cell, nb, prec)
    if prec == 0:
        dpsi, v = to_dev(psi), to_dev(cell.V)
    else:
        dpsi, v = to_dev(psi, torch.complex64), to_dev(cell.V, torch.float32)
    out = torch.empty_like(dpsi)
    b.ks_apply_h(plan, v, dpsi, out)
    got = out.cpu().numpy().astype(np.complex128)
    err = np.abs(got - ref).max() / np.abs(ref).max()
    _say("  rel err", err)
    assert err <= (1e-12 if prec == 0 else 2e-6)


@pytest.mark.parametrize("name,nb", [("C1", 16), ("tiny10_sp", 6), ("C2", 12), ("big72", 3), ("big112", 3)])
def test_tpa_preconditioner_and_residual_match_oracle(ks, name, nb):
    import torch

    from paper_2512_04447_amd import binding as b

    cfg = CELLS[name]()
    cell = ki.make_cell(cfg)
    _say("precond", name, nb)
    oc = oh.oracle_cell(cfg, cell.D)
    X0 = ki.make_x0(cfg, nb=nb)
    st = olob.initial_state(oc, X0)
    R, res = olob.residual(st)
    E = opc.band_kinetic_energy(st.X, cfg.n, cfg.L)
    Wref = opc.tpa_apply(R, E, cfg.n, cfg.L)
    plan = make_plan(ks, cell, nb)
    W = torch.empty((nb, cfg.Ng), dtype=torch.complex128, device="cuda")
    dres = torch.empty(nb, dtype=torch.float64, device="cuda")
    b.ks_precond_apply(plan, b.KS_PRECOND_TPA, to_dev(st.X), to_dev(st.AX), to_dev(st.theta), W, dres, 0.0)
    assert np.abs(dres.cpu().numpy() - res).max() <= 1e-12 * res.max()
    assert np.abs(W.cpu().numpy() - Wref).max() <= 1e-12 * np.abs(Wref).max()
    # lock mask: columns with res <= lock_tol are exact zeros
    rs = np.sort(res)
    lock = float(0.5 * (rs[nb // 2] + rs[nb // 2 + 1]))  # strictly between two residuals
    b.ks_precond_apply(plan, b.KS_PRECOND_TPA, to_dev(st.X), to_dev(st.AX), to_dev(st.theta), W, dres, lock)
    Wl = W.cpu().numpy()
    for i in range(nb):
        if res[i] <= lock:
            assert np.all(Wl[i] == 0)
        else:
            assert np.abs(Wl[i] - Wref[i]).max() <= 1e-12 * np.abs(Wref).max()


def random_hpd(n, rng, cond=1e4):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    s = np.logspace(0, -math.log10(cond), n)
    return (Q * s) @ Q.conj().T


def colmajor(A):
    import torch

    # column-major storage: the transpose is contiguous, stride(1) = n
    return torch.from_numpy(np.ascontiguousarray(A.T)).cuda().T


# 97: the LDS tail alone (trailing matrix of 96); 98: one column step
# (product, then update) before it; 99: one fused step between them;
# 514: one two-launch step (trailing size 513), then fused steps from 512;
# 960: two launches per column while the trailing matrix is above 512, then
# one per column, then the LDS tail; back-transform with 16 entries per
# lane; 1440: the subspace of the 216-atom cell (trailing matrix resident in
# LDS from the first step); 1800: one column per launch first, then resident
@pytest.mark.parametrize("n,nev", [(1, 1), (2, 1), (5, 3), (33, 11), (48, 16), (97, 32), (98, 33), (99, 33),
                                   (100, 40), (480, 160), (514, 171), (960, 320), (1440, 480), (1800, 600)])
def test_hegv_reduce_solve_matches_oracle(ks, n, nev):
    import torch

    from paper_2512_04447_amd import binding as b

    _say("hegv", n, nev)
    rng = np.random.default_rng(1000 + n)
    S = random_hpd(n, rng)
    Hm = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Hm = 0.5 * (Hm + Hm.conj().T)
    if n <= 100:
        wref, _, info = ola.hegv_two_trsm(Hm, S, nev)
        assert info == 0
    else:
        import scipy.linalg

        wref = scipy.linalg.eigh(Hm, S, eigvals_only=True)[:nev]
    dH, dS = colmajor(Hm), colmajor(S)
    w = torch.zeros(nev, dtype=torch.float64, device="cuda")
    Cm = torch.zeros((nev, n), dtype=torch.complex128, device="cuda").T  # column-major n x nev
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    b.hegv_reduce_solve(dH, dS, nev, w, Cm, info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    wg = w.cpu().numpy()
    Cg = Cm.cpu().numpy()
    scale = max(1.0, np.abs(wref).max())
    _say("  max |dw|", np.abs(wg - wref).max())
    assert np.abs(wg - wref).max() <= 1e-10 * scale
    assert np.abs(Cg.conj().T @ S @ Cg - np.eye(nev)).max() <= 1e-9
    assert np.abs(Hm @ Cg - S @ Cg * wg).max() <= 1e-8 * scale


def test_hegv_reports_indefinite_overlap(ks):
    import torch

    from paper_2512_04447_amd import binding as b

    n = 40
    S = np.eye(n, dtype=complex)
    S[37, 37] = -1.0
    Hm = np.eye(n, dtype=complex)
    w = torch.zeros(4, dtype=torch.float64, device="cuda")
    Cm = torch.zeros((4, n), dtype=torch.complex128, device="cuda").T
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    b.hegv_reduce_solve(colmajor(Hm), colmajor(S), 4, w, Cm, info)
    assert int(info.item()) == n + 38


def _gpu_state_from_oracle(lob, st):
    import torch

    lob.buf["X"].copy_(to_dev(st.X))
    lob.buf["AX"].copy_(to_dev(st.AX))
    lob.theta.copy_(to_dev(st.theta))
    for k in ("X", "AX"):
        setattr(lob.st, k, int(lob.buf[k].data_ptr()))
    if st.P is not None:
        lob.buf["P"].copy_(to_dev(st.P))
        lob.st.P = int(lob.buf["P"].data_ptr())
        lob.st.has_p = 1
    lob.st.p_gram_ok = 0  # P replaced: the next step forms its Gram from P
    torch.cuda.synchronize()


def _subspace_gap(A, B):
    """max |P_A - P_B| for orthonormal band-major blocks."""
    PA = A.T @ np.conj(A)
    PB = B.T @ np.conj(B)
    return np.abs(PA - PB).max()


@pytest.mark.parametrize("name", ["C1", "tiny10_sp"])
def test_single_lobpcg_step_matches_oracle(ks, name):
    from paper_2512_04447_amd import binding as b

    cfg = CELLS[name]()
    cell = ki.make_cell(cfg)
    _say("single step", name)
    oc = oh.oracle_cell(cfg, cell.D)
    pc = olob.tpa_preconditioner(oc)
    st = olob.initial_state(oc, ki.make_x0(cfg))
    for _ in range(3):
        st = olob.step(oc, st, pc)
    plan = make_plan(ks, cell, cfg.nb)
    lob = b.Lobpcg(plan, to_dev(cell.V), to_dev(st.X))
    _gpu_state_from_oracle(lob, st)
    lob.step(b.KS_PRECOND_TPA, 0.0)
    ref = olob.step(oc, st, pc)
    th = lob.theta.cpu().numpy()
    assert np.abs(th - ref.theta).max() <= 1e-12 * max(1.0, np.abs(ref.theta).max())
    Xg = lob.X.cpu().numpy()
    # compare spans only across clusters that are separated (degenerate sets
    # may be split differently)
    w = ref.theta
    cut = [k for k in range(1, cfg.nb) if w[k] - w[k - 1] > 1e-6] + [cfg.nb]
    assert _subspace_gap(Xg[:cut[0]], ref.X[:cut[0]]) <= 1e-10
    assert _subspace_gap(Xg, ref.X) <= 1e-10


@pytest.mark.parametrize("name", ["C1", "tiny10_sp"])
def test_soft_locked_step_matches_oracle_and_skips_locked_columns(ks, name):
    """A step with lock_tol between two residuals: the oracle zeroes the
    locked bands' W and P columns; the GPU does the same and skips their FFT
    passes in the W and P H-applies (writing zeros).  Ritz values and the
    subspace as in the unlocked step's test, and the locked columns of W, AW,
    P and AP exactly zero."""
    from paper_2512_04447_amd import binding as b

    cfg = CELLS[name]()
    cell = ki.make_cell(cfg)
    _say("soft-locked step", name)
    oc = oh.oracle_cell(cfg, cell.D)
    pc = olob.tpa_preconditioner(oc)
    st = olob.initial_state(oc, ki.make_x0(cfg))
    for _ in range(4):
        st = olob.step(oc, st, pc)
    _, res = olob.residual(st)
    rs = np.sort(res)
    lock = float(0.5 * (rs[cfg.nb // 2] + rs[cfg.nb // 2 + 1]))
    locked = res <= lock
    assert 0 < locked.sum() < cfg.nb
    ref = olob.step(oc, st, pc, lock_tol=lock)
    plan = make_plan(ks, cell, cfg.nb)
    lob = b.Lobpcg(plan, to_dev(cell.V), to_dev(st.X))
    _gpu_state_from_oracle(lob, st)
    lob.step(b.KS_PRECOND_TPA, lock)
    assert np.array_equal(lob.res_host <= lock, locked)
    th = lob.theta.cpu().numpy()
    assert np.abs(th - ref.theta).max() <= 1e-12 * max(1.0, np.abs(ref.theta).max())
    Xg = lob.X.cpu().numpy()
    assert _subspace_gap(Xg, ref.X) <= 1e-10
    # this step's W, AW, AP (P was rotated into the next step's P, so the
    # locked columns of the masked P are seen through AP)
    for k in ("W", "AW", "AP"):
        blk = lob.block(k).cpu().numpy()
        assert np.all(blk[locked] == 0), k
        assert np.all(np.abs(blk[~locked]).max(axis=1) > 0), k


def test_lobpcg_c1_converges_to_oracle_eigenvalues(ks):
    from paper_2512_04447_amd import binding as b

    cfg = ki.config("C1")
    cell = ki.make_cell(cfg)
    oc = oh.oracle_cell(cfg, cell.D)
    _say("C1 run")
    st_ref, _ = olob.run(oc, ki.make_x0(cfg), cfg.ntrack, 1e-8, 200, olob.tpa_preconditioner(oc))
    plan = make_plan(ks, cell, cfg.nb)
    lob = b.Lobpcg(plan, to_dev(cell.V), to_dev(ki.make_x0(cfg)))
    lob.init()
    tol = 1e-8
    for it in range(200):
        lob.step(b.KS_PRECOND_TPA, 0.1 * tol)
        res = lob.res_host  # the step's one device-to-host copy
        assert lob.status_host[b.KS_ST_FLAGS] & (b.KS_FLAG_SOLVE_FAILED | b.KS_FLAG_NONFINITE) == 0
        if res[:cfg.ntrack].max() <= tol:
            break
    _say("  gpu iterations", it + 1, "status", lob.status_host.tolist())
    assert res[:cfg.ntrack].max() <= tol
    np.testing.assert_array_equal(res, lob.res.cpu().numpy())
    np.testing.assert_array_equal(lob.theta_host, lob.theta.cpu().numpy())
    th = lob.theta.cpu().numpy()
    assert np.abs(th - st_ref.theta).max() <= 1e-10
    X = lob.X.cpu().numpy()
    assert np.abs(np.conj(X) @ X.T - np.eye(cfg.nb)).max() <= 1e-12


# ---------------------------------------------------------------- deflation and hard pencils


@pytest.mark.parametrize("variant", ["p_in_span_of_x", "p_duplicate_columns"])
def test_lobpcg_step_deflation_matches_oracle(ks, variant):
    """Numerically dependent columns are dropped on the device exactly as
    the oracle's deflating Cholesky drops them: P inside span(X) loses every
    column in the basis Cholesky; P with two equal columns loses one in its
    own orthonormalisation."""
    from paper_2512_04447_amd import binding as b

    cfg = CELLS["tiny10_sp"]()
    cell = ki.make_cell(cfg)
    _say("deflation", variant)
    oc = oh.oracle_cell(cfg, cell.D)
    pc = olob.tpa_preconditioner(oc)
    st = olob.initial_state(oc, ki.make_x0(cfg))
    for _ in range(2):
        st = olob.step(oc, st, pc)
    rng = np.random.default_rng(5)
    nb = cfg.nb
    if variant == "p_in_span_of_x":
        M = rng.standard_normal((nb, nb)) + 1j * rng.standard_normal((nb, nb))
        P = M.T @ st.X
    else:
        P = st.P.copy()
        P[3] = P[1]
    st.P = P
    ref = olob.step(oc, st, pc)
    plan = make_plan(ks, cell, nb)
    lob = b.Lobpcg(plan, to_dev(cell.V), to_dev(st.X))
    _gpu_state_from_oracle(lob, st)
    lob.step(b.KS_PRECOND_TPA, 0.0)
    status = lob.status_host
    _say("  status", status.tolist(), "oracle events", ref.events)
    if variant == "p_in_span_of_x":
        assert f"basis_deflated_{nb}" in ref.events
        assert status[b.KS_ST_DEAD_BASIS] == nb and status[b.KS_ST_DEAD_P] == 0
    else:
        assert "p_deflated_1" in ref.events
        assert status[b.KS_ST_DEAD_P] == 1
    assert status[b.KS_ST_FLAGS] == b.KS_FLAG_DEFLATED
    th = lob.theta_host
    assert np.abs(th - ref.theta).max() <= 1e-12 * max(1.0, np.abs(ref.theta).max())
    assert _subspace_gap(lob.X.cpu().numpy(), ref.X) <= 1e-10


def _pencil_with_spectrum(n, lam, cond, rng):
    """(H, S) with generalised eigenvalues exactly lam: S = B B^H, H = B diag(lam) B^H
    for a random B with singular values logspaced over sqrt(cond)."""
    Q1, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    Q2, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    sv = np.logspace(0, -0.5 * math.log10(cond), n)
    B = (Q1 * sv) @ Q2.conj().T
    S = B @ B.conj().T
    Hm = (B * lam) @ B.conj().T
    return 0.5 * (Hm + Hm.conj().T), 0.5 * (S + S.conj().T)


@pytest.mark.parametrize("n,cond", [(480, 1e4), (480, 1e8), (480, 1e12), (1440, 1e4), (1440, 1e10)])
def test_hegv_degenerate_clusters_and_ill_conditioned_overlap(ks, n, cond):
    """Closed-form spectra: H C = S C diag(w) with exactly repeated
    eigenvalues (multiplicities 6, 12 and 24, as in the free-electron-like
    8-atom cell) and cond(S) up to 1e12.  Eigenvalues within the bound a
    backward-stable reduction allows (its error grows like eps cond(S)),
    never more than 10x the LAPACK generalised solve's error on the same
    matrices; C^H S C = I and the residual to the same scale."""
    import scipy.linalg
    import torch

    from paper_2512_04447_amd import binding as b

    nev = n // 3
    rng = np.random.default_rng(int(n + math.log10(cond)))
    # low end: clusters of 6, 12, 24 (then singles) at well separated levels
    lam = list(np.repeat([-2.0, -1.5, -1.0], [6, 12, 24]))
    lam += list(np.linspace(-0.5, 3.0, n - len(lam)))
    lam = np.array(lam)
    _say("hegv hard", n, cond)
    Hm, S = _pencil_with_spectrum(n, lam, cond, rng)
    exact = np.sort(lam)[:nev]
    lap = scipy.linalg.eigh(Hm, S, eigvals_only=True)[:nev]
    lap_err = np.abs(lap - exact).max()
    dH, dS = colmajor(Hm), colmajor(S)
    w = torch.zeros(nev, dtype=torch.float64, device="cuda")
    Cm = torch.zeros((nev, n), dtype=torch.complex128, device="cuda").T
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    b.hegv_reduce_solve(dH, dS, nev, w, Cm, info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    wg, Cg = w.cpu().numpy(), Cm.cpu().numpy()
    err = np.abs(wg - exact).max()
    bound = 1e-13 * cond * 3.0
    _say("  gpu err", err, "lapack err", lap_err, "bound", bound)
    assert err <= max(bound, 1e-11)
    assert err <= 10 * lap_err + 1e-11
    orth = np.abs(Cg.conj().T @ S @ Cg - np.eye(nev)).max()
    resid = np.abs(Hm @ Cg - S @ Cg * wg).max() / np.abs(Hm).max()
    _say("  C^H S C - I", orth, "residual", resid)
    assert orth <= max(1e-13 * cond, 1e-10)
    assert resid <= max(1e-13 * cond, 1e-10)
    # the strict solve leaves w and C untouched on a failed factorisation
    S2 = S.copy()
    S2[n - 5, n - 5] = -1.0
    w.fill_(7.0)
    Cm.fill_(3.0)
    b.hegv_reduce_solve(colmajor(Hm), colmajor(S2), nev, w, Cm, info)
    torch.cuda.synchronize()
    assert int(info.item()) > n
    assert bool((w == 7.0).all()) and bool((Cm == 3.0).all())


@pytest.mark.parametrize("n,cond", [(480, 1e2), (1440, 1e6)])
def test_hegv_chained_cluster(ks, n, cond):
    """A dense run of distinct eigenvalues, each closer to the next than
    the cluster tolerance (1e-5 |T|), forms one chained cluster of nev - 8
    values: inverse iteration re-orthogonalises each vector against the
    earlier ones within the tolerance window only.  Eigenvalues within
    1e-11 of the closed form, C^H S C = I and the residual to 1e-10 (the
    window's bound on the orthogonality of vectors outside it is
    eps |T| / 1e-5 |T|, about 1e-11)."""
    import torch

    from paper_2512_04447_amd import binding as b

    nev = n // 3
    rng = np.random.default_rng(n + 3)
    # |T| is about 3 here (the spectrum's extent): spacing 1e-6 < 3e-5
    run = -1.0 + 1e-6 * np.arange(nev - 8)
    lam = np.concatenate([np.linspace(-2.0, -1.5, 8), run, np.linspace(0.5, 3.0, n - nev)])
    _say("hegv chain", n, cond, len(run))
    Hm, S = _pencil_with_spectrum(n, lam, cond, rng)
    exact = np.sort(lam)[:nev]
    w = torch.zeros(nev, dtype=torch.float64, device="cuda")
    Cm = torch.zeros((nev, n), dtype=torch.complex128, device="cuda").T
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    b.hegv_reduce_solve(colmajor(Hm), colmajor(S), nev, w, Cm, info)
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    wg, Cg = w.cpu().numpy(), Cm.cpu().numpy()
    err = np.abs(wg - exact).max()
    orth = np.abs(Cg.conj().T @ S @ Cg - np.eye(nev)).max()
    resid = np.abs(Hm @ Cg - S @ Cg * wg).max() / np.abs(Hm).max()
    _say("  err", err, "C^H S C - I", orth, "residual", resid)
    assert err <= max(1e-13 * cond * 3.0, 1e-11)
    assert orth <= max(1e-13 * cond, 1e-10)
    assert resid <= max(1e-13 * cond, 1e-10)


def test_apply_h_with_an_atom_without_projectors(ks):
    """An atom with support points but no projectors contributes nothing and
    is not read: H-apply equals the oracle with only the other atom's
    projectors."""
    import torch

    from paper_2512_04447_amd import binding as b

    cfg = CELLS["tiny10_sp"]()
    cell = ki.make_cell(cfg)
    _say("atom without projectors")
    sp, si, pp, bp = cell.atom_supp_ptr, cell.supp_idx, cell.atom_proj_ptr, cell.beta_ptr
    np0 = int(pp[1] - pp[0])
    # atom 0 keeps its support list, loses its projectors
    proj = b.ProjectorArrays(np.array(sp, np.int32), np.array(si, np.int32),
                             np.array([0, 0, pp[2] - np0], np.int32),
                             np.array([0, 0, bp[2] - bp[1]], np.int64),
                             np.ascontiguousarray(cell.beta[bp[1]:bp[2]]),
                             np.ascontiguousarray(cell.D[np0:]))
    nb = 4
    plan = b.Plan(cell.n, cell.L, proj, nb, b.KS_FP64)
    X0 = ki.make_x0(cfg, nb=nb)
    hx = torch.empty((nb, cfg.Ng), dtype=torch.complex128, device="cuda")
    b.ks_apply_h(plan, to_dev(cell.V), to_dev(X0), hx)
    ns1 = int(sp[2] - sp[1])
    supp1 = np.asarray(si[sp[1]:sp[2]])
    vals = [np.asarray(cell.beta[bp[1] + j * ns1: bp[1] + (j + 1) * ns1]) for j in range(int(pp[2] - pp[1]))]
    oc = oh.from_arrays(cfg.n, cfg.L, cell.V, [supp1] * len(vals), vals, cell.D[np0:])
    ref = oh.apply_h(oc, X0)
    err = np.abs(hx.cpu().numpy() - ref).max() / np.abs(ref).max()
    _say("  rel err", err)
    assert err <= 1e-12


@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("n", [1, 5, 33, 64, 100, 257])
def test_real_symmetric_reduction_variants_match_oracle(ks, variant, n):
    """The Gamma-point (real symmetric) reduction by its three methods
    against the oracle's Cholesky and two forward substitutions, which on a
    real pencil return real values (imaginary parts exactly zero)."""
    import torch

    from paper_2512_04447_amd import binding as b

    _say("real reduce variant", variant, n)
    rng = np.random.default_rng(4000 + n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    S = (Q * np.logspace(0, -4, n)) @ Q.T
    S = 0.5 * (S + S.T)
    Hm = rng.standard_normal((n, n))
    Hm = 0.5 * (Hm + Hm.T)
    L, info = ola.cholesky_lower(S)
    assert info == 0 and not np.any(L.imag)
    Y = ola.solve_lower(L, Hm)
    Kref = ola.solve_lower(L, Y.T)
    assert not np.any(Kref.imag)
    Kref = 0.5 * (Kref.real + Kref.real.T)
    dH, dS = colmajor(Hm), colmajor(S)
    dK = torch.zeros((n, n), dtype=torch.float64, device="cuda").T
    dinfo = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    b.sygv_reduce_variant(variant, dH, dS, dK, dinfo)
    torch.cuda.synchronize()
    assert int(dinfo.item()) == 0
    Lg = np.tril(dS.cpu().numpy())
    assert np.abs(Lg - L.real).max() <= 1e-12 * np.abs(L).max()
    Kg = dK.cpu().numpy()
    assert np.array_equal(Kg, Kg.T)
    err = np.abs(Kg - Kref).max() / np.abs(Kref).max()
    _say("  rel err", err)
    assert err <= 5e-12
    assert np.array_equal(dH.cpu().numpy(), Hm)


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_real_symmetric_reduction_reports_indefinite_overlap(ks, variant):
    """A real S whose leading minor 37 is singular: info = n + 37, as the
    oracle's Cholesky reports 37."""
    import torch

    from paper_2512_04447_amd import binding as b

    n = 70
    rng = np.random.default_rng(77)
    A = rng.standard_normal((n, n))
    S = A @ A.T + n * np.eye(n)
    S[36, :36] = S[35, :36]
    S[:36, 36] = S[:36, 35]
    S[36, 36] = S[35, 35]
    S[36, 35] = S[35, 36] = S[35, 35]
    _, info = ola.cholesky_lower(S)
    assert info == 37
    dH = colmajor(np.eye(n))
    dS = colmajor(S)
    dK = torch.zeros((n, n), dtype=torch.float64, device="cuda").T
    dinfo = torch.zeros(1, dtype=torch.int32, device="cuda")
    b.sygv_reduce_variant(variant, dH, dS, dK, dinfo)
    torch.cuda.synchronize()
    assert int(dinfo.item()) == n + 37


@pytest.mark.parametrize("variant", [0, 1, 2])
@pytest.mark.parametrize("n", [1, 5, 33, 64, 100, 257])
def test_reduction_variants_match_oracle(ks, variant, n):
    """K = L^-1 H L^-H by the explicit inverse, by two triangular solves and
    by the blocked two-sided reduction, each against the oracle's two
    forward substitutions; the factor against the oracle's Cholesky."""
    import torch

    from paper_2512_04447_amd import binding as b

    _say("reduce variant", variant, n)
    rng = np.random.default_rng(3000 + n)
    # the reduction's rounding error grows like eps cond(S) (L^-1 on both
    # sides); with cond(S) = 1e4 two correct orderings agree to about 1e-12
    S = random_hpd(n, rng, cond=1e4)
    Hm = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    Hm = 0.5 * (Hm + Hm.conj().T)
    L, info = ola.cholesky_lower(S)
    assert info == 0
    Y = ola.solve_lower(L, Hm)
    Kref = ola.solve_lower(L, np.conj(Y.T))
    Kref = 0.5 * (Kref + Kref.conj().T)
    dH, dS = colmajor(Hm), colmajor(S)
    dK = torch.zeros((n, n), dtype=torch.complex128, device="cuda").T
    dinfo = torch.zeros(1, dtype=torch.int32, device="cuda")
    b.hegv_reduce_variant(variant, dH, dS, dK, dinfo)
    torch.cuda.synchronize()
    assert int(dinfo.item()) == 0
    Lg = np.tril(dS.cpu().numpy())
    assert np.abs(Lg - L).max() <= 1e-12 * np.abs(L).max()
    err = np.abs(dK.cpu().numpy() - Kref).max() / np.abs(Kref).max()
    _say("  rel err", err)
    assert err <= 5e-12
    # H is not modified
    assert np.array_equal(dH.cpu().numpy(), Hm)
