"""The mixed-precision plan (complex64 blocks, FP32 FFT/H-apply and Gram
products, FP64 subspace solve) against the FP64 oracle."""
import sys

import numpy as np
import pytest

import ksinputs as ki
from oracle import hamiltonian as oh
from oracle import lobpcg as olob

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    import torch

    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


@pytest.mark.parametrize("name", ["C1", "C2"])
def test_fp32_apply_h_matches_oracle(ks, name):
    import torch

    from paper_2512_04447_amd import binding as b

    cfg = ki.config(name)
    cell = ki.make_cell(cfg)
    oc = oh.oracle_cell(cfg, cell.D)
    nb = 8
    rng = np.random.default_rng(3)
    psi = rng.standard_normal((nb, cfg.Ng)) + 1j * rng.standard_normal((nb, cfg.Ng))
    ref = oh.apply_h(oc, psi)
    proj = b.ProjectorArrays.from_cell(cell) if cell.nproj else None
    plan = b.Plan(cell.n, cell.L, proj, nb, b.KS_MIXED_FP32)
    d = dev(psi, torch.complex64)
    out = torch.empty_like(d)
    b.ks_apply_h(plan, dev(cell.V, torch.float32), d, out)
    err = np.abs(out.cpu().numpy() - ref).max() / np.abs(ref).max()
    _say(name, "fp32 apply_h rel err", err)
    assert err <= 2e-6


def test_mixed_lobpcg_c1_eigenvalues_within_1e6(ks):
    import torch

    from paper_2512_04447_amd import binding as b

    cfg = ki.config("C1")
    cell = ki.make_cell(cfg)
    oc = oh.oracle_cell(cfg, cell.D)
    st_ref, _ = olob.run(oc, ki.make_x0(cfg), cfg.ntrack, 1e-8, 200, olob.tpa_preconditioner(oc))
    plan = b.Plan(cell.n, cell.L, None, cfg.nb, b.KS_MIXED_FP32)
    lob = b.Lobpcg(plan, dev(cell.V, torch.float32), dev(ki.make_x0(cfg), torch.complex64))
    lob.init()
    best = None
    for it in range(60):
        # lock above the FP32 residual floor (about eps32 * ||H||)
        lob.step(b.KS_PRECOND_TPA, 1e-4)
        th = lob.theta.cpu().numpy()
        err = np.abs(th - st_ref.theta).max()
        best = err if best is None else min(best, err)
        if err <= 1e-7:
            break
    _say("mixed C1: iterations", it + 1, "max |dtheta|", err, "res", float(lob.res.max()))
    assert err <= 1e-6
    X = lob.X.cpu().numpy().astype(np.complex128)
    assert np.abs(np.conj(X) @ X.T - np.eye(cfg.nb)).max() <= 1e-5
