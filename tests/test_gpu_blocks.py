"""The Gram and rotation products as standalone entry points against the
matrix product on the CPU (numpy, FP64)."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("m,K,prec", [(1, 100, 0), (37, 1000, 0), (64, 4097, 0), (130, 2500, 0), (37, 1000, 1),
                                      (130, 5000, 1), (257, 257, 0), (511, 511, 1)])
def test_gram_general_and_rotation_match_numpy(ks, m, K, prec):
    import torch

    from paper_2512_04447_amd import binding as b

    _say("blocks", m, K, prec)
    rng = np.random.default_rng(m + K)
    A = (rng.standard_normal((m, K)) + 1j * rng.standard_normal((m, K))) / np.sqrt(2)
    B = (rng.standard_normal((m, K)) + 1j * rng.standard_normal((m, K))) / np.sqrt(2)
    cdt = torch.complex128 if prec == 0 else torch.complex64
    if prec == 1:
        A = A.astype(np.complex64).astype(np.complex128)
        B = B.astype(np.complex64).astype(np.complex128)
    dA = torch.from_numpy(A).to(cdt).cuda()
    dB = torch.from_numpy(B).to(cdt).cuda()
    G = torch.zeros((m, m), dtype=torch.complex128, device="cuda").T
    b.ks_gram_general(prec, dA, dB, G)
    ref = np.conj(A) @ B.T
    err = np.abs(G.cpu().numpy() - ref).max() / np.abs(ref).max()
    _say("  gram rel err", err)
    assert err <= (1e-13 if prec == 0 else 2e-6)
    ncol = max(1, m // 2)
    Cm = (rng.standard_normal((m, ncol)) + 1j * rng.standard_normal((m, ncol)))
    if prec == 1:
        Cm = Cm.astype(np.complex64).astype(np.complex128)
    dC = torch.from_numpy(np.ascontiguousarray(Cm.T)).to(cdt).cuda().T  # column-major m x ncol
    Y = torch.zeros((ncol, K), dtype=cdt, device="cuda")
    b.ks_rotate_block(prec, dA, dC, Y)
    yref = Cm.T @ A
    err = np.abs(Y.cpu().numpy() - yref).max() / np.abs(yref).max()
    _say("  rotate rel err", err)
    assert err <= (1e-13 if prec == 0 else 2e-6)


@pytest.mark.parametrize("prec", [0, 1])
def test_rotation_of_a_tall_block_matches_numpy_on_sampled_points(ks, prec):
    """K = 400037 points, 64 columns in and 480 out: the launch gives each
    workgroup eight 64-point row tiles, the last workgroup three, the last
    tile ragged.  Compared on every 61st point (at least one per tile) and
    the last 200 points."""
    import torch

    from paper_2512_04447_amd import binding as b

    m, ncol, K = 64, 480, 400037
    _say("tall rotation", m, ncol, K, prec)
    rng = np.random.default_rng(prec + 11)
    A = (rng.standard_normal((m, K)) + 1j * rng.standard_normal((m, K))) / np.sqrt(2)
    Cm = rng.standard_normal((m, ncol)) + 1j * rng.standard_normal((m, ncol))
    cdt = torch.complex128 if prec == 0 else torch.complex64
    if prec == 1:
        A = A.astype(np.complex64).astype(np.complex128)
        Cm = Cm.astype(np.complex64).astype(np.complex128)
    dA = torch.from_numpy(A).to(cdt).cuda()
    dC = torch.from_numpy(np.ascontiguousarray(Cm.T)).to(cdt).cuda().T
    Y = torch.zeros((ncol, K), dtype=cdt, device="cuda")
    b.ks_rotate_block(prec, dA, dC, Y)
    idx = np.unique(np.concatenate([np.arange(0, K, 61), np.arange(K - 200, K)]))
    got = Y[:, torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.complex128)
    ref = Cm.T @ A[:, idx]
    err = np.abs(got - ref).max() / np.abs(ref).max()
    _say("  rel err", err)
    assert err <= (1e-13 if prec == 0 else 2e-6)
    del dA, Y
    torch.cuda.empty_cache()
