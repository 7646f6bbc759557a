"""The no-allocation dense solve (hegv_reduce_solve_noalloc) against the
allocating entry point, through the C ABI: two calls in a row on the same
GPU, the second smaller, each equal to hegv_reduce_solve on the same
matrices."""
import ctypes as C
import math
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _pencil(n, rng):
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    S = (Q * np.logspace(0, -4, n)) @ Q.conj().T
    Hm = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    return 0.5 * (Hm + Hm.conj().T), 0.5 * (S + S.conj().T)


def _colmajor(A):
    import torch

    return torch.from_numpy(np.ascontiguousarray(A.T)).cuda().T


def _solve(lib, b, Hm, S, nev, noalloc):
    import torch

    n = Hm.shape[0]
    dH, dS = _colmajor(Hm), _colmajor(S)
    w = torch.zeros(nev, dtype=torch.float64, device="cuda")
    Cm = torch.zeros((nev, n), dtype=torch.complex128, device="cuda").T
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    s = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    if noalloc:
        rc = lib.hegv_reduce_solve_noalloc(n, nev, dH.data_ptr(), n, dS.data_ptr(), n, w.data_ptr(), Cm.data_ptr(),
                                           n, info.data_ptr(), s)
    else:
        b.hegv_reduce_solve(dH, dS, nev, w, Cm, info)
        rc = 0
    b.check(rc, "hegv_reduce_solve_noalloc")
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    return w.cpu().numpy(), Cm.cpu().numpy()


def test_noalloc_solve_equals_the_allocating_one_on_two_calls(ks):
    from paper_2512_04447_amd import binding as b

    lib = b.load()
    rng = np.random.default_rng(77)
    for n, nev in ((480, 160), (100, 33)):  # the second call is smaller
        _say("noalloc hegv", n, nev)
        Hm, S = _pencil(n, rng)
        w0, C0 = _solve(lib, b, Hm, S, nev, noalloc=False)
        w1, C1 = _solve(lib, b, Hm, S, nev, noalloc=True)
        # the same kernels on the same inputs: identical results
        np.testing.assert_array_equal(w1, w0)
        np.testing.assert_array_equal(C1, C0)
        assert np.abs(C1.conj().T @ S @ C1 - np.eye(nev)).max() <= 1e-9
    # sizes beyond the static array are refused before any launch
    fake = C.c_void_p(16)
    assert lib.hegv_reduce_solve_noalloc(513, 10, fake, 513, fake, 513, fake, fake, 513, fake, None) == -1
    assert "no-allocation" in lib.ks_last_error().decode()
