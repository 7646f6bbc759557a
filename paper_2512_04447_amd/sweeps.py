"""Microbenchmark sweeps of the path's kernels (the shapes of the paper's
GEMM and FFT figures), run on one GPU through the C ABI.

* GEMM: the Gram product G = A^H B of the LOBPCG subspace matrices on the
  matrix cores, complex128 (8 flops per complex multiply-add), square
  (K = m = N) at N = 2^p and 2^p +- 1, and rectangular with K = 250 N (the
  tall-skinny shape of the Gram GEMMs: Ng grid points by m basis vectors);
  the rotation Y = V C for the same rectangular shapes.
* FFT: the batched kinetic-energy application (forward 3D FFT, |G|^2/2,
  inverse 3D FFT, no potential or projectors) through ks_apply_h, with one
  orbital against a batch of 512, across cubic grid sizes: time per
  orbital.  FP64 planes fit the LDS up to n = 96, FP32 up to n = 128.
* Reduction: K = L^-1 H L^-H at the cells' subspace sizes by the explicit
  inverse, the paper's two triangular solves and a blocked two-sided
  (HEGST-type) reduction.

Prints one JSON object per measurement and a summary table.

Usage: python -m paper_2512_04447_amd.sweeps [--gemm] [--fft] [--reduce] [--quick]
"""
from __future__ import annotations

import argparse
import json
import statistics
import sys
import time

from . import binding as b


def _time(fn, reps: int) -> float:
    import torch

    fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return statistics.median(ts)


def gemm_sweep(quick: bool, out):
    import torch

    ps = [8, 9, 10, 11, 12] if quick else [8, 9, 10, 11, 12, 13]
    for prec, cdt, peak in ((b.KS_FP64, torch.complex128, 78.6), (b.KS_MIXED_FP32, torch.complex64, 157.3)):
        for p in ps:
            for N in (2 ** p - 1, 2 ** p, 2 ** p + 1):
                A = torch.randn((N, N), dtype=cdt, device="cuda")
                G = torch.empty((N, N), dtype=torch.complex128, device="cuda").T
                n = b.C.c_size_t()
                b.check(b.load().ks_gram_workspace_size(N, N, b.C.byref(n)), "ks_gram_workspace_size")
                work = b._work(n.value, A.device)
                t = _time(lambda: b.ks_gram_general(prec, A, A, G, work), 3 if N < 4000 else 1)
                tf = 8.0 * N ** 3 / t / 1e12
                rec = {"sweep": "gemm_square", "precision": "fp64" if prec == b.KS_FP64 else "fp32", "N": N,
                       "seconds": t, "tflops": round(tf, 2), "frac_of_peak": round(tf / peak, 3)}
                out(rec)
                del A, G, work
                torch.cuda.empty_cache()
        for N in ([128, 256, 512, 1024] if quick else [128, 256, 512, 1024, 2048]):
            K = 250 * N
            A = torch.randn((N, K), dtype=cdt, device="cuda")
            G = torch.empty((N, N), dtype=torch.complex128, device="cuda").T
            n = b.C.c_size_t()
            b.check(b.load().ks_gram_workspace_size(K, N, b.C.byref(n)), "ks_gram_workspace_size")
            work = b._work(n.value, A.device)
            t = _time(lambda: b.ks_gram_general(prec, A, A, G, work), 3)
            tf = 8.0 * K * N * N / t / 1e12
            out({"sweep": "gemm_rect_gram", "precision": "fp64" if prec == b.KS_FP64 else "fp32", "N": N, "K": K,
                 "seconds": t, "tflops": round(tf, 2), "frac_of_peak": round(tf / peak, 3)})
            Cm = torch.randn((N, N), dtype=cdt, device="cuda").T
            Y = torch.empty((N, K), dtype=cdt, device="cuda")
            t = _time(lambda: b.ks_rotate_block(prec, A, Cm, Y), 3)
            tf = 8.0 * K * N * N / t / 1e12
            out({"sweep": "gemm_rect_rotate", "precision": "fp64" if prec == b.KS_FP64 else "fp32", "N": N, "K": K,
                 "seconds": t, "tflops": round(tf, 2), "frac_of_peak": round(tf / peak, 3)})
            del A, G, work, Cm, Y
            torch.cuda.empty_cache()


def fft_sweep(quick: bool, out):
    import torch

    sizes = {b.KS_FP64: [16, 24, 32, 40, 48, 64, 72, 80, 96],
             b.KS_MIXED_FP32: [16, 24, 32, 40, 48, 64, 72, 80, 96, 112, 128]}
    for prec, sz in sizes.items():
        cdt = torch.complex128 if prec == b.KS_FP64 else torch.complex64
        rdt = torch.float64 if prec == b.KS_FP64 else torch.float32
        es = 16 if prec == b.KS_FP64 else 8
        for n in sz:
            L = 0.21 * n
            for nb in (1, 512):
                plan = b.Plan(n, L, None, nb, prec)
                v = torch.zeros(n ** 3, dtype=rdt, device="cuda")
                psi = torch.randn((nb, n ** 3), dtype=cdt, device="cuda")
                hpsi = torch.empty_like(psi)
                work = b._work(plan.workspace_size(b.KS_OP_APPLY_H, nb), psi.device)
                reps = 20 if nb == 1 else 3
                t = _time(lambda: b.ks_apply_h(plan, v, psi, hpsi, nb, work), reps)
                # three passes, each reading and writing the block, plus the
                # extra read of psi in the last pass: 7 block transfers
                gbs = 7.0 * nb * n ** 3 * es / t / 1e9
                out({"sweep": "fft_laplacian", "precision": "fp64" if prec == b.KS_FP64 else "fp32", "n": n,
                     "orbitals": nb, "seconds": t, "us_per_orbital": round(1e6 * t / nb, 3),
                     "hbm_gbs": round(gbs, 1)})
                plan.destroy()
                del plan, v, psi, hpsi, work
                torch.cuda.empty_cache()


def reduce_sweep(quick: bool, out):
    """The reduction K = L^-1 H L^-H at the subspace sizes of the three
    cells (m = 3 nb = 480, 1440, 2880) by the explicit inverse, the two
    triangular solves and the blocked two-sided reduction (the Cholesky
    included in each), for Hermitian (complex128) and real symmetric
    (float64, the Gamma-point case) matrices."""
    import numpy as np
    import torch

    names = {b.KS_REDUCE_INVERSE: "inverse_and_products", b.KS_REDUCE_TWO_TRSM: "two_trsm",
             b.KS_REDUCE_TWO_SIDED: "two_sided_hegst"}
    for n in ([480, 1440] if quick else [480, 1440, 2880]):
        rng = np.random.default_rng(n)
        A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        S = A @ A.conj().T + n * np.eye(n)
        H = 0.5 * (A + A.conj().T)
        dS0 = torch.from_numpy(np.ascontiguousarray(S.T)).cuda().T
        dH = torch.from_numpy(np.ascontiguousarray(H.T)).cuda().T
        dS = torch.empty_like(dS0)
        dK = torch.empty_like(dH)
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        work = b._work(b.hegv_workspace_size(n, 1), dH.device)
        for v, nm in names.items():
            def run():
                dS.copy_(dS0)
                b.hegv_reduce_variant(v, dH, dS, dK, info, work)
            t = _time(run, 5)
            out({"sweep": "reduction", "field": "hermitian", "n": n, "variant": nm, "seconds": t,
                 "ms": round(1e3 * t, 3)})
        del dS0, dH, dS, dK, work
        # the real symmetric pencil of the same size
        Sr = A.real @ A.real.T + n * np.eye(n)
        Hr = 0.5 * (A.real + A.real.T)
        dS0 = torch.from_numpy(np.ascontiguousarray(Sr.T)).cuda().T
        dH = torch.from_numpy(np.ascontiguousarray(Hr.T)).cuda().T
        dS = torch.empty_like(dS0)
        dK = torch.empty_like(dH)
        work = b._work(b.sygv_reduce_workspace_size(n), dH.device)
        for v, nm in names.items():
            def run():
                dS.copy_(dS0)
                b.sygv_reduce_variant(v, dH, dS, dK, info, work)
            t = _time(run, 5)
            out({"sweep": "reduction", "field": "real", "n": n, "variant": nm, "seconds": t,
                 "ms": round(1e3 * t, 3)})
        del dS0, dH, dS, dK, work
        torch.cuda.empty_cache()


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gemm", action="store_true")
    ap.add_argument("--fft", action="store_true")
    ap.add_argument("--reduce", action="store_true")
    ap.add_argument("--quick", action="store_true")
    a = ap.parse_args(argv)
    import torch

    assert torch.cuda.is_available(), "the sweeps need a GPU"
    b.load()
    rows = []

    def out(rec):
        rows.append(rec)
        print(json.dumps(rec), flush=True)

    every = not (a.gemm or a.fft or a.reduce)
    if a.gemm or every:
        gemm_sweep(a.quick, out)
    if a.fft or every:
        fft_sweep(a.quick, out)
    if a.reduce or every:
        reduce_sweep(a.quick, out)
    for r in rows:
        key = {k: r[k] for k in r if k in ("sweep", "precision", "field", "N", "K", "n", "orbitals", "variant")}
        val = r.get("tflops", r.get("us_per_orbital", r.get("ms")))
        print(f"# {key} -> {val}", file=sys.stderr)


if __name__ == "__main__":
    main()
