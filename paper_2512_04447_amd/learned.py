"""Learned LOBPCG preconditioner: data generation and training drivers.

Training pairs come from the method itself: LOBPCG (with the
Teter-Payne-Allan preconditioner) runs on small cells; at every iterate the
residual r_i of each band and the correction t_i solving the
Jacobi-Davidson-projected equation P (H - theta_i) P t_i = P r_i are formed
by the library (``ks_precond_apply``, ``ks_jd_correction``).  The network
(3 -> 16 -> 16 -> 2 periodic 3x3x3 convolutions) is trained with the
library's forward/backward kernels and Adam.  This module only orchestrates
calls and moves tensors; every arithmetic step runs in libksh.so.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass

import numpy as np

from . import binding as b


def kaiming_params(seed: int = 2) -> np.ndarray:
    """Flat FP32 parameter vector, Kaiming-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)
    out = []
    for cin, cout in ((3, 16), (16, 16), (16, 2)):
        bound = math.sqrt(6.0 / (cin * 27))
        out.append(rng.uniform(-bound, bound, size=(cout, cin, 3, 3, 3)).ravel())
        out.append(np.zeros(cout))
    return np.concatenate(out).astype(np.float32)


@dataclass
class PairSet:
    x: "object"  # torch float32 (N, 3, Ng)
    t: "object"  # torch float32 (N, 2, Ng)
    theta: np.ndarray
    iterations: list


def generate_pairs(cell, cfg, X0, n_iters: int, max_pairs: int, cg_maxit: int = 300, cg_rtol: float = 1e-6,
                   log=print) -> PairSet:
    """Run LOBPCG on one cell; after each step collect (input, target)."""
    import torch

    proj = b.ProjectorArrays.from_cell(cell) if cell.nproj else None
    nb = cfg.nb
    plan = b.Plan(cell.n, cell.L, proj, nb, b.KS_FP64)
    v = torch.from_numpy(cell.V).cuda()
    lob = b.Lobpcg(plan, v, torch.from_numpy(X0).cuda())
    lob.init()
    R = torch.empty((nb, plan.Ng), dtype=torch.complex128, device="cuda")
    T = torch.empty_like(R)
    res = torch.empty(nb, dtype=torch.float64, device="cuda")
    iters = torch.zeros(nb, dtype=torch.int32, device="cuda")
    xin = torch.empty((nb, 3, plan.Ng), dtype=torch.float32, device="cuda")
    xs, ts, ths, its = [], [], [], []
    count = 0
    for it in range(n_iters):
        b.ks_precond_apply(plan, b.KS_PRECOND_NONE, lob.X, lob.AX, lob.theta, R, res, 0.0)
        b.ks_jd_correction(plan, v, lob.X, lob.theta, R, T, iters, maxit=cg_maxit, rtol=cg_rtol)
        b.cnn_make_input(plan, R, res, v, lob.theta, xin)
        ok = (iters > 0) & (res > 1e-12)
        sel = torch.nonzero(ok).flatten()
        if sel.numel():
            xs.append(xin[sel].clone())
            # target channels: real and imaginary parts of t (layout only)
            tt = torch.view_as_real(T[sel]).permute(0, 2, 1).to(torch.float32).contiguous()
            ts.append(tt)
            ths.append(lob.theta[sel].cpu().numpy())
            its.extend(iters[sel].cpu().tolist())
            count += sel.numel()
        log(f"[pairs] {cfg.name} iter {it}: {sel.numel()} pairs (total {count}), max res {float(res.max()):.2e}")
        if count >= max_pairs:
            break
        lob.step(b.KS_PRECOND_TPA, 0.0)
    x = torch.cat(xs)[:max_pairs]
    t = torch.cat(ts)[:max_pairs]
    return PairSet(x, t, np.concatenate(ths)[:max_pairs], its[:max_pairs])


def train(plan, pairs: PairSet, epochs: int, batch: int = 16, lr: float = 1e-3, seed: int = 2, val_frac: float = 0.1,
          log=print):
    """Adam on the scale-invariant loss; returns (params tensor, history)."""
    import torch

    n = pairs.x.shape[0]
    rng = np.random.default_rng(seed)
    perm = rng.permutation(n)
    nval = max(1, int(round(val_frac * n)))
    val, tr = perm[:nval], perm[nval:]
    net = b.Cnn(plan, torch.from_numpy(kaiming_params(seed)).cuda(), batch)
    hist = []

    def evaluate(idx):
        tot = 0.0
        for s in range(0, len(idx), batch):
            j = torch.from_numpy(idx[s:s + batch]).cuda()
            xb, tb = pairs.x[j], pairs.t[j]
            net.forward(xb)
            tot += float(net.loss_grad(tb).sum())
        return tot / len(idx)

    hist.append((0, evaluate(val)))
    log(f"[train] epoch 0 val loss {hist[-1][1]:.4f}")
    for ep in range(1, epochs + 1):
        t0 = time.time()
        order = rng.permutation(tr)
        for s in range(0, len(order) - batch + 1, batch):
            j = torch.from_numpy(order[s:s + batch]).cuda()
            xb, tb = pairs.x[j], pairs.t[j]
            net.forward(xb)
            net.loss_grad(tb)
            net.backward(xb)
            net.adam(lr)
        hist.append((ep, evaluate(val)))
        log(f"[train] epoch {ep} val loss {hist[-1][1]:.4f} ({time.time() - t0:.1f}s)")
    return net.params, hist
