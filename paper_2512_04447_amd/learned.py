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
                   inputs: str = "residual", log=print) -> PairSet:
    """Run LOBPCG on one cell; after each step collect (input, target).

    ``inputs`` = "residual": the network sees the residual r (the plain
    learned preconditioner); "tpa": it sees the Teter-Payne-Allan output
    K_TPA(r), each column scaled by its own norm (the residual variant)."""
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
    P = torch.empty_like(R) if inputs == "tpa" else None
    dummy = torch.empty(nb, dtype=torch.float64, device="cuda")
    xs, ts, ths, its = [], [], [], []
    count = 0
    for it in range(n_iters):
        b.ks_precond_apply(plan, b.KS_PRECOND_NONE, lob.X, lob.AX, lob.theta, R, res, 0.0)
        b.ks_jd_correction(plan, v, lob.X, lob.theta, R, T, iters, maxit=cg_maxit, rtol=cg_rtol)
        if inputs == "tpa":
            b.ks_precond_apply(plan, b.KS_PRECOND_TPA, lob.X, lob.AX, lob.theta, P, dummy, 0.0)
            b.cnn_make_input(plan, P, None, v, lob.theta, xin)
        else:
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


def zero_last_layer(params):
    """Zero the weights and biases of the last convolution (flat layout
    w1, b1, w2, b2, w3, b3): the residual network then starts at its input."""
    n_w3 = 2 * 16 * 27
    params[-(n_w3 + 2):] = 0
    return params


def train_multi(sets, epochs: int, batch: int = 16, lr: float = 1e-3, seed: int = 2, val_frac: float = 0.1,
                log=print, params=None, skip: bool = False):
    """Adam over pairs from several grids: ``sets`` is a list of (plan, PairSet).

    Every batch comes from one grid (the convolution kernels take one grid
    per call); batches of all grids are shuffled together.  One parameter
    vector and one Adam state are shared.  Returns (params, history) with the
    validation loss (mean over held-out pairs of all grids) per epoch.
    """
    import torch

    rng = np.random.default_rng(seed)
    if params is None:
        p0 = kaiming_params(seed)
        params = torch.from_numpy(zero_last_layer(p0) if skip else p0).cuda()
    nets, splits = [], []
    for plan, pairs in sets:
        net = b.Cnn(plan, params, batch)
        if nets:
            net.params, net.m, net.v, net.grads = nets[0].params, nets[0].m, nets[0].v, nets[0].grads
        nets.append(net)
        n = pairs.x.shape[0]
        perm = rng.permutation(n)
        nval = max(1, int(round(val_frac * n)))
        splits.append((perm[:nval], perm[nval:]))
    step = [0]

    def evaluate():
        tot, cnt = 0.0, 0
        for net, (plan, pairs), (val, _) in zip(nets, sets, splits):
            for s0 in range(0, len(val), batch):
                j = torch.from_numpy(val[s0:s0 + batch]).cuda()
                net.forward(pairs.x[j], skip=skip)
                tot += float(net.loss_grad(pairs.t[j]).sum())
                cnt += len(j)
        return tot / max(cnt, 1)

    hist = [(0, evaluate())]
    log(f"[train] epoch 0 val loss {hist[-1][1]:.4f}")
    for ep in range(1, epochs + 1):
        t0 = time.time()
        work = []
        for g, (_, tr) in enumerate(splits):
            order = rng.permutation(tr)
            work.extend((g, order[s0:s0 + batch]) for s0 in range(0, len(order) - batch + 1, batch))
        for k in rng.permutation(len(work)):
            g, idx = work[k]
            net, pairs = nets[g], sets[g][1]
            j = torch.from_numpy(idx).cuda()
            xb, tb = pairs.x[j], pairs.t[j]
            net.forward(xb, skip=skip)
            net.loss_grad(tb)
            net.backward(xb)
            step[0] += 1
            net.t = step[0] - 1
            net.adam(lr)
        hist.append((ep, evaluate()))
        log(f"[train] epoch {ep} val loss {hist[-1][1]:.4f} ({time.time() - t0:.1f}s, {len(work)} batches)")
    return nets[0].params, hist


def run_to_tolerance(*args, **kwargs):
    """The driver of :mod:`paper_2512_04447_amd.solve` (kept here for callers
    of the training module)."""
    from .solve import run_to_tolerance as run

    return run(*args, **kwargs)


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


_WDIR = __import__("os").path.join(__import__("os").path.dirname(__file__), "weights")
WEIGHTS = __import__("os").path.join(_WDIR, "cnn_precond.npy")
WEIGHTS_TPA = __import__("os").path.join(_WDIR, "cnn_tpa.npy")


def main(argv=None):
    """Generate pairs on the 8-atom (16^3) and 64-atom (48^3) cells, train
    on the GPU and save the FP32 parameters."""
    import argparse
    import json
    import os
    import sys

    import torch

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import ksinputs as ki

    ap = argparse.ArgumentParser()
    ap.add_argument("--c1-seeds", type=int, default=8)
    ap.add_argument("--c1-iters", type=int, default=40)
    ap.add_argument("--c2-seeds", type=int, default=2)
    ap.add_argument("--c2-iters", type=int, default=25)
    ap.add_argument("--max-pairs", type=int, default=12000)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--variant", default="tpa", choices=["tpa", "residual"],
                    help="tpa: network on the TPA output with a skip connection; residual: network on r")
    ap.add_argument("--out", default=None)
    ap.add_argument("--log", default=None)
    a = ap.parse_args(argv)

    def log(*x):
        print(*x, flush=True)

    sets = []
    for name, nseed, nit in (("C1", a.c1_seeds, a.c1_iters), ("C2", a.c2_seeds, a.c2_iters)):
        cfg = ki.config(name)
        cell = ki.make_cell(cfg)
        parts = []
        for sd in range(1, nseed + 1):
            ps = generate_pairs(cell, cfg, ki.make_x0(cfg, seed=sd), nit, a.max_pairs // 2,
                                inputs="tpa" if a.variant == "tpa" else "residual", log=log)
            parts.append(ps)
        pairs = PairSet(torch.cat([p.x for p in parts]), torch.cat([p.t for p in parts]),
                        np.concatenate([p.theta for p in parts]), sum((p.iterations for p in parts), []))
        # the convolution kernels take only the grid from a plan
        plan = b.Plan(cell.n, cell.L, None, 16, b.KS_MIXED_FP32)
        log(f"[pairs] {name}: {pairs.x.shape[0]} pairs, CG iterations median {int(np.median(pairs.iterations))}")
        sets.append((plan, pairs))
    t0 = time.time()
    params, hist = train_multi(sets, a.epochs, log=log, skip=a.variant == "tpa")
    out = a.out or (WEIGHTS_TPA if a.variant == "tpa" else WEIGHTS)
    log(f"[train] {a.epochs} epochs in {time.time() - t0:.1f}s")
    os.makedirs(os.path.dirname(os.path.abspath(out)), exist_ok=True)
    np.save(out, params.cpu().numpy())
    log(f"[train] wrote {out}")
    if a.log:
        with open(a.log, "w") as f:
            json.dump({"variant": a.variant, "pairs": {n: int(s[1].x.shape[0]) for n, s in zip(("C1", "C2"), sets)},
                       "val_loss": hist}, f)


if __name__ == "__main__":
    main()
