"""Write the oracle's converged eigenvalues of the 64-atom diamond-like cell.

Cell: diamond 2x2x2 supercell, L = 13.48 bohr, 48^3 grid, 160 bands,
Gaussian local potential (depth -2 Ha, sigma 0.8 bohr) and s+p Gaussian KB
projectors (rc = 1.0 bohr, couplings uniform in [-1, 1] Ha, seed 0), random
initial block (seed 1).  Runs the CPU oracle's LOBPCG with the
Teter-Payne-Allan preconditioner until the 128 tracked bands reach a residual
norm of 1e-8 and writes every Ritz value and residual.

Calls only oracle/ (and the seeded input generator).  Takes about ten
minutes on 8 cores.
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import ksinputs as ki  # noqa: E402
from oracle import hamiltonian as oh  # noqa: E402
from oracle import lobpcg as olob  # noqa: E402


def main(out=os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_eigenvalues.txt")):
    cfg = ki.config("C2")
    cell = ki.make_cell(cfg)
    oc = oh.oracle_cell(cfg, cell.D)
    X0 = ki.make_x0(cfg)
    t0 = time.time()
    it = [0]

    def cb(st, res):
        print(f"iter {it[0]:3d}  max tracked res {res[:cfg.ntrack].max():.3e}  t={time.time() - t0:.0f}s", flush=True)
        it[0] += 1

    st, hist = olob.run(oc, X0, cfg.ntrack, tol=1e-8, maxit=200, precond=olob.tpa_preconditioner(oc), callback=cb)
    theta, res = hist[-1]
    with open(out, "w") as f:
        f.write("# oracle LOBPCG (FP64, TPA preconditioner, lock at 0.1*tol), diamond 2x2x2, 48^3, 160 bands\n")
        f.write(f"# iterations {len(hist) - 1}, max tracked residual {res[:cfg.ntrack].max():.3e}\n")
        f.write("# band  theta_Ha  residual_norm\n")
        for i, (t, r) in enumerate(zip(theta, res)):
            f.write(f"{i:4d} {t:.17e} {r:.3e}\n")
    print(f"wrote {out} after {len(hist) - 1} iterations in {time.time() - t0:.0f}s")


if __name__ == "__main__":
    main()
