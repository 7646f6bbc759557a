"""Seeded synthetic inputs for the Kohn-Sham LOBPCG eigensolve.

This package only *describes and samples* the problem instances: atom
positions, the Gaussian local potential on the grid, the Gaussian
Kleinman-Bylander projector tables and the random initial orbital block.
It contains none of the eigensolver's arithmetic (no FFT, no Gram, no
factorisation).  Both the CPU oracle and the HIP path consume its output;
the oracle independently recomputes the potential and projectors from the
cell description and a test checks that the two agree.
"""
from .cells import (  # noqa: F401
    CellConfig,
    Cell,
    CONFIGS,
    config,
    custom_config,
    make_cell,
    make_x0,
    diamond_sites,
    bcc_sites,
)
