"""Writes the stored oracle results that the full-size GPU parity tests read.

Calls only the CPU oracle (``oracle/``) and the seeded input recipes
(``hps_inputs``); nothing here touches the GPU library.  Run from the
repository root:

    python tests/golden/make_golden.py [config2 config3 config5]

Each problem is evaluated at the oracle's own nodes and solved by the oracle's
Algorithms 1 and 2 in FP64 (all merges, every Gauss node):

* ``config2.npz``: convection-diffusion, 64 x 64 leaves, p = 16, q = 14,
  f = cos(2 x1)(1 - 2 x2); u at all 116,480 Gauss nodes.
* ``config3.npz``: variable Helmholtz (kappa = 40, Gaussian bump), 128 x 128
  leaves, p = 16, q = 14; u for right-hand sides 0 and 63 of the 64 seeded
  ones (seeds 3000 and 3063) at all 462,336 Gauss nodes, and 16 rows of the
  7168 x 7168 root DtN (rows 0, 448, ..., 6720).
* ``config5.npz``: sweep field 5000 (c11 = c22 = 1 + g/2, c = 1 + g'),
  256 x 256 leaves, p = 12, q = 10; u at all 1,315,840 Gauss nodes.
"""
from __future__ import annotations

import os
import sys
import time
import warnings

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import hps_inputs as hi  # noqa: E402
from oracle import hps  # noqa: E402

ROOT_ROWS = np.arange(0, 7168, 448)


def _solve(pr, rhs=None):
    nx, ny = pr.nleaf
    grid = hps.Grid(pr.box, nx, ny, pr.q)
    C = pr.coeffs_at(grid.cheb_xy(pr.p))
    t0 = time.time()
    op = hps.build(C, pr.box, (nx, ny), pr.p, pr.q)
    f = pr.bc_at(hps.gamma_xy(op))
    if rhs is not None:
        f = f[rhs]
    u = hps.solve(op, f)
    print(f"{pr.name} {nx}x{ny} p={pr.p} q={pr.q}: oracle {time.time() - t0:.1f} s", flush=True)
    return op, u


def config2():
    op, u = _solve(hi.convdiff())
    np.savez_compressed(os.path.join(HERE, "config2.npz"), u=u)


def config3():
    rhs = [0, 63]
    op, u = _solve(hi.helmholtz_bump(), rhs=rhs)
    np.savez_compressed(os.path.join(HERE, "config3.npz"), u=u, rhs=np.array(rhs),
                        root_rows=ROOT_ROWS, rootT_rows=op.rootT[ROOT_ROWS])


def config5():
    op, u = _solve(hi.sweep_field(5000))
    np.savez_compressed(os.path.join(HERE, "config5.npz"), u=u)


if __name__ == "__main__":
    warnings.simplefilter("ignore")
    which = sys.argv[1:] or ["config2", "config3", "config5"]
    for w in which:
        globals()[w]()
