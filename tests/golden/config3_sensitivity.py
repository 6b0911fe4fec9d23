"""How far correct FP64 computations of config 3 spread (CPU, oracle only).

Config 3 (variable Helmholtz, kappa = 40, Gaussian bump; 128 x 128 leaves,
p = 16, q = 14) is close to a resonance, so its solution reacts strongly to
rounding-level changes of the leaf DtN maps.  This script compares the stored
oracle solution (tests/golden/config3.npz, right-hand sides 0 and 63) with

* the oracle with the other tree order (split x2 first on ties),
* the oracle with every leaf solve done by Householder QR instead of LU,
* the oracle with every leaf DtN multiplied entrywise by 1 + 1e-14 z,
  z standard normal (seeded),

and prints cond2 of the merge matrices of the top three depths.  Run from the
repository root: python tests/golden/config3_sensitivity.py  (about 10 min).
"""
from __future__ import annotations

import os
import sys
import warnings

import numpy as np
import scipy.linalg as sla

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import hps_inputs as hi  # noqa: E402
from oracle import hps  # noqa: E402


def leaf_qr(coef, p, q, hx, hy, mats=None):
    m = mats if mats is not None else hps.leaf_matrices(p, q, hx, hy)
    A = hps.collocation_matrix(coef, m)
    Je, Ji = m["Je"], m["Ji"]
    Qm, Rm = np.linalg.qr(A[np.ix_(Ji, Ji)])
    X = -sla.solve_triangular(Rm, Qm.T @ A[np.ix_(Ji, Je)])
    L2 = np.zeros((p * p, len(Je)))
    L2[Je, :] = np.eye(len(Je))
    L2[Ji, :] = X
    return hps.LeafOp(T=m["L4"] @ m["L3"] @ L2 @ m["L1"], X=X, L1=m["L1"], Je=Je, Ji=Ji)


def main():
    warnings.simplefilter("ignore")
    g = np.load(os.path.join(HERE, "config3.npz"), allow_pickle=False)
    pr = hi.helmholtz_bump()
    nx, ny = pr.nleaf
    grid = hps.Grid(pr.box, nx, ny, pr.q)
    C = pr.coeffs_at(grid.cheb_xy(pr.p))

    def run(label, **kw):
        op = hps.build(C, pr.box, (nx, ny), pr.p, pr.q, keep=False, **kw)
        u = hps.solve(op, pr.bc_at(hps.gamma_xy(op))[list(g["rhs"])])
        d = [float(np.max(np.abs(u[k] - g["u"][k])) / np.max(np.abs(g["u"][k])))
             for k in range(len(g["rhs"]))]
        print(f"{label}: rel diff to the stored oracle u, rhs {list(g['rhs'])}: "
              + ", ".join(f"{x:.2e}" for x in d), flush=True)
        return op

    op = run("tree split x2 first", x_first=False)
    for t, mo in op.merges.items():
        if op.boxes[t].level <= 2:
            s = np.linalg.svd(mo.M, compute_uv=False)
            print(f"  (x2-first tree) box {t} depth {op.boxes[t].level}: cond2(M) {s[0] / s[-1]:.2e}")
    del op
    orig = hps.leaf_dtn
    hps.leaf_dtn = leaf_qr
    run("leaf solves by QR")
    rng = np.random.default_rng(1)

    def perturbed(*a, **k):
        lo = orig(*a, **k)
        lo.T = lo.T * (1.0 + 1e-14 * rng.standard_normal(lo.T.shape))
        return lo

    hps.leaf_dtn = perturbed
    run("leaf DtNs times (1 + 1e-14 z)")
    hps.leaf_dtn = orig
    op = hps.build(C, pr.box, (nx, ny), pr.p, pr.q, keep=False)
    for t, mo in op.merges.items():
        if op.boxes[t].level <= 2:
            s = np.linalg.svd(mo.M, compute_uv=False)
            print(f"box {t} depth {op.boxes[t].level}: cond2(M) {s[0] / s[-1]:.2e}")


if __name__ == "__main__":
    main()
