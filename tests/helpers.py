"""Shared test helpers: seeded problems evaluated on each side's own nodes."""
from __future__ import annotations

import functools
import sys

import numpy as np

import hps_inputs as hi
from oracle import hps


def say(msg: str) -> None:
    print(msg, flush=True)
    sys.stdout.flush()


def rel_err(a, b) -> float:
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def oracle_problem(pr: hi.Problem, nleaf=None, **kw):
    """Oracle operator + coefficients at the oracle's Chebyshev nodes + boundary data."""
    nleaf = tuple(nleaf or pr.nleaf)
    grid = hps.Grid(pr.box, nleaf[0], nleaf[1], pr.q)
    C = pr.coeffs_at(grid.cheb_xy(pr.p))
    op = hps.build(C, pr.box, nleaf, pr.p, pr.q, **kw)
    f = pr.bc_at(hps.gamma_xy(op))
    return op, C, f, grid


def library_inputs(pr: hi.Problem, nleaf=None):
    """Coefficients and boundary data evaluated at the library's own nodes."""
    import paper_1307_2665_amd as H
    nleaf = tuple(nleaf or pr.nleaf)
    xy = H.cheb_nodes(pr.box, nleaf, pr.p)
    C = pr.coeffs_at(xy)
    gxy = H.gauss_nodes_grid(pr.box, nleaf, pr.q)
    ids = H.boundary_ids(nleaf, pr.q)
    f = pr.bc_at(gxy[ids])
    return C, f


def hbs_oracle_factors(fac: dict, L: int, m: int, k: int) -> dict:
    """The generator's HBS blocks (library layout: V stored as V*) as the oracle's dict."""
    F = dict(L=L, m=m, M=m << L, D=[fac["D"][j] for j in range(1 << L)], U={}, V={}, B={})
    for j in range(1 << L):
        F["U"][(L, j)] = fac["U"][j]
        F["V"][(L, j)] = fac["Vt"][j].T
    for l in range(1, L):
        for j in range(1 << l):
            F["U"][(l, j)] = fac["Up"][l][j]
            F["V"][(l, j)] = fac["Vtp"][l][j].T
    for l in range(L):
        for j in range(1 << l):
            F["B"][(l, j)] = fac["B"][l][j]
    return F
