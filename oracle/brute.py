"""Brute-force global solves that pin the hierarchical oracle (Remark 5.1).

Test infrastructure only (see ``oracle/__init__.py``).

Remark 5.1 says the merges are exact in exact arithmetic, so the hierarchical
build/solve must reproduce, up to rounding, the solution of one global discrete
system.  Two independent assemblies of that system are provided:

* ``collocation_solve``: the full composite collocation system.  Unknowns are the
  Gauss values on interior edges and every leaf's interior Chebyshev values;
  equations are every leaf's interior collocation rows (eq:A_interior, with the
  boundary Chebyshev values obtained from the Gauss values by step 1 of section
  3.2) and flux matching at every interior Gauss node (flux by steps 3 and 4).
  No leaf DtN and no merge is formed.
* ``interface_solve`` / ``interface_root_dtn``: the system on the Gauss nodes
  alone, assembled from the leaf DtNs (eq:bittersweet1 for every leaf pair),
  solved densely; this pins the merges on their own.
"""
from __future__ import annotations

import numpy as np

from . import hps


def _leaf_blocks(coef, mats):
    A = hps.collocation_matrix(coef, mats)
    Je, Ji = mats["Je"], mats["Ji"]
    F = mats["L4"] @ mats["L3"]              # Chebyshev potential -> Gauss fluxes, [4q, p^2]
    return A[np.ix_(Ji, Ji)], A[np.ix_(Ji, Je)], F[:, Je], F[:, Ji]


def _side_sign(q):
    # E and N sides: the leaf is alpha of the edge (+); S and W: beta (-).
    return np.concatenate([-np.ones(q), np.ones(q), np.ones(q), -np.ones(q)])


def collocation_solve(coeffs, box, nleaf, p, q, f, with_interior=False, body=None):
    """Solve the full composite collocation system densely; returns u at all Gauss nodes.

    With with_interior=True also returns every leaf's interior Chebyshev values,
    [nx*ny, (p-2)^2] in ascending node order, the unknowns w_i of the same
    global system (section 5.3 recovers them leaf by leaf).  body [nx*ny, p*p]
    is a body load g (A u = g) at the Chebyshev nodes: it becomes the
    right-hand side of the interior collocation rows."""
    nx, ny = nleaf
    grid = hps.Grid(box, nx, ny, q)
    gamma = grid.boundary(0, nx, 0, ny)
    on_gamma = np.zeros(grid.N, dtype=bool)
    on_gamma[gamma] = True
    interior = np.nonzero(~on_gamma)[0]
    col_of = -np.ones(grid.N, dtype=np.int64)
    col_of[interior] = np.arange(len(interior))
    ni = (p - 2) ** 2
    nleafs = nx * ny
    nunk = len(interior) + nleafs * ni
    K = np.zeros((nunk, nunk))
    rhs = np.zeros(nunk)
    ufix = np.zeros(grid.N)
    ufix[gamma] = f
    mats = hps.leaf_matrices(p, q, grid.hx, grid.hy)
    sgn = _side_sign(q)
    row = 0
    flux_row0 = nleafs * ni
    for j in range(ny):
        for i in range(nx):
            lf = i + nx * j
            Aii, Aie, Fe, Fi = _leaf_blocks(coeffs[lf], mats)
            Ie = grid.boundary(i, i + 1, j, j + 1)
            wcol = len(interior) + lf * ni
            # Interior collocation rows: Aii w_i + Aie L1 u_d = g_i (0 without a load).
            G = Aie @ mats["L1"]                      # acts on the 4q Gauss values
            K[row:row + ni, wcol:wcol + ni] = Aii
            if body is not None:
                rhs[row:row + ni] += np.asarray(body)[lf][mats["Ji"]]
            for k, g in enumerate(Ie):
                if on_gamma[g]:
                    rhs[row:row + ni] -= G[:, k] * ufix[g]
                else:
                    K[row:row + ni, col_of[g]] += G[:, k]
            row += ni
            # Flux contributions at interior Gauss nodes: flux = Fe L1 u_d + Fi w_i.
            H = Fe @ mats["L1"]
            for k, g in enumerate(Ie):
                if on_gamma[g]:
                    continue
                r = flux_row0 + col_of[g]
                K[r, wcol:wcol + ni] += sgn[k] * Fi[k, :]
                for kk, gg in enumerate(Ie):
                    if on_gamma[gg]:
                        rhs[r] -= sgn[k] * H[k, kk] * ufix[gg]
                    else:
                        K[r, col_of[gg]] += sgn[k] * H[k, kk]
    x = np.linalg.solve(K, rhs)
    u = ufix.copy()
    ni_g = len(interior)
    u[interior] = x[:ni_g]
    if with_interior:
        return u, x[ni_g:].reshape(nleafs, ni)
    return u


def _interface_matrix(grid, leafT_by_ij, q):
    """Rows: flux jump at interior nodes and flux at Gamma nodes, as a matrix on all N nodes."""
    nx, ny = grid.nx, grid.ny
    Jmp = np.zeros((grid.N, grid.N))
    sgn = _side_sign(q)
    for j in range(ny):
        for i in range(nx):
            T = leafT_by_ij[(i, j)]
            Ie = grid.boundary(i, i + 1, j, j + 1)
            Jmp[np.ix_(Ie, Ie)] += sgn[:, None] * T
    return Jmp


def interface_solve(op: hps.Operator, f):
    """Dense solve of 'flux jump = 0 at interior nodes, u = f on Gamma' from leaf DtNs."""
    grid = op.grid
    leafT = {(op.boxes[t].i0, op.boxes[t].j0): T for t, T in op.leafT.items()}
    J = _interface_matrix(grid, leafT, op.q)
    gamma = op.boxes[0].Ie
    on_gamma = np.zeros(grid.N, dtype=bool)
    on_gamma[gamma] = True
    I = np.nonzero(~on_gamma)[0]
    u = np.zeros(grid.N)
    u[gamma] = f
    u[I] = np.linalg.solve(J[np.ix_(I, I)], -J[np.ix_(I, gamma)] @ f)
    return u


def interface_root_dtn(op: hps.Operator):
    """Root DtN as the Schur complement of the interface system onto Gamma.

    On Gamma each node belongs to exactly one leaf, so the 'jump' rows there are
    that leaf's flux with sign -1 on its S/W sides; undo the sign to get v.
    """
    grid = op.grid
    leafT = {(op.boxes[t].i0, op.boxes[t].j0): T for t, T in op.leafT.items()}
    J = _interface_matrix(grid, leafT, op.q)
    gamma = op.boxes[0].Ie
    on_gamma = np.zeros(grid.N, dtype=bool)
    on_gamma[gamma] = True
    I = np.nonzero(~on_gamma)[0]
    X = -np.linalg.solve(J[np.ix_(I, I)], J[np.ix_(I, gamma)])
    V = J[np.ix_(gamma, gamma)] + J[np.ix_(gamma, I)] @ X
    # Sign of each Gamma node's own leaf side: S/W of the root are S/W of leaves (-).
    nq = len(gamma) // 1
    sg = np.empty(nq)
    nx, ny, q = grid.nx, grid.ny, grid.q
    sg[:nx * q] = -1.0                       # S
    sg[nx * q:(nx + ny) * q] = 1.0           # E
    sg[(nx + ny) * q:(2 * nx + ny) * q] = 1.0  # N
    sg[(2 * nx + ny) * q:] = -1.0            # W
    return sg[:, None] * V
