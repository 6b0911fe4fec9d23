"""Plain FP64 oracle of HBS matrices (section 6) and their fast inversion (section 7).

Test infrastructure only (see ``oracle/__init__.py``).

An HBS matrix H of size M = m 2^L is tied to the uniform binary tree of
section 6.3: level l has the 2^l nodes j = 0 .. 2^l - 1, node (l, j) owns the
contiguous index range [j M / 2^l, (j + 1) M / 2^l), and its children are
(l + 1, 2j) and (l + 1, 2j + 1).  The factors of section 6.4 (the table of its
figure of factor sizes) are kept in a dict:

* ``D[j]``       -- leaf j's diagonal block H(I_j, I_j) (eq:def5);
* ``U[(l, j)]``, ``V[(l, j)]`` -- the bases of node (l, j) for l = 1 .. L
  (rows x rank, one rank for both: m rows at a leaf, the sum of the
  children's ranks at a parent);
* ``B[(l, j)]``  -- for every parent, l = 0 .. L-1, the interaction block of its
  children, [[0, Ht12], [Ht21, 0]] (eq:def6).

Ranks may differ from node to node; the GPU form keeps one rank k everywhere.

Functions:

* ``compress``  -- dense H to HBS factors by brute force (Remark 8.2: the dense
  matrices of the finer levels are compressed directly), with orthonormal
  nested bases taken from SVDs of the (reduced) off-diagonal block rows and
  columns (the rank conditions eq:def2 and eq:def4).
* ``to_dense``  -- the telescoping factorization eq:tele1 - eq:tele3 written out
  with block-diagonal matrices.
* ``apply``     -- y = H x through the same factorization, one level at a time.
* ``invert``    -- Algorithm 3 (factors E, F, G of H^-1).
* ``solve``     -- Algorithm 4 (y = H^-1 x).  Its downward and leaf lines
  multiply E by y-hat of the parent (the printed q-hat and x-hat there are read
  as y-hat: with a single level the algorithm must reduce to eq:woodbury,
  H^-1 = E (Ht + Dhat)^-1 F* + G, which needs y-hat).
* ``low_rank``  -- thin factors X Y of a matrix of low numerical rank, as the
  solve stage of section 8 uses for S.
"""
from __future__ import annotations

from typing import Dict, Optional, Tuple

import numpy as np
import scipy.linalg as sla


def node_range(M: int, l: int, j: int) -> slice:
    """Index range of node (l, j) of the uniform tree of section 6.3."""
    w = M >> l
    return slice(j * w, (j + 1) * w)


def _complement(M: int, l: int, j: int) -> np.ndarray:
    w = M >> l
    return np.r_[0:j * w, (j + 1) * w:M]


def _bases(R: np.ndarray, C: np.ndarray, tol_abs: Optional[float],
           rank: Optional[int]) -> Tuple[np.ndarray, np.ndarray]:
    """Orthonormal bases of the leading left singular vectors of R and of C,
    of one common size (Algorithm 3 inverts V* Dt^-1 U, which must be
    square): the larger of the two counts of singular values above tol_abs,
    or ``rank``."""
    Qr, sr, _ = np.linalg.svd(R, full_matrices=False)
    Qc, sc, _ = np.linalg.svd(C, full_matrices=False)
    if rank is not None:
        r = rank
    else:
        r = max(int(np.sum(sr > tol_abs)), int(np.sum(sc > tol_abs)), 1)
    r = min(r, Qr.shape[1], Qc.shape[1])
    return Qr[:, :r], Qc[:, :r]


def compress(H: np.ndarray, L: int, tol: Optional[float] = None,
             rank: Optional[int] = None) -> Dict:
    """HBS factors of the dense M x M matrix H on a tree of L levels (section 6.4).

    Either ``tol`` (singular values above tol * ||H||_2 are kept at every node)
    or a fixed ``rank`` per node.  Bases are orthonormal, so the middle blocks
    of eq:def2 / eq:def4 are projections: Ht(s1, s2) = Ubig(s1)* H(I_s1, I_s2)
    Vbig(s2), with Ubig the node's basis expressed in the original indices.
    """
    M = H.shape[0]
    assert H.shape == (M, M) and L >= 1 and M % (1 << L) == 0
    assert (tol is None) != (rank is None)
    m = M >> L
    tol_abs = None if tol is None else tol * np.linalg.norm(H, 2)
    U, V, Ub, Vb, B = {}, {}, {}, {}, {}
    D = [H[node_range(M, L, j), node_range(M, L, j)].copy() for j in range(1 << L)]
    for l in range(L, 0, -1):
        for j in range(1 << l):
            I, Ic = node_range(M, l, j), _complement(M, l, j)
            row_blk = H[I][:, Ic]               # off-diagonal block row of the node
            col_blk = H[Ic][:, I].T             # its off-diagonal block column, transposed
            if l < L:
                c1, c2 = (l + 1, 2 * j), (l + 1, 2 * j + 1)
                P = sla.block_diag(Ub[c1], Ub[c2])
                Q = sla.block_diag(Vb[c1], Vb[c2])
                row_blk = P.T @ row_blk          # reduced to the children's bases (eq:def3)
                col_blk = Q.T @ col_blk
            U[(l, j)], V[(l, j)] = _bases(row_blk, col_blk, tol_abs, rank)
            Ub[(l, j)] = U[(l, j)] if l == L else P @ U[(l, j)]
            Vb[(l, j)] = V[(l, j)] if l == L else Q @ V[(l, j)]
    for l in range(L - 1, -1, -1):
        for j in range(1 << l):
            c1, c2 = (l + 1, 2 * j), (l + 1, 2 * j + 1)
            I1, I2 = node_range(M, *c1), node_range(M, *c2)
            h12 = Ub[c1].T @ H[I1, I2] @ Vb[c2]
            h21 = Ub[c2].T @ H[I2, I1] @ Vb[c1]
            B[(l, j)] = np.block([[np.zeros((h12.shape[0], h21.shape[1])), h12],
                                  [h21, np.zeros((h21.shape[0], h12.shape[1]))]])
    return dict(L=L, m=m, M=M, D=D, U=U, V=V, B=B)


def ranks(F: Dict) -> Dict[Tuple[int, int], int]:
    """Rank of every non-root node's basis."""
    return {key: u.shape[1] for key, u in F["U"].items()}


def to_dense(F: Dict) -> np.ndarray:
    """H from its factors by eq:tele1 - eq:tele3: Ht(1) = B(0), then
    Ht(l+1) = U(l) Ht(l) V(l)* + B(l) for l = 1 .. L-1, and
    H = U(L) Ht(L) V(L)* + D(L), with the underlined block-diagonal matrices
    of section 6.5."""
    L = F["L"]
    Ht = F["B"][(0, 0)]
    for l in range(1, L + 1):
        Ul = sla.block_diag(*[F["U"][(l, j)] for j in range(1 << l)])
        Vl = sla.block_diag(*[F["V"][(l, j)] for j in range(1 << l)])
        if l < L:
            Bl = sla.block_diag(*[F["B"][(l, j)] for j in range(1 << l)])
        else:
            Bl = sla.block_diag(*F["D"])
        Ht = Ul @ Ht @ Vl.T + Bl
    return Ht


def apply(F: Dict, x: np.ndarray) -> np.ndarray:
    """y = H x through the telescoping factorization, node by node: x-hat up
    the tree through V*, the sibling blocks of B, y-hat down through U, and the
    leaves' D."""
    L, M = F["L"], F["M"]
    x = np.asarray(x, dtype=np.float64)
    xh = {}
    for j in range(1 << L):
        xh[(L, j)] = F["V"][(L, j)].T @ x[node_range(M, L, j)]
    for l in range(L - 1, 0, -1):
        for j in range(1 << l):
            xc = np.concatenate([xh[(l + 1, 2 * j)], xh[(l + 1, 2 * j + 1)]])
            xh[(l, j)] = F["V"][(l, j)].T @ xc
    yh = {}
    for l in range(0, L):
        for j in range(1 << l):
            c1, c2 = (l + 1, 2 * j), (l + 1, 2 * j + 1)
            k1 = xh[c1].shape[0]
            yc = F["B"][(l, j)] @ np.concatenate([xh[c1], xh[c2]])
            if l > 0:
                yc = yc + F["U"][(l, j)] @ yh[(l, j)]
            yh[c1], yh[c2] = yc[:k1], yc[k1:]
    y = np.empty_like(x)
    for j in range(1 << L):
        I = node_range(M, L, j)
        y[I] = F["U"][(L, j)] @ yh[(L, j)] + F["D"][j] @ x[I]
    return y


def invert(F: Dict) -> Dict:
    """Algorithm 3: factors {E, F, G} of H^-1, finer levels first.

    For each node, Dt is its leaf block D, or for a parent the children's
    Dhat with the parent's sibling blocks off the diagonal; then
    Dhat = (V* Dt^-1 U)^-1, E = Dt^-1 U Dhat, F* = Dhat V* Dt^-1 and
    G = Dt^-1 - Dt^-1 U Dhat V* Dt^-1.  The root keeps
    G = [[Dhat_2, B_23], [B_32, Dhat_3]]^-1."""
    L = F["L"]
    E, Fs, G, Dh = {}, {}, {}, {}

    def dtilde(l, j):
        c1, c2 = (l + 1, 2 * j), (l + 1, 2 * j + 1)
        Bt = F["B"][(l, j)]
        k1 = Dh[c1].shape[0]
        return np.block([[Dh[c1], Bt[:k1, k1:]], [Bt[k1:, :k1], Dh[c2]]])

    for l in range(L, 0, -1):
        for j in range(1 << l):
            Dt = F["D"][j] if l == L else dtilde(l, j)
            Dinv = np.linalg.inv(Dt)
            Un, Vn = F["U"][(l, j)], F["V"][(l, j)]
            Dh[(l, j)] = np.linalg.inv(Vn.T @ Dinv @ Un)
            E[(l, j)] = Dinv @ Un @ Dh[(l, j)]
            Fs[(l, j)] = Dh[(l, j)] @ Vn.T @ Dinv
            G[(l, j)] = Dinv - Dinv @ Un @ Dh[(l, j)] @ Vn.T @ Dinv
    G[(0, 0)] = np.linalg.inv(dtilde(0, 0))
    return dict(L=L, m=F["m"], M=F["M"], E=E, Fs=Fs, G=G)


def solve(Fi: Dict, x: np.ndarray) -> np.ndarray:
    """Algorithm 4: y = H^-1 x from the factors of ``invert``."""
    L, M = Fi["L"], Fi["M"]
    x = np.asarray(x, dtype=np.float64)
    xh = {}
    for j in range(1 << L):
        xh[(L, j)] = Fi["Fs"][(L, j)] @ x[node_range(M, L, j)]
    for l in range(L - 1, 0, -1):
        for j in range(1 << l):
            xh[(l, j)] = Fi["Fs"][(l, j)] @ np.concatenate([xh[(l + 1, 2 * j)], xh[(l + 1, 2 * j + 1)]])
    yh = {}
    k1 = xh[(1, 0)].shape[0]
    y0 = Fi["G"][(0, 0)] @ np.concatenate([xh[(1, 0)], xh[(1, 1)]])
    yh[(1, 0)], yh[(1, 1)] = y0[:k1], y0[k1:]
    for l in range(1, L):
        for j in range(1 << l):
            c1, c2 = (l + 1, 2 * j), (l + 1, 2 * j + 1)
            k1 = xh[c1].shape[0]
            yc = Fi["E"][(l, j)] @ yh[(l, j)] + Fi["G"][(l, j)] @ np.concatenate([xh[c1], xh[c2]])
            yh[c1], yh[c2] = yc[:k1], yc[k1:]
    y = np.empty_like(x)
    for j in range(1 << L):
        I = node_range(M, L, j)
        y[I] = Fi["E"][(L, j)] @ yh[(L, j)] + Fi["G"][(L, j)] @ x[I]
    return y


def low_rank(A: np.ndarray, tol: float) -> Tuple[np.ndarray, np.ndarray]:
    """Thin factors X (rows x r) and Y (r x cols) with A = X Y up to the
    singular values not above tol ||A||_2 (truncated SVD)."""
    Q, s, Wt = np.linalg.svd(A, full_matrices=False)
    r = int(np.sum(s > tol * s[0])) if s.size and s[0] > 0 else 0
    return Q[:, :r] * s[:r], Wt[:r]
