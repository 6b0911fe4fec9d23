"""Plain FP64 oracle of the dense composite spectral solver (sections 2-5).

Test infrastructure only (see ``oracle/__init__.py``).

Conventions (the paper leaves them open; the readings are listed in the design
notes of the repository):

* Leaf grid: Chebyshev-Lobatto points x_j = -cos(j pi / (p-1)), ascending, in
  each direction (section 3.1, Trefethen's nodes); node (a, b) -> a + p*b with a
  counting along x1.
* Edge nodes: q Gauss-Legendre points per leaf edge (section 2).
* Every box boundary is ordered S (x1 ascending), E (x2 ascending),
  N (x1 ascending), W (x2 ascending).
* Fluxes follow section 2: v = du/dx2 on horizontal edges and du/dx1 on
  vertical edges (not the outward normal).
* Tree: split the longer side (in leaf units) at floor(n/2), x1 first on ties;
  the west/south child is alpha, the east/north child is beta.
* Global Gauss numbering: horizontal edge (i, j) (i < nx, j <= ny) has id
  j*nx + i; vertical edge (i, j) (i <= nx, j < ny) has id
  nx*(ny+1) + j*(nx+1) + i; node k of an edge is id*q + k, ascending along
  the edge.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np
import scipy.linalg as sla


# ---------------------------------------------------------------------------
# Section 2 / 3.1: nodes, spectral differentiation, interpolation.
# ---------------------------------------------------------------------------

def cheb_points(p: int) -> np.ndarray:
    """Chebyshev-Lobatto points on [-1, 1], ascending (section 3.1)."""
    j = np.arange(p)
    return -np.cos(np.pi * j / (p - 1))


def cheb_diff(p: int) -> np.ndarray:
    """Spectral differentiation matrix on ``cheb_points(p)``.

    Off-diagonal entries from the closed form for Chebyshev-Lobatto points,
    D_ij = (c_i / c_j) (-1)^(i+j) / (x_i - x_j) with c = 2 at both ends and 1
    inside; the diagonal by the negative-sum rule (each row annihilates
    constants).  Trefethen, Spectral Methods in MATLAB, ch. 6 (cited in
    section 3.1).
    """
    x = cheb_points(p)
    c = np.ones(p)
    c[0] = c[-1] = 2.0
    D = np.zeros((p, p))
    for i in range(p):
        for j in range(p):
            if i != j:
                D[i, j] = (c[i] / c[j]) * (-1.0) ** (i + j) / (x[i] - x[j])
    for i in range(p):
        D[i, i] = -np.sum(D[i, :])
    return D


def gauss_points(q: int) -> np.ndarray:
    """q-point Gauss-Legendre nodes on [-1, 1], ascending (section 2)."""
    g, _ = np.polynomial.legendre.leggauss(q)
    return g


def lagrange_matrix(src: np.ndarray, dst: np.ndarray) -> np.ndarray:
    """Evaluate the interpolant through ``src`` at ``dst``: L[i, j] = l_j(dst_i)."""
    n = len(src)
    L = np.ones((len(dst), n))
    for j in range(n):
        for k in range(n):
            if k != j:
                L[:, j] *= (dst - src[k]) / (src[j] - src[k])
    return L


# ---------------------------------------------------------------------------
# Section 3: the leaf DtN map T = L4 L3 L2 L1.
# ---------------------------------------------------------------------------

SIDES = ("S", "E", "N", "W")


@dataclasses.dataclass
class LeafOp:
    T: np.ndarray          # [4q, 4q] DtN (section 3.2)
    X: np.ndarray          # [(p-2)^2, 4(p-1)] local solution operator -A_ii^-1 A_ie
    L1: np.ndarray         # [4(p-1), 4q]
    Je: np.ndarray         # boundary Chebyshev node indices
    Ji: np.ndarray         # interior Chebyshev node indices


def leaf_indices(p: int):
    """J_e (boundary) and J_i (interior) Chebyshev node sets (section 3.1)."""
    a = np.arange(p * p) % p
    b = np.arange(p * p) // p
    on_bd = (a == 0) | (a == p - 1) | (b == 0) | (b == p - 1)
    return np.nonzero(on_bd)[0], np.nonzero(~on_bd)[0]


def leaf_matrices(p: int, q: int, hx: float, hy: float):
    """Coefficient-independent pieces of the leaf computation for a hx-by-hy box."""
    D = cheb_diff(p)
    Dx = D * (2.0 / hx)
    Dy = D * (2.0 / hy)
    I = np.eye(p)
    # Node k = a + p*b: D1 acts along a, D2 along b.
    D1 = np.kron(I, Dx)
    D2 = np.kron(Dy, I)
    xc = cheb_points(p)
    xg = gauss_points(q)
    Je, Ji = leaf_indices(p)

    # L1: Gauss values on the four sides -> boundary Chebyshev nodes, corners
    # averaged over the two sides meeting there (section 3.2, step 1).
    G2C = lagrange_matrix(xg, xc)          # [p, q]
    L1 = np.zeros((len(Je), 4 * q))
    for r, k in enumerate(Je):
        a, b = k % p, k // p
        contrib = []
        if b == 0:
            contrib.append((0, a))       # S side, position along x
        if a == p - 1:
            contrib.append((1, b))       # E side, position along y
        if b == p - 1:
            contrib.append((2, a))       # N side
        if a == 0:
            contrib.append((3, b))       # W side
        w = 1.0 / len(contrib)
        for side, pos in contrib:
            L1[r, side * q:(side + 1) * q] += w * G2C[pos, :]

    # L3: du/dx2 at the Chebyshev nodes of S and N, du/dx1 at those of E and W
    # (section 3.2, step 3; flux convention of section 2).
    rows = []
    for a in range(p):
        rows.append(D2[a + p * 0, :])            # S
    for b in range(p):
        rows.append(D1[(p - 1) + p * b, :])      # E
    for a in range(p):
        rows.append(D2[a + p * (p - 1), :])      # N
    for b in range(p):
        rows.append(D1[0 + p * b, :])            # W
    L3 = np.array(rows)                          # [4p, p^2]

    # L4: per side, Chebyshev -> Gauss (section 3.2, step 4).
    C2G = lagrange_matrix(xc, xg)                # [q, p]
    L4 = np.zeros((4 * q, 4 * p))
    for s in range(4):
        L4[s * q:(s + 1) * q, s * p:(s + 1) * p] = C2G
    return dict(D1=D1, D2=D2, D11=D1 @ D1, D12=D1 @ D2, D22=D2 @ D2,
                Je=Je, Ji=Ji, L1=L1, L3=L3, L4=L4)


def collocation_matrix(coef: np.ndarray, mats) -> np.ndarray:
    """The p^2 x p^2 matrix A of section 3.1.

    coef has shape [6, p*p]: c11, c12, c22, c1, c2, c at the Chebyshev nodes.
    Left-multiplying by a diagonal matrix C is written as scaling the rows.
    """
    c11, c12, c22, c1, c2, c = coef
    return (-c11[:, None] * mats["D11"] - 2.0 * c12[:, None] * mats["D12"]
            - c22[:, None] * mats["D22"] + c1[:, None] * mats["D1"] + c2[:, None] * mats["D2"]
            + np.diag(c))


def leaf_dtn(coef: np.ndarray, p: int, q: int, hx: float, hy: float, mats=None) -> LeafOp:
    """Leaf DtN T = L4 L3 L2 L1 (section 3.2)."""
    m = mats if mats is not None else leaf_matrices(p, q, hx, hy)
    A = collocation_matrix(coef, m)
    Je, Ji = m["Je"], m["Ji"]
    Aii = A[np.ix_(Ji, Ji)]
    Aie = A[np.ix_(Ji, Je)]
    # Step 2: w_i = -A_ii^-1 A_ie w_e (eq:leaf_solve), LAPACK gesv.
    X = -np.linalg.solve(Aii, Aie)
    # L2 = [I; X] placed on J_e, J_i.
    L2 = np.zeros((p * p, len(Je)))
    L2[Je, :] = np.eye(len(Je))
    L2[Ji, :] = X
    T = m["L4"] @ m["L3"] @ L2 @ m["L1"]
    return LeafOp(T=T, X=X, L1=m["L1"], Je=Je, Ji=Ji)


# ---------------------------------------------------------------------------
# Section 2: tessellation, global numbering, binary tree.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Box:
    i0: int
    i1: int
    j0: int
    j1: int
    level: int
    parent: int = -1
    children: tuple = ()
    Ie: Optional[np.ndarray] = None   # exterior Gauss nodes (global ids), S,E,N,W order
    Ii: Optional[np.ndarray] = None   # interior nodes not interior to a child (J3)

    @property
    def is_leaf(self):
        return not self.children


class Grid:
    """Leaf tessellation of a rectangle with nx-by-ny leaves and q nodes per edge."""

    def __init__(self, box, nx, ny, q):
        self.box = tuple(float(v) for v in box)
        self.nx, self.ny, self.q = nx, ny, q
        self.nh = nx * (ny + 1)
        self.nv = (nx + 1) * ny
        self.N = q * (self.nh + self.nv)
        self.hx = (self.box[1] - self.box[0]) / nx
        self.hy = (self.box[3] - self.box[2]) / ny

    def hedge(self, i, j):
        return np.arange(self.q) + (j * self.nx + i) * self.q

    def vedge(self, i, j):
        return np.arange(self.q) + (self.nh + j * (self.nx + 1) + i) * self.q

    def boundary(self, i0, i1, j0, j1):
        """Exterior nodes of the box of leaves [i0,i1) x [j0,j1), ordered S, E, N, W."""
        S = [self.hedge(i, j0) for i in range(i0, i1)]
        E = [self.vedge(i1, j) for j in range(j0, j1)]
        N = [self.hedge(i, j1) for i in range(i0, i1)]
        W = [self.vedge(i0, j) for j in range(j0, j1)]
        return np.concatenate(S + E + N + W)

    def node_xy(self):
        """Coordinates of all N Gauss nodes."""
        g = gauss_points(self.q)
        x0, _, y0, _ = self.box
        xy = np.zeros((self.N, 2))
        for j in range(self.ny + 1):
            for i in range(self.nx):
                idx = self.hedge(i, j)
                xy[idx, 0] = x0 + (i + 0.5 * (g + 1.0)) * self.hx
                xy[idx, 1] = y0 + j * self.hy
        for j in range(self.ny):
            for i in range(self.nx + 1):
                idx = self.vedge(i, j)
                xy[idx, 0] = x0 + i * self.hx
                xy[idx, 1] = y0 + (j + 0.5 * (g + 1.0)) * self.hy
        return xy

    def leaf_box(self, i, j):
        x0, _, y0, _ = self.box
        return (x0 + i * self.hx, x0 + (i + 1) * self.hx, y0 + j * self.hy, y0 + (j + 1) * self.hy)

    def cheb_xy(self, p):
        """Chebyshev nodes of every leaf, [nx*ny, p*p, 2], leaf i + nx*j, node a + p*b."""
        xc = cheb_points(p)
        out = np.zeros((self.nx * self.ny, p * p, 2))
        for j in range(self.ny):
            for i in range(self.nx):
                bx = self.leaf_box(i, j)
                X = bx[0] + 0.5 * (xc + 1.0) * (bx[1] - bx[0])
                Y = bx[2] + 0.5 * (xc + 1.0) * (bx[3] - bx[2])
                xx, yy = np.meshgrid(X, Y)   # [b, a]
                out[i + self.nx * j, :, 0] = xx.ravel()
                out[i + self.nx * j, :, 1] = yy.ravel()
        return out


def build_tree(nx: int, ny: int, x_first: bool = True) -> List[Box]:
    """Binary tree over the leaves; parents precede children (section 2).

    The longer side (in leaf units) is split at floor(n/2); ties split x1 first
    unless ``x_first`` is False (used to check that the root DtN does not depend
    on the tree shape).
    """
    boxes = [Box(0, nx, 0, ny, 0)]
    k = 0
    while k < len(boxes):
        b = boxes[k]
        w, h = b.i1 - b.i0, b.j1 - b.j0
        if w > 1 or h > 1:
            vertical = (w > h) or (w == h and x_first)
            if vertical:
                m = b.i0 + w // 2
                ca = Box(b.i0, m, b.j0, b.j1, b.level + 1, parent=k)
                cb = Box(m, b.i1, b.j0, b.j1, b.level + 1, parent=k)
            else:
                m = b.j0 + h // 2
                ca = Box(b.i0, b.i1, b.j0, m, b.level + 1, parent=k)
                cb = Box(b.i0, b.i1, m, b.j1, b.level + 1, parent=k)
            b.children = (len(boxes), len(boxes) + 1)
            boxes.append(ca)
            boxes.append(cb)
        k += 1
    return boxes


# ---------------------------------------------------------------------------
# Section 4: merging two DtN maps.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class MergeOp:
    S: np.ndarray        # [m3, m1+m2] solution operator (eq:U_parent), columns in I_e^tau order
    T: np.ndarray        # [m1+m2, m1+m2] parent DtN (eq:merge)
    M: np.ndarray        # T33^alpha - T33^beta
    Q: np.ndarray        # [T13^alpha; T23^beta] in parent order, [m1+m2, m3]
    in_alpha: np.ndarray  # bool per parent boundary node: node belongs to alpha (J1) or beta (J2)
    pa: np.ndarray       # position of each parent node in its child's boundary list
    a3: np.ndarray       # positions of J3 in alpha's list
    b3: np.ndarray       # positions of J3 in beta's list


def merge(Ta, Iea, Tb, Ieb, Ie_parent) -> MergeOp:
    """Merge sibling DtNs (section 4).

    alpha is the west/south child and beta the east/north child; J3 is their
    shared edge.  With the section-2 flux convention the third block row of
    eq:premerge reads T31a u1 + T33a u3 = T32b u2 + T33b u3.
    """
    pos_a = {int(g): k for k, g in enumerate(Iea)}
    pos_b = {int(g): k for k, g in enumerate(Ieb)}
    J3 = [int(g) for g in Iea if int(g) in pos_b]
    a3 = np.array([pos_a[g] for g in J3])
    b3 = np.array([pos_b[g] for g in J3])
    in_alpha = np.array([int(g) in pos_a for g in Ie_parent])
    pa = np.array([pos_a[int(g)] if int(g) in pos_a else pos_b[int(g)] for g in Ie_parent])
    n = len(Ie_parent)
    M = Ta[np.ix_(a3, a3)] - Tb[np.ix_(b3, b3)]
    B = np.zeros((len(J3), n))
    Q = np.zeros((n, len(J3)))
    D = np.zeros((n, n))
    for c in range(n):
        if in_alpha[c]:
            B[:, c] = -Ta[a3, pa[c]]
            Q[c, :] = Ta[pa[c], a3]
        else:
            B[:, c] = Tb[b3, pa[c]]
            Q[c, :] = Tb[pa[c], b3]
    ia = np.nonzero(in_alpha)[0]
    ib = np.nonzero(~in_alpha)[0]
    D[np.ix_(ia, ia)] = Ta[np.ix_(pa[ia], pa[ia])]       # T11^alpha block
    D[np.ix_(ib, ib)] = Tb[np.ix_(pa[ib], pa[ib])]       # T22^beta block
    S = sla.solve(M, B)                      # eq:U_parent (LAPACK gesv, partial pivoting)
    T = D + Q @ S                            # eq:merge
    return MergeOp(S=S, T=T, M=M, Q=Q, in_alpha=in_alpha, pa=pa, a3=a3, b3=b3)


# ---------------------------------------------------------------------------
# Section 5: Algorithms 1 and 2.
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class Operator:
    grid: Grid
    p: int
    q: int
    boxes: List[Box]
    leafT: Dict[int, np.ndarray]        # leaf box index -> T (kept for residuals)
    leafX: Dict[int, np.ndarray]        # leaf box index -> local solution operator
    merges: Dict[int, MergeOp]          # parent box index -> merge data
    rootT: np.ndarray

    @property
    def n_bdry(self):
        return len(self.boxes[0].Ie)


def leaf_index_of(box: Box, nx: int) -> int:
    return box.i0 + nx * box.j0


def build(coeffs: np.ndarray, box, nleaf, p: int, q: int, x_first=True, keep=True,
          allow_singular=False) -> Operator:
    """Algorithm 1 (build stage).

    ``coeffs`` has shape [nx*ny, 6, p*p] (leaf i + nx*j, node a + p*b).
    Boxes are processed from the last index to the first, so every parent
    comes after its children.

    q must be below p.  Step 1 of section 3.2 maps the 4q Gauss values of a
    leaf onto its 4(p-1) boundary Chebyshev nodes, averaging the two sides at
    each corner; for q >= p that map has a null space, and at an interior
    cross point the four edges can carry a mode +a, -a, +a, -a that none of
    the four leaves sees, so the merge systems are singular.  (The leaf DtN
    itself is still well defined: ``leaf_dtn`` accepts q = p.)
    ``allow_singular`` lets the pins build such an operator on purpose.
    """
    if q >= p and not allow_singular:
        raise ValueError(f"q = {q} must be below p = {p}: with q >= p the merges are singular")
    nx, ny = nleaf
    grid = Grid(box, nx, ny, q)
    boxes = build_tree(nx, ny, x_first=x_first)
    for b in boxes:
        b.Ie = grid.boundary(b.i0, b.i1, b.j0, b.j1)
    mats = leaf_matrices(p, q, grid.hx, grid.hy)
    T: Dict[int, np.ndarray] = {}
    leafT, leafX, merges = {}, {}, {}
    for t in range(len(boxes) - 1, -1, -1):
        b = boxes[t]
        if b.is_leaf:
            lo = leaf_dtn(coeffs[leaf_index_of(b, nx)], p, q, grid.hx, grid.hy, mats)
            T[t] = lo.T
            if keep:
                leafT[t] = lo.T
                leafX[t] = lo.X
        else:
            a, c = b.children
            mo = merge(T[a], boxes[a].Ie, T[c], boxes[c].Ie, b.Ie)
            b.Ii = boxes[a].Ie[mo.a3]
            T[t] = mo.T
            merges[t] = mo
            del T[a], T[c]                    # Algorithm 1: children's T no longer needed
    return Operator(grid=grid, p=p, q=q, boxes=boxes, leafT=leafT, leafX=leafX,
                    merges=merges, rootT=T[0])


def solve(op: Operator, f: np.ndarray, z: Optional[Dict[int, np.ndarray]] = None) -> np.ndarray:
    """Algorithm 2 (solve stage); optional interface terms z^tau (refinement)."""
    f = np.atleast_2d(f)
    u = np.zeros((f.shape[0], op.grid.N))
    u[:, op.boxes[0].Ie] = f
    for t, b in enumerate(op.boxes):
        if b.is_leaf:
            continue
        mo = op.merges[t]
        u3 = u[:, b.Ie] @ mo.S.T
        if z is not None:
            u3 = u3 + z[t]
        u[:, b.Ii] = u3
    return u


def level_conditions(op: Operator) -> np.ndarray:
    """Per tree depth, the largest max|M| / min |u_kk| over its merges, where
    M = T33a - T33b and u_kk are the pivots of its LU factorization with partial
    pivoting (LAPACK getrf).  A cheap lower-side estimate of cond(M); the
    deepest depth (leaves only) gets 0."""
    depth = max(b.level for b in op.boxes)
    out = np.zeros(depth + 1)
    for t, mo in op.merges.items():
        lu, _ = sla.lu_factor(mo.M, check_finite=False)
        pmin = np.min(np.abs(np.diag(lu)))
        est = np.max(np.abs(mo.M)) / pmin if pmin > 0 else np.inf
        d = op.boxes[t].level
        out[d] = max(out[d], est)
    return out


def gamma_xy(op: Operator) -> np.ndarray:
    return op.grid.node_xy()[op.boxes[0].Ie]


# ---------------------------------------------------------------------------
# Interface residual and the upward source pass (iterative refinement).
# ---------------------------------------------------------------------------

def interface_residual(op: Operator, u: np.ndarray) -> np.ndarray:
    """Flux jump at every interior Gauss node: r = v_alpha - v_beta.

    v is evaluated with each leaf's FP64 DtN; alpha is the leaf west/south of
    the edge, beta the one east/north of it.  The global system that the
    hierarchical build solves exactly (Remark 5.1) is r = 0 with u = f on the
    boundary.  Boundary nodes get 0.
    """
    u = np.atleast_2d(u)
    r = np.zeros_like(u)
    q = op.q
    for t, T in op.leafT.items():
        b = op.boxes[t]
        v = u[:, b.Ie] @ T.T
        # S and W sides: this leaf is beta of those edges; E and N: alpha.
        sgn = np.concatenate([-np.ones(q), np.ones(q), np.ones(q), -np.ones(q)])
        r[:, b.Ie] += v * sgn
    r[:, op.boxes[0].Ie] = 0.0
    return r


def upward(op: Operator, s: np.ndarray,
           h_leaf: Optional[Dict[int, np.ndarray]] = None) -> Dict[int, np.ndarray]:
    """Upward pass for interface sources s (jump v_alpha - v_beta = s).

    Third block row of eq:premerge with a source term and with particular
    fluxes h carried up from the children:
        (T33a - T33b) u3 = -T31a u1 + T32b u2 + s3 - h3a + h3b,
    so u3 = S u_e + z with z = M^-1 (s3 - h3a + h3b), and the parent's
    particular flux is h = [h1a; h2b] + Q z.  Leaves have h = 0, or the
    fluxes h_leaf[t] [nrhs, 4q] of a body load's leaf particular solutions.
    """
    s = np.atleast_2d(s)
    nr = s.shape[0]
    h: Dict[int, np.ndarray] = {}
    z: Dict[int, np.ndarray] = {}
    for t in range(len(op.boxes) - 1, -1, -1):
        b = op.boxes[t]
        if b.is_leaf:
            h[t] = (np.zeros((nr, len(b.Ie))) if h_leaf is None
                    else np.atleast_2d(h_leaf[t]).copy())
            continue
        a, c = b.children
        mo = op.merges[t]
        rhs = s[:, b.Ii] - h[a][:, mo.a3] + h[c][:, mo.b3]
        z[t] = sla.solve(mo.M, rhs.T).T
        hp = np.zeros((nr, len(b.Ie)))
        hp[:, mo.in_alpha] = h[a][:, mo.pa[mo.in_alpha]]
        hp[:, ~mo.in_alpha] = h[c][:, mo.pa[~mo.in_alpha]]
        h[t] = hp + z[t] @ mo.Q.T
        del h[a], h[c]
    return z


def refine_step(op: Operator, u: np.ndarray) -> np.ndarray:
    """One correction: r = jump(u); solve for delta with jump(delta) = -r, delta = 0 on the boundary."""
    r = interface_residual(op, u)
    z = upward(op, -r)
    return solve(op, np.zeros((np.atleast_2d(u).shape[0], op.n_bdry)), z=z)


# ---------------------------------------------------------------------------
# Section 5.3: post-processing on a leaf's Chebyshev grid.
# ---------------------------------------------------------------------------

def leaf_cheb_values(op: Operator, u: np.ndarray, t: int) -> np.ndarray:
    """Potential on leaf t's p x p Chebyshev grid from the Gauss values on its boundary."""
    p = op.p
    b = op.boxes[t]
    mats = leaf_matrices(p, op.q, op.grid.hx, op.grid.hy)
    ue = np.atleast_2d(u)[:, b.Ie]
    we = ue @ mats["L1"].T
    w = np.zeros((ue.shape[0], p * p))
    w[:, mats["Je"]] = we
    w[:, mats["Ji"]] = we @ op.leafX[t].T
    return w


# ---------------------------------------------------------------------------
# Body loads, A u = g (an extension; the paper treats A u = 0).  In every
# leaf u = v + w: w solves the leaf's collocation equations with the load and
# zero boundary values, v the homogeneous ones.  w adds its flux h = (L4 L3) w
# to the leaf's DtN relation (flux = T v + h); the merges carry these fluxes
# up with the interface-source recursion above (s = 0), and the downward pass
# adds the resulting z.
# ---------------------------------------------------------------------------

def leaf_particular(coef: np.ndarray, g: np.ndarray, p: int, q: int, hx: float, hy: float,
                    mats=None):
    """Particular solution of one leaf: A_ii w_i = g_i, w = 0 on the leaf's
    Chebyshev boundary.  g [nrhs, p*p] at the leaf's Chebyshev nodes (only the
    interior ones are used).  Returns w_i [nrhs, (p-2)^2] and its flux
    h = L4 L3 [w on J_i, 0 on J_e], [nrhs, 4q]."""
    m = mats if mats is not None else leaf_matrices(p, q, hx, hy)
    A = collocation_matrix(coef, m)
    Ji = m["Ji"]
    g = np.atleast_2d(g)
    wi = np.linalg.solve(A[np.ix_(Ji, Ji)], g[:, Ji].T).T
    w = np.zeros((g.shape[0], p * p))
    w[:, Ji] = wi
    h = w @ (m["L4"] @ m["L3"]).T
    return wi, h


def body_solve(op: Operator, coeffs: np.ndarray, f: np.ndarray, g: np.ndarray):
    """A u = g in the domain, u = f on its boundary.  coeffs [nx*ny, 6, p*p]
    (as for build), f [nrhs, n_bdry], g [nrhs, nx*ny, p*p] at every leaf's
    Chebyshev nodes.  Returns u at the Gauss nodes [nrhs, N] and the leaf
    particular solutions {leaf box: w_i [nrhs, (p-2)^2]}."""
    g = np.asarray(g)
    if g.ndim == 2:
        g = g[None]
    nx = op.grid.nx
    mats = leaf_matrices(op.p, op.q, op.grid.hx, op.grid.hy)
    h_leaf, wpart = {}, {}
    for t, b in enumerate(op.boxes):
        if b.is_leaf:
            k = leaf_index_of(b, nx)
            wpart[t], h_leaf[t] = leaf_particular(coeffs[k], g[:, k], op.p, op.q,
                                                  op.grid.hx, op.grid.hy, mats)
    z = upward(op, np.zeros((g.shape[0], op.grid.N)), h_leaf)
    return solve(op, f, z=z), wpart


def body_cheb_values(op: Operator, u: np.ndarray, t: int, wpart) -> np.ndarray:
    """Leaf t's Chebyshev-grid values of a body-load solution: the homogeneous
    part from the leaf's Gauss values (section 5.3) plus the particular part."""
    w = leaf_cheb_values(op, u, t)
    Ji = leaf_matrices(op.p, op.q, op.grid.hx, op.grid.hy)["Ji"]
    w[:, Ji] += wpart[t]
    return w


def find_leaf(op: Operator, i: int, j: int) -> int:
    for t, b in enumerate(op.boxes):
        if b.is_leaf and b.i0 == i and b.j0 == j:
            return t
    raise KeyError((i, j))
