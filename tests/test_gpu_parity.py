"""GPU parity of the HIP path against the CPU oracle (FP64 path: 1e-10).

Every comparison is element by element on the same seeded inputs; errors are
max-abs differences relative to the max-abs entry of the oracle's result
(per matrix for operators, per right-hand side for solutions).
"""
import numpy as np
import pytest

import hps_inputs as hi
from oracle import brute, hps

from .helpers import library_inputs, oracle_problem, rel_err, say

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def H(gpu):
    import paper_1307_2665_amd as H
    return H


def _t(x, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


# ---------------------------------------------------------------------------
# Batched dense layer.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("Mr,Nc,K,nb", [(64, 64, 16, 1), (70, 130, 37, 3), (5, 3, 200, 2),
                                        (257, 65, 64, 1)])
def test_gemm_f64(H, gpu, Mr, Nc, K, nb):
    say(f"gemm_f64 {Mr}x{Nc}x{K} batch {nb}")
    rng = np.random.default_rng(Mr * 7 + Nc)
    A, B, C0 = rng.standard_normal((nb, Mr, K)), rng.standard_normal((nb, K, Nc)), rng.standard_normal((nb, Mr, Nc))
    C = _t(C0, gpu)
    H.batched_gemm(_t(A, gpu), _t(B, gpu), C, alpha=-0.5)
    ref = C0 - 0.5 * A @ B
    assert rel_err(C.cpu().numpy(), ref) < 1e-14


def test_gemm_split32_accuracy(H, gpu):
    say("gemm_split32 300x200x448")
    rng = np.random.default_rng(5)
    A, B = rng.standard_normal((1, 300, 448)), rng.standard_normal((1, 448, 200))
    C = _t(np.zeros((1, 300, 200)), gpu)
    H.batched_gemm(_t(A, gpu), _t(B, gpu), C, split32=True)
    ref = A @ B
    err = rel_err(C.cpu().numpy(), ref)
    # hi/lo splitting removes the input rounding; the FP32 accumulation of each
    # 16-deep slab leaves an error of a few units of 2^-24 (~6e-8).
    assert err < 5e-7


def test_gemm_bf16x6_accuracy(H, gpu):
    """BF16 MFMA on three-slice splits: the operand slices carry 24 bits, the six
    products are exact in FP32 and summed in FP32 over 32-deep slabs, so the
    error is a few units of 2^-24 like the split-FP32 form.  Ragged tiles in all
    three dimensions; a transposed fragment or a dropped slice product fails."""
    say("gemm_bf16x6 300x200x448 and 70x130x37 batch 3")
    rng = np.random.default_rng(6)
    for (Mr, Nc, K, nb) in [(300, 200, 448, 1), (70, 130, 37, 3)]:
        A, B = rng.standard_normal((nb, Mr, K)), rng.standard_normal((nb, K, Nc))
        C0 = rng.standard_normal((nb, Mr, Nc))
        C = _t(C0, gpu)
        H.batched_gemm(_t(A, gpu), _t(B, gpu), C, alpha=-0.5, bf16x6=True)
        ref = C0 - 0.5 * A @ B
        err = rel_err(C.cpu().numpy(), ref)
        say(f"  {Mr}x{Nc}x{K}: rel err {err:.2e}")
        assert err < 5e-7
    # scale spread: values over 2^-40 .. 2^40 keep their relative accuracy
    A = rng.standard_normal((1, 64, 64)) * np.exp2(rng.integers(-40, 40, (1, 64, 1)))
    B = rng.standard_normal((1, 64, 64))
    C = _t(np.zeros((1, 64, 64)), gpu)
    H.batched_gemm(_t(A, gpu), _t(B, gpu), C, bf16x6=True)
    ref = A @ B
    rowerr = np.max(np.abs(C.cpu().numpy() - ref), axis=2) / np.max(np.abs(ref), axis=2)
    assert rowerr.max() < 5e-7


# Sizes cover the one-wave panel (n <= 128: 5, 33, 70), the multi-wave
# 32-wide panel (130 .. 900, two to eight waves) and the 16-wide panel with six
# rows per lane (1100, 2100).
@pytest.mark.parametrize("n,m,nb", [(5, 3, 2), (33, 40, 3), (70, 17, 2), (130, 9, 1), (196, 56, 2),
                                    (448, 30, 2), (900, 40, 1), (1100, 20, 1), (2100, 7, 1)])
def test_batched_solve_with_pivoting(H, gpu, n, m, nb):
    say(f"batched_solve n={n} m={m} batch {nb}")
    rng = np.random.default_rng(n + m)
    M = rng.standard_normal((nb, n, n))
    M[:, np.arange(n), np.arange(n)] = 0.0          # forces row interchanges
    B = rng.standard_normal((nb, n, m))
    X = H.batched_solve(_t(M, gpu), _t(B, gpu)).cpu().numpy()
    ref = np.linalg.solve(M, B)
    assert rel_err(X, ref) < 1e-10


def test_batched_solve_deep_pivots(H, gpu):
    """The top 300 x 300 block has rank one and the top rows are tiny, so every
    pivot of the first panels must come from rows far below (other chunks of
    the tournament)."""
    say("batched_solve deep pivots n=600")
    rng = np.random.default_rng(77)
    n, m = 600, 12
    M = rng.standard_normal((1, n, n))
    M[0, :300, :300] = 1e-8 * np.outer(rng.standard_normal(300), rng.standard_normal(300))
    B = rng.standard_normal((1, n, m))
    X = H.batched_solve(_t(M, gpu), _t(B, gpu)).cpu().numpy()
    ref = np.linalg.solve(M, B)
    assert rel_err(X, ref) < 1e-9


def test_batched_solve_reports_singular(H, gpu):
    say("batched_solve singular")
    M = np.zeros((2, 8, 8))
    M[0] = np.eye(8)
    B = np.ones((2, 8, 3))
    with pytest.raises(H.HpsError) as e:
        H.batched_solve(_t(M, gpu), _t(B, gpu))
    assert e.value.status == H.HPS_ESINGULAR


@pytest.mark.parametrize("n", [70, 300, 1100])
def test_batched_solve_singular_last_pivot(H, gpu, n):
    """A zero last pivot (the identity with its last diagonal entry zeroed) is
    reported by every panel form: one-wave, multi-wave and 16-wide."""
    say(f"batched_solve singular last pivot n={n}")
    M = np.eye(n)[None].repeat(2, axis=0)
    M[1, n - 1, n - 1] = 0.0
    B = np.ones((2, n, 2))
    with pytest.raises(H.HpsError) as e:
        H.batched_solve(_t(M, gpu), _t(B, gpu))
    assert e.value.status == H.HPS_ESINGULAR


# ---------------------------------------------------------------------------
# Leaf stage (section 3).
# ---------------------------------------------------------------------------

# p <= 12 (and q below p) take the MFMA leaf kernel; p = 16 the register
# Gauss-Jordan kernel; p = 20 and 21 the unfused path.
@pytest.mark.parametrize("p,q", [(16, 14), (12, 10), (20, 18), (21, 20), (6, 4), (7, 5), (8, 6),
                                 (9, 7), (10, 8), (11, 9), (12, 11), (12, 6)])
def test_leaf_dtn_parity(H, gpu, p, q):
    say(f"leaf_dtn p={p} q={q}")
    rng = np.random.default_rng(p * 31 + q)
    nl = 7
    hx, hy = 1.0 / 64, 1.0 / 32
    C = np.zeros((nl, 6, p * p))
    C[:, 0] = 1.0 + 0.4 * rng.random((nl, p * p))
    C[:, 1] = 0.2 * rng.standard_normal((nl, p * p))
    C[:, 2] = 1.0 + 0.4 * rng.random((nl, p * p))
    C[:, 3] = 10.0 * rng.standard_normal((nl, p * p))
    C[:, 4] = 10.0 * rng.standard_normal((nl, p * p))
    C[:, 5] = -40.0 * rng.random((nl, p * p))
    T = H.leaf_dtn(_t(C, gpu), hx, hy, p, q).cpu().numpy()
    mats = hps.leaf_matrices(p, q, hx, hy)
    worst = 0.0
    for i in range(nl):
        ref = hps.leaf_dtn(C[i], p, q, hx, hy, mats).T
        worst = max(worst, rel_err(T[i], ref))
        assert rel_err(T[i], ref) < TOL, (i, rel_err(T[i], ref))
    say(f"  worst rel err {worst:.2e}")


@pytest.mark.parametrize("p,q", [(12, 10), (8, 6)])
def test_leaf_mfma_matches_register_kernel(H, gpu, p, q):
    """The MFMA leaf kernel against the register Gauss-Jordan kernel and the
    separate T product (leaf_mfma off), on 300 leaves (several waves of
    workgroups), a Helmholtz-like zeroth-order term and large convection."""
    rng = np.random.default_rng(5 * p + q)
    nl = 300
    C = np.zeros((nl, 6, p * p))
    C[:, 0] = 1.0 + 0.4 * rng.random((nl, p * p))
    C[:, 2] = 1.0 + 0.4 * rng.random((nl, p * p))
    C[:, 3] = 30.0 * rng.standard_normal((nl, p * p))
    C[:, 4] = 30.0 * rng.standard_normal((nl, p * p))
    C[:, 5] = -2000.0 * rng.random((nl, p * p))
    Cd = _t(C, gpu)
    T_m = H.leaf_dtn(Cd, 1.0 / 16, 1.0 / 16, p, q).cpu().numpy()
    H.tune_set("leaf_mfma", 0)
    try:
        T_r = H.leaf_dtn(Cd, 1.0 / 16, 1.0 / 16, p, q).cpu().numpy()
    finally:
        H.tune_set("leaf_mfma", -1)
    errs = [rel_err(T_m[i], T_r[i]) for i in range(nl)]
    say(f"  MFMA vs register kernel: worst rel diff {max(errs):.2e}")
    assert max(errs) < TOL
    mats = hps.leaf_matrices(p, q, 1.0 / 16, 1.0 / 16)
    for i in (0, 137, nl - 1):
        assert rel_err(T_m[i], hps.leaf_dtn(C[i], p, q, 1.0 / 16, 1.0 / 16, mats).T) < TOL


# ---------------------------------------------------------------------------
# Build and solve (Algorithms 1, 2).
# ---------------------------------------------------------------------------

def _compare_operator(H, op_g, op_o, check_S=True):
    if check_S:
        for t, mo in op_o.merges.items():
            S = op_g.export_S(t)
            assert S.shape == mo.S.shape
            e = rel_err(S, mo.S)
            assert e < TOL, (t, e)
    e = rel_err(op_g.export_root_dtn(), op_o.rootT)
    assert e < TOL, ("root T", e)


def test_config1_laplace(H, gpu):
    """4x4 leaves, p=16, q=14, u = log|x - (1.5, 1.5)|."""
    say("config1 build")
    pr = hi.laplace_log()
    op_o, C_o, f_o, grid = oracle_problem(pr)
    C, f = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
    _compare_operator(H, op, op_o)
    for lf in range(16):
        t = hps.find_leaf(op_o, lf % 4, lf // 4)
        assert rel_err(op.export_leaf_dtn(lf), op_o.leafT[t]) < TOL
    say("config1 solve")
    u = op.solve(_t(f, gpu)).cpu().numpy()
    u_o = hps.solve(op_o, f_o)
    assert rel_err(u, u_o) < TOL
    ex = pr.exact(*grid.node_xy().T)
    assert np.max(np.abs(u[0] - ex)) < 1e-11
    # host-pointer path gives the same numbers
    u2 = op.solve(f)
    assert np.max(np.abs(u2 - u)) == 0.0


@pytest.mark.parametrize("nleaf", [(3, 5), (7, 2), (1, 1), (2, 1)])
def test_rectangles_and_uneven_trees(H, gpu, nleaf):
    say(f"manufactured build nleaf={nleaf}")
    pr = hi.manufactured_variable(nleaf=nleaf, p=10, q=8)
    pr.box = (0.0, 1.5, -0.5, 0.5)
    op_o, C_o, f_o, grid = oracle_problem(pr)
    C, f = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, nleaf, pr.p, pr.q)
    _compare_operator(H, op, op_o)
    u = op.solve(_t(f, gpu)).cpu().numpy()
    assert rel_err(u, hps.solve(op_o, f_o)) < TOL
    assert np.max(np.abs(u[0] - pr.exact(*grid.node_xy().T))) < 1e-10


def test_convdiff_16x16_multi_rhs(H, gpu):
    say("convdiff 16x16 p16 q14, 3 rhs")
    pr = hi.convdiff(nleaf=(16, 16), p=16, q=14, nrhs=3)
    op_o, C_o, f_o, grid = oracle_problem(pr)
    C, f = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
    _compare_operator(H, op, op_o)
    u = op.solve(_t(f, gpu)).cpu().numpy()
    u_o = hps.solve(op_o, f_o)
    for k in range(3):
        assert rel_err(u[k], u_o[k]) < TOL
    v = op.root_dtn_apply(_t(f, gpu)).cpu().numpy()
    assert rel_err(v, f_o @ op_o.rootT.T) < TOL


def test_helmholtz_bump_small(H, gpu):
    say("helmholtz bump 16x16")
    pr = hi.helmholtz_bump(nleaf=(16, 16), nrhs=2)
    op_o, C_o, f_o, grid = oracle_problem(pr)
    C, f = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
    _compare_operator(H, op, op_o, check_S=False)
    u = op.solve(_t(f, gpu)).cpu().numpy()
    u_o = hps.solve(op_o, f_o)
    for k in range(2):
        assert rel_err(u[k], u_o[k]) < TOL


def test_interface_residual_and_sources(H, gpu):
    say("residual + sources 5x4")
    pr = hi.convdiff(nleaf=(5, 4), p=10, q=8)
    op_o, C_o, f_o, grid = oracle_problem(pr)
    C, f = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q, keep_factors=True)
    rng = np.random.default_rng(1)
    u = rng.standard_normal((2, op.N))
    r = op.interface_residual(_t(u, gpu)).cpu().numpy()
    r_o = hps.interface_residual(op_o, u)
    assert rel_err(r, r_o) < TOL
    s = rng.standard_normal((2, op.N))
    s[:, op_o.boxes[0].Ie] = 0.0
    ug = op.solve_with_sources(_t(f_o[:1].repeat(2, 0), gpu), _t(s, gpu)).cpu().numpy()
    z = hps.upward(op_o, s)
    uo = hps.solve(op_o, f_o[:1].repeat(2, 0), z=z)
    assert rel_err(ug, uo) < TOL


def test_invalid_inputs(H, gpu):
    say("invalid inputs")
    p, q = 8, 6
    C = np.zeros((4, 6, p * p))
    C[:, 0] = C[:, 2] = 1.0
    C[2, 5, 10] = np.nan
    with pytest.raises(H.HpsError) as e:
        H.build_solution_operator(_t(C, gpu), (0, 1, 0, 1), (2, 2), p, q)
    assert e.value.status == H.HPS_EINVAL
    with pytest.raises(H.HpsError) as e:
        H.build_solution_operator(_t(np.zeros((4, 6, p * p)), gpu), (0, 1, 0, 1), (2, 2), p, q)
    assert e.value.status == H.HPS_ESINGULAR
    with pytest.raises(H.HpsError) as e:
        H.build_solution_operator(_t(C, gpu), (0, 1, 0, 1), (2, 2), p, p + 1)
    assert e.value.status == H.HPS_EINVAL


def test_config2_full_size_sampled(H, gpu):
    """64x64, p=16, q=14 (the benchmark workload): sampled leaf DtNs against the
    oracle, and the oracle's flux-matching equations at every edge of sampled
    leaves evaluated on the GPU solution."""
    say("config2 full size build")
    pr = hi.convdiff()
    C, f = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
    u = op.solve(_t(f, gpu)).cpu().numpy()[0]
    grid = hps.Grid(pr.box, 64, 64, pr.q)
    Co = pr.coeffs_at(grid.cheb_xy(pr.p))
    mats = hps.leaf_matrices(pr.p, pr.q, grid.hx, grid.hy)
    rng = np.random.default_rng(2)
    sample = rng.choice(64 * 64, size=24, replace=False)
    say("config2 sampled leaves")
    Tcache = {}

    def leafT(i, j):
        k = i + 64 * j
        if k not in Tcache:
            Tcache[k] = hps.leaf_dtn(Co[k], pr.p, pr.q, grid.hx, grid.hy, mats).T
        return Tcache[k]

    q = pr.q
    for k in sample:
        i, j = int(k % 64), int(k // 64)
        Tg = op.export_leaf_dtn(int(k))
        assert rel_err(Tg, leafT(i, j)) < TOL
        # flux matching across this leaf's east and north edges (oracle T's, GPU u)
        vk = leafT(i, j) @ u[grid.boundary(i, i + 1, j, j + 1)]
        scale = np.max(np.abs(leafT(i, j))) * np.max(np.abs(u))
        if i + 1 < 64:
            ve = leafT(i + 1, j) @ u[grid.boundary(i + 1, i + 2, j, j + 1)]
            assert np.max(np.abs(vk[q:2 * q] - ve[3 * q:])) < 1e-10 * scale
        if j + 1 < 64:
            vn = leafT(i, j + 1) @ u[grid.boundary(i, i + 1, j + 1, j + 2)]
            assert np.max(np.abs(vk[2 * q:3 * q] - vn[:q])) < 1e-10 * scale
    # boundary data is reproduced exactly
    ids = H.boundary_ids((64, 64), q)
    assert np.max(np.abs(u[ids] - f[0])) == 0.0


def test_gj_lookahead_matches_serial_steps(H, gpu):
    """The merge solver's look-ahead (next panel's columns first, the rest on a
    side stream) computes the same tiles as the serial step order: identical
    bits for a batched solve of several panels and for a whole operator."""
    say("gj look-ahead vs serial steps")
    rng = np.random.default_rng(12)
    M, B = rng.standard_normal((3, 900, 900)), rng.standard_normal((3, 900, 70))
    out = {}
    pr = hi.convdiff(nleaf=(16, 16))
    C, f = library_inputs(pr)
    try:
        for la in (1, 0):
            H.tune_set("gj_lookahead", la)
            X = H.batched_solve(_t(M, gpu), _t(B, gpu)).cpu().numpy()
            op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
            out[la] = (X, op.export_root_dtn(), op.solve(_t(f, gpu)).cpu().numpy())
    finally:
        H.tune_set("gj_lookahead", 0)
    assert rel_err(out[1][0], np.linalg.solve(M, B)) < 1e-10
    for a, b in zip(out[1], out[0]):
        assert np.array_equal(a, b)


# ---------------------------------------------------------------------------
# Merge systems by blocked Gauss-Jordan (pivoting inside 64 x 64 diagonal
# blocks) and its fall-back to partial pivoting.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("maker,nleaf", [
    (lambda: hi.convdiff(nleaf=(16, 16), p=12, q=10), (16, 16)),
    (lambda: hi.helmholtz_bump(kappa=25.0, nleaf=(8, 16), p=12, q=10, nrhs=3), (8, 16)),
    (lambda: hi.manufactured_variable(nleaf=(12, 10), p=10, q=8), (12, 10)),
])
def test_blocked_gauss_jordan_merges_match_oracle(H, gpu, maker, nleaf):
    """Every merge level on the blocked path (bgj_min_rows = 1): every merge's S, the root DtN
    and u against the oracle at 1e-10 (ragged last blocks: m3 is not a multiple of 64)."""
    pr = maker()
    op_o, Co, fo, grid = oracle_problem(pr)
    C, f = library_inputs(pr)
    before = H.bgj_fallbacks()
    H.tune_set("bgj_min_rows", 1)
    H.tune_set("merge_small", 0)
    try:
        op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
    finally:
        H.tune_set("bgj_min_rows", -1)
        H.tune_set("merge_small", -1)
    assert H.bgj_fallbacks() == before
    _compare_operator(H, op, op_o)
    u = op.solve(_t(f, gpu)).cpu().numpy()
    e = rel_err(u, hps.solve(op_o, fo))
    say(f"  blocked Gauss-Jordan {pr.name} {nleaf}: u rel err {e:.2e}")
    assert e < TOL


def test_blocked_gauss_jordan_fallback(H, gpu):
    """A fall-back threshold of max|M| sends every blocked level back to partial pivoting: the
    counter moves and the operator still matches the oracle."""
    pr = hi.convdiff(nleaf=(8, 8), p=12, q=10)
    op_o, Co, fo, grid = oracle_problem(pr)
    C, f = library_inputs(pr)
    before = H.bgj_fallbacks()
    H.tune_set("bgj_min_rows", 1)
    H.tune_set("bgj_fallback_tol_exp", 0)
    H.tune_set("merge_small", 0)
    try:
        op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
    finally:
        H.tune_set("bgj_min_rows", -1)
        H.tune_set("bgj_fallback_tol_exp", -1)
        H.tune_set("merge_small", -1)
    fell = H.bgj_fallbacks() - before
    say(f"  fallbacks: {fell}")
    assert fell == len([d for d in range(20) if any(b.level == d and not b.is_leaf
                                                     for b in op_o.boxes)])
    _compare_operator(H, op, op_o)


# ---------------------------------------------------------------------------
# Parked operators: a destroyed operator's buffers and descriptors serve the
# next build of the same shape.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kw,host", [({}, False), ({"keep_factors": True}, False), ({}, True)])
def test_parked_operator_rebuild_matches_fresh(H, gpu, kw, host):
    """A build that takes back a parked operator (other coefficients before) gives bit for bit
    what a fresh build gives, and matches the oracle; hps_mem_trim frees the parked ones."""
    import torch
    first = hi.convdiff(seed_g=41, seed_h=42, nleaf=(8, 8), p=12, q=10)
    pr = hi.convdiff(seed_g=43, seed_h=44, nleaf=(8, 8), p=12, q=10)
    C1, _ = library_inputs(first)
    C, f = library_inputs(pr)
    arg = (lambda c: np.ascontiguousarray(c)) if host else (lambda c: _t(c, gpu))
    H.tune_set("parked_ops", 0)
    try:
        op = H.build_solution_operator(arg(C), pr.box, pr.nleaf, pr.p, pr.q, **kw)
        u_fresh = op.solve(_t(f, gpu)).cpu().numpy()
        op.destroy()
        H.tune_set("parked_ops", 2)
        op1 = H.build_solution_operator(arg(C1), first.box, first.nleaf, first.p, first.q, **kw)
        op1.solve(_t(f, gpu))
        op1.destroy()
        torch.cuda.synchronize()
        in_use_parked = H.mem_stats()["in_use"]
        op = H.build_solution_operator(arg(C), pr.box, pr.nleaf, pr.p, pr.q, **kw)
        u = op.solve(_t(f, gpu)).cpu().numpy()
        if kw.get("keep_factors"):
            ur = op.solve(_t(f, gpu), refine=True, tol=1e-12, max_iter=3).cpu().numpy()
            assert rel_err(ur, u_fresh) < 1e-12
        op.destroy()
    finally:
        H.tune_set("parked_ops", -1)
    assert np.array_equal(u, u_fresh)
    op_o, Co, fo, grid = oracle_problem(pr)
    e = rel_err(u, hps.solve(op_o, fo))
    say(f"  parked rebuild {kw} host={host}: u rel err {e:.2e}")
    assert e < TOL
    H.mem_trim()
    assert H.mem_stats()["in_use"] < in_use_parked


def test_blocked_gauss_jordan_lookahead_matches_serial(H, gpu):
    """The look-ahead (next block's columns first, the rest on a second stream beside the
    next diagonal-block kernel) gives bit for bit the one-launch-per-step result."""
    pr = hi.helmholtz_bump(kappa=25.0, nleaf=(16, 16), p=12, q=10, nrhs=2)
    C, f = library_inputs(pr)
    us = []
    H.tune_set("bgj_min_rows", 1)
    H.tune_set("merge_small", 0)
    try:
        for look in (0, 1):
            H.tune_set("bgj_lookahead", look)
            op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
            us.append(op.solve(_t(f, gpu)).cpu().numpy())
            T = op.export_root_dtn()
            us.append(T)
            op.destroy()
    finally:
        H.tune_set("bgj_min_rows", -1)
        H.tune_set("bgj_lookahead", -1)
        H.tune_set("merge_small", -1)
    assert np.array_equal(us[0], us[2]) and np.array_equal(us[1], us[3])


# ---------------------------------------------------------------------------
# Small merges in one launch per level (interfaces of at most 64 nodes).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("maker", [
    lambda: hi.convdiff(nleaf=(16, 16), p=12, q=10),
    lambda: hi.helmholtz_bump(kappa=25.0, nleaf=(8, 16), p=16, q=14, nrhs=2),
    lambda: hi.manufactured_variable(nleaf=(7, 5), p=10, q=7),
])
def test_small_merges_match_oracle_and_level_path(H, gpu, maker):
    """The one-launch small-merge path against the oracle (every merge's S, the root DtN, u) and
    against the level-wise path (gather, elimination, two GEMMs); uneven trees and odd q."""
    pr = maker()
    op_o, Co, fo, grid = oracle_problem(pr)
    C, f = library_inputs(pr)
    us = []
    try:
        for on in (0, 1):
            H.tune_set("merge_small", on)
            op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
            if on:
                _compare_operator(H, op, op_o)
            us.append(op.solve(_t(f, gpu)).cpu().numpy())
            op.destroy()
    finally:
        H.tune_set("merge_small", -1)
    e = rel_err(us[1], hps.solve(op_o, fo))
    say(f"  small merges {pr.name}: u rel err {e:.2e}, against level path {rel_err(us[1], us[0]):.1e}")
    assert e < TOL
    assert rel_err(us[1], us[0]) < 1e-12


def test_small_merges_keep_factors_refinement(H, gpu):
    """With the factors kept (M^-1 and Q written by the small-merge kernel), the refined solve
    of a mixed-precision operator matches the oracle."""
    pr = hi.convdiff(nleaf=(16, 16), p=12, q=10)
    op_o, Co, fo, grid = oracle_problem(pr)
    C, f = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q,
                                   mode=H.HPS_MIXED_BF16X6)
    u = op.solve(_t(f, gpu), refine=True, tol=1e-12, max_iter=10).cpu().numpy()
    e = rel_err(u, hps.solve(op_o, fo))
    say(f"  small merges, kept factors, refined: u rel err {e:.2e}")
    assert e < TOL


# ---------------------------------------------------------------------------
# Algorithm 2 as one cooperative launch (grid-wide barrier between levels).
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("maker", [
    lambda: hi.convdiff(nleaf=(16, 16), p=12, q=10, nrhs=3),
    lambda: hi.helmholtz_bump(kappa=25.0, nleaf=(32, 32), p=10, q=8, nrhs=2),
    lambda: hi.manufactured_variable(nleaf=(7, 5), p=10, q=7),
])
def test_persistent_solve_matches_level_passes(H, gpu, maker):
    """The persistent downward pass gives bit for bit the level-by-level passes (eager and
    graph replay) for 1 to 15 right-hand sides, and u matches the oracle; an operator whose
    depths hold merges of different shapes keeps the level passes."""
    pr = maker()
    op_o, Co, fo, grid = oracle_problem(pr)
    C, f = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
    rng = np.random.default_rng(3)
    try:
        for nrhs in (1, 4, 15):
            fr = _t(rng.standard_normal((nrhs, op.n_bdry)), gpu)
            H.tune_set("solve_persist", 0)
            ref = [op.solve(fr).cpu().numpy() for _ in range(3)]   # eager, then graph replays
            H.tune_set("solve_persist", 1)
            for _ in range(2):
                up = op.solve(fr).cpu().numpy()
                assert all(np.array_equal(up, r) for r in ref), nrhs
    finally:
        H.tune_set("solve_persist", -1)
    u = op.solve(_t(f, gpu)).cpu().numpy()
    e = rel_err(u, hps.solve(op_o, fo))
    say(f"  persistent solve {pr.name} {pr.nleaf}: u rel err {e:.2e}")
    assert e < TOL


# ---------------------------------------------------------------------------
# The section 9.2 problems (strong constant and variable convection, a
# high-frequency Helmholtz coefficient) at small sizes: large coefficients
# stress the pivoting of the leaf and merge eliminations.
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("maker", [
    lambda: hi.paper_constant_convection(nleaf=(8, 8), p=12, q=10),
    lambda: hi.paper_diffusion_convection(nleaf=(8, 8), p=14, q=12),
    # kappa = 30 keeps the merges well conditioned (oracle max|M|/min|pivot| about 8; at
    # kappa = 80 one depth reaches 1e3 and S differs from the oracle by 1.3e-10).
    lambda: hi.paper_variable_helmholtz(nleaf=(16, 16), p=12, q=10, kappa=30.0),
])
def test_section9_problems_match_oracle(H, gpu, maker):
    pr = maker()
    op_o, Co, fo, grid = oracle_problem(pr)
    C, f = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
    _compare_operator(H, op, op_o)
    u = op.solve(_t(f, gpu)).cpu().numpy()
    e = rel_err(u, hps.solve(op_o, fo))
    say(f"  {pr.name} {pr.nleaf} p={pr.p}: u rel err {e:.2e}")
    assert e < TOL


@pytest.mark.parametrize("p,q,nleaf", [(16, 14, (6, 5)), (20, 18, (4, 4)), (14, 12, (5, 3))])
def test_leaf_blocked_gauss_jordan_matches_oracle(H, gpu, p, q, nleaf):
    """Leaf systems eliminated by blocked Gauss-Jordan (knob leaf_bgj): every leaf DtN, the
    root DtN and u against the oracle; with the fall-back threshold at max|A_ii| every chunk
    is redone with partial pivoting and still matches."""
    pr = hi.helmholtz_bump(kappa=20.0, nleaf=nleaf, p=p, q=q, nrhs=2)
    op_o, Co, fo, grid = oracle_problem(pr)
    C, f = library_inputs(pr)
    for forced in (0, 1):
        before = H.bgj_fallbacks()
        H.tune_set("leaf_bgj", 1)
        if forced:
            H.tune_set("bgj_fallback_tol_exp", 0)
        try:
            op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
        finally:
            H.tune_set("leaf_bgj", -1)
            H.tune_set("bgj_fallback_tol_exp", -1)
        fell = H.bgj_fallbacks() - before
        assert (fell > 0) == bool(forced), fell
        for lf in range(nleaf[0] * nleaf[1]):
            t = hps.find_leaf(op_o, lf % nleaf[0], lf // nleaf[0])
            assert rel_err(op.export_leaf_dtn(lf), op_o.leafT[t]) < TOL, lf
        _compare_operator(H, op, op_o)
        u = op.solve(_t(f, gpu)).cpu().numpy()
        e = rel_err(u, hps.solve(op_o, fo))
        say(f"  leaf blocked GJ p={p} forced fall-back {forced}: u rel err {e:.2e}")
        assert e < TOL
        op.destroy()
