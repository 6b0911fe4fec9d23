"""Kernel variants and the autotuner.

Every variant the autotuner may pick is checked against plain definitions
(numpy products and solves) or the oracle's leaf DtN, so a tuned build is held
to the same bar as the default one; then the autotuner runs on small shapes,
its cache is saved, and a build using the tuned table matches the oracle.
"""
import json

import numpy as np
import pytest

import hps_inputs as hi
from oracle import hps

from .helpers import library_inputs, oracle_problem, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H(gpu):
    import paper_1307_2665_amd as H
    yield H
    H.tune_set("gemm_variant", -1)
    H.tune_set("gj_variant", -1)
    H.tune_set("leaf_variant", -1)
    H.tune_reset()


def _t(x, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


# Shapes: odd leading dimensions (single-double loads of the 128 x 128 tile),
# even ones with ragged K and N (pair loads with a single tail), and grids of
# 8 x 8 and 9 x 16 tiles (the XCD-grouped tile order, with a partial group).
GEMM_SHAPES = [(70, 130, 37, 3), (257, 65, 64, 1), (5, 3, 200, 2), (130, 300, 33, 1),
               (300, 260, 96, 2), (140, 258, 50, 1), (1024, 1024, 48, 1), (1152, 2048, 32, 1)]


@pytest.mark.parametrize("variant", range(8))
def test_gemm_variants(H, gpu, variant):
    say(f"gemm variant {variant}")
    H.tune_set("gemm_variant", variant)
    try:
        for Mr, Nc, K, nb in GEMM_SHAPES:
            rng = np.random.default_rng(Mr + 3 * Nc + K)
            A, B = rng.standard_normal((nb, Mr, K)), rng.standard_normal((nb, K, Nc))
            C0 = rng.standard_normal((nb, Mr, Nc))
            C = _t(C0, gpu)
            H.batched_gemm(_t(A, gpu), _t(B, gpu), C, alpha=-0.5)
            assert rel_err(C.cpu().numpy(), C0 - 0.5 * A @ B) < 1e-14, (Mr, Nc, K)
    finally:
        H.tune_set("gemm_variant", -1)


# update tile * 4 + TRSM block: every tile once, every block size once
@pytest.mark.parametrize("variant", [0, 1, 2, 4, 8, 13, 16, 22])
def test_merge_solver_variants(H, gpu, variant):
    say(f"gj variant {variant}")
    H.tune_set("gj_variant", variant)
    try:
        for n, m, nb in [(70, 17, 2), (448, 30, 1), (130, 9, 3)]:
            rng = np.random.default_rng(n + m + variant)
            M = rng.standard_normal((nb, n, n))
            M[:, np.arange(n), np.arange(n)] = 0.0
            B = rng.standard_normal((nb, n, m))
            X = H.batched_solve(_t(M, gpu), _t(B, gpu)).cpu().numpy()
            assert rel_err(X, np.linalg.solve(M, B)) < 1e-10, (n, m)
    finally:
        H.tune_set("gj_variant", -1)


@pytest.mark.parametrize("variant", range(5))
@pytest.mark.parametrize("p,q", [(16, 14), (12, 10)])
def test_leaf_variants(H, gpu, variant, p, q):
    say(f"leaf variant {variant} p={p}")
    rng = np.random.default_rng(variant + p)
    nl, hx, hy = 5, 1.0 / 64, 1.0 / 64
    C = np.zeros((nl, 6, p * p))
    C[:, 0] = 1.0 + 0.4 * rng.random((nl, p * p))
    C[:, 2] = 1.0 + 0.4 * rng.random((nl, p * p))
    C[:, 3] = 10.0 * rng.standard_normal((nl, p * p))
    C[:, 5] = -40.0 * rng.random((nl, p * p))
    H.tune_set("leaf_variant", variant)
    try:
        T = H.leaf_dtn(_t(C, gpu), hx, hy, p, q).cpu().numpy()
    finally:
        H.tune_set("leaf_variant", -1)
    mats = hps.leaf_matrices(p, q, hx, hy)
    for i in range(nl):
        assert rel_err(T[i], hps.leaf_dtn(C[i], p, q, hx, hy, mats).T) < 1e-10


def test_autotune_then_build_matches_oracle(H, gpu, tmp_path):
    H.tune_reset()
    shapes = [dict(nleaf=(8, 8), p=16, q=14), dict(nleaf=(4, 6), p=12, q=10)]
    sec = H.autotune(shapes)
    path = tmp_path / "tune.json"
    H.tune_save(path)
    entries = json.loads(path.read_text())["entries"]
    names = {e["name"] for e in entries}
    say(f"autotune {sec:.2f} s, {len(entries)} buckets: " +
        ", ".join(f"{e['name']}{e['key']}->{e['variant']} ({e['default_ms']:.3f}->{e['ms']:.3f} ms)"
                  for e in entries))
    assert names == {"leaf", "gemm", "gj"} and sec > 0
    assert all(e["ms"] <= e["default_ms"] * 1.0001 for e in entries)
    # GEMM buckets list every tile's time, the chosen one the fastest.
    for e in (e for e in entries if e["name"] == "gemm"):
        assert len(e["all_ms"]) == 8 and e["ms"] == pytest.approx(min(e["all_ms"]), rel=1e-5)
    # A second run finds every bucket already tuned.
    assert H.autotune(shapes) < sec
    # Reloading the cache restores the same table.
    H.tune_reset()
    H.tune_load(path)
    H.tune_save(tmp_path / "again.json")
    assert json.loads((tmp_path / "again.json").read_text())["entries"] == entries
    pr = hi.convdiff(seed_g=21, seed_h=22, nleaf=(8, 8), p=16, q=14)
    C, f = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
    u = op.solve(_t(f, gpu)).cpu().numpy()
    op_o, C_o, f_o, grid = oracle_problem(pr)
    u_o = hps.solve(op_o, f_o)
    e = max(rel_err(u[k], u_o[k]) for k in range(u_o.shape[0]))
    say(f"tuned build vs oracle: u {e:.2e}")
    assert e < 1e-10
    H.tune_reset()


@pytest.mark.parametrize("variant", [0, 7])
@pytest.mark.parametrize("nleaf,p,q", [((8, 8), 12, 10), ((5, 3), 10, 7)])
def test_build_with_gemm_variant_matches_oracle(H, gpu, variant, nleaf, p, q):
    """Every merge's Schur product T = diag(T11a, T22b) + Q S on one forced
    tile; q = 7 on 5 x 3 leaves gives odd interface lengths (single-double
    operand loads)."""
    pr = hi.convdiff(seed_g=31, seed_h=32, nleaf=nleaf, p=p, q=q)
    C, f = library_inputs(pr)
    H.tune_set("gemm_variant", variant)
    try:
        op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
        u = op.solve(_t(f, gpu)).cpu().numpy()
    finally:
        H.tune_set("gemm_variant", -1)
    op_o, C_o, f_o, grid = oracle_problem(pr)
    u_o = hps.solve(op_o, f_o)
    e = max(rel_err(u[k], u_o[k]) for k in range(u_o.shape[0]))
    say(f"gemm variant {variant} {nleaf} p={p} q={q}: u {e:.2e}")
    assert e < 1e-10


def test_graph_solve_replays_match_eager(H, gpu):
    """The captured solve graph, replayed many times with different boundary
    data, right-hand-side counts and output buffers, with eager work and
    synchronisation in between, gives exactly the launch-by-launch result."""
    import torch
    pr = hi.helmholtz_bump(nleaf=(8, 8), p=12, q=10, nrhs=3)
    C, f = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
    rng = np.random.default_rng(9)
    for it in range(6):
        nrhs = (1, 3, 2)[it % 3]
        fr = _t(rng.standard_normal((nrhs, op.n_bdry)), gpu)
        H.tune_set("solve_graph", 0)
        ue = op.solve(fr).clone()
        H.tune_set("solve_graph", 1)
        junk = torch.randn(1000, device=gpu, dtype=torch.float64).sum()  # eager work between
        torch.cuda.synchronize()
        ug = op.solve(fr)
        assert torch.equal(ug, ue), it
    op_o, C_o, f_o, grid = oracle_problem(pr)
    u_o = hps.solve(op_o, f_o)
    ug = op.solve(_t(f, gpu)).cpu().numpy()
    assert max(rel_err(ug[k], u_o[k]) for k in range(u_o.shape[0])) < 1e-10
    del junk
