"""Many right-hand sides: the node-major MFMA passes against the CPU oracle.

From 16 right-hand sides on (the "solve_mm_min_rhs" knob) solves, source
solves, refinement and batched solves keep the solution node by node and run
the downward pass, the upward pass and the interface residual as grouped FP64
MFMA GEMMs.  Each case is checked against the oracle (1e-10) and against the
right-hand-side-at-a-time path (same arithmetic up to summation order).
Counts are chosen to leave ragged column tiles (16-, 32- and 64-wide tiles).
"""
import numpy as np
import pytest

import hps_inputs as hi
from oracle import hps

from .helpers import library_inputs, oracle_problem, rel_err, say

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def H(gpu):
    import paper_1307_2665_amd as H
    yield H
    H.tune_set("solve_mm_min_rhs", -1)
    H.tune_set("split_min_chunk", -1)


def _t(x, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


def _both_paths(H, fn):
    """fn() on the node-major path (threshold 1) and on the per-RHS path (0).

    The node-major path runs twice and must repeat itself exactly: its scratch
    comes from a stream-ordered pool, so a pass that read a buffer before
    writing it would pick up the first call's values."""
    H.tune_set("solve_mm_min_rhs", 1)
    a = fn()
    a2 = fn()
    H.tune_set("solve_mm_min_rhs", 0)
    b = fn()
    H.tune_set("solve_mm_min_rhs", -1)
    assert np.array_equal(a, a2)
    return a, b


@pytest.mark.parametrize("nleaf,p,q,nrhs", [((8, 6), 10, 8, 20), ((5, 7), 12, 10, 70),
                                            ((4, 4), 16, 14, 17)])
def test_solve_many_rhs(H, gpu, nleaf, p, q, nrhs):
    say(f"many-rhs solve {nleaf} p{p} q{q} nrhs {nrhs}")
    pr = hi.convdiff(nleaf=nleaf, p=p, q=q)
    op_o, C_o, f_o, grid = oracle_problem(pr)
    C, _ = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
    f = np.random.default_rng(nrhs).standard_normal((nrhs, op.n_bdry))
    fd = _t(f, gpu)
    u_mm, u_1 = _both_paths(H, lambda: op.solve(fd).cpu().numpy())
    u_o = hps.solve(op_o, f)
    e = max(rel_err(u_mm[k], u_o[k]) for k in range(nrhs))
    d = rel_err(u_mm, u_1)
    say(f"  vs oracle {e:.2e}, vs per-rhs path {d:.2e}")
    assert e < TOL and d < 1e-12


def test_sources_many_rhs(H, gpu):
    say("many-rhs sources 6x5 p10 q8, 18 rhs")
    pr = hi.convdiff(nleaf=(6, 5), p=10, q=8)
    op_o, C_o, f_o, grid = oracle_problem(pr)
    C, _ = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q, keep_factors=True)
    rng = np.random.default_rng(3)
    nrhs = 18
    f = rng.standard_normal((nrhs, op.n_bdry))
    s = rng.standard_normal((nrhs, op.N))
    s[:, op_o.boxes[0].Ie] = 0.0
    fd, sd = _t(f, gpu), _t(s, gpu)
    u_mm, u_1 = _both_paths(H, lambda: op.solve_with_sources(fd, sd).cpu().numpy())
    uo = hps.solve(op_o, f, z=hps.upward(op_o, s))
    e = max(rel_err(u_mm[k], uo[k]) for k in range(nrhs))
    say(f"  vs oracle {e:.2e}, vs per-rhs path {rel_err(u_mm, u_1):.2e}")
    assert e < TOL and rel_err(u_mm, u_1) < 1e-12


@pytest.mark.parametrize("maker", [hi.convdiff, hi.helmholtz_bump])
def test_refinement_many_rhs(H, gpu, maker):
    say(f"many-rhs refinement {maker.__name__} 8x8, 24 rhs")
    pr = maker(nleaf=(8, 8))
    op_o, C_o, f_o, grid = oracle_problem(pr)
    C, _ = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q,
                                   mode=H.HPS_MIXED_SPLIT32)
    nrhs = 24
    f = np.random.default_rng(7).standard_normal((nrhs, op.n_bdry))
    fd = _t(f, gpu)
    infos = []

    def run():
        info = {}
        u = op.solve(fd, refine=True, tol=1e-12, max_iter=20, info=info).cpu().numpy()
        infos.append(info)
        return u

    u_mm, u_1 = _both_paths(H, run)
    u_o = hps.solve(op_o, f)
    e = max(rel_err(u_mm[k], u_o[k]) for k in range(nrhs))
    say(f"  vs oracle {e:.2e} after {infos[0]['iters']} sweeps (per-rhs path "
        f"{infos[1]['iters']} sweeps), paths differ by {rel_err(u_mm, u_1):.2e}")
    assert e < TOL
    assert infos[0]["last_update_rel"] <= 1e-12
    assert rel_err(u_mm, u_1) < 1e-10


def test_batch_many_rhs(H, gpu):
    say("many-rhs batch: 3 uneven problems, 17/20/33 rhs")
    import torch
    probs = [hi.convdiff(nleaf=(4, 3), p=10, q=8), hi.convdiff(nleaf=(6, 6), p=12, q=10),
             hi.helmholtz_bump(nleaf=(3, 5))]
    ins = [library_inputs(pr) for pr in probs]
    ops = H.build_batch([dict(coeffs=_t(C, gpu), box=pr.box, nleaf=pr.nleaf, p=pr.p, q=pr.q)
                         for pr, (C, f) in zip(probs, ins)])
    rng = np.random.default_rng(11)
    fs = [_t(rng.standard_normal((k, op.n_bdry)), gpu) for k, op in zip((17, 20, 33), ops)]
    us = H.solve_batch(ops, fs)
    for pr, op, fd, u in zip(probs, ops, fs, us):
        op_o, *_ = oracle_problem(pr)
        u_o = hps.solve(op_o, fd.cpu().numpy())
        e = max(rel_err(u[k].cpu().numpy(), u_o[k]) for k in range(fd.shape[0]))
        say(f"  {pr.name} {pr.nleaf}: vs oracle {e:.2e}")
        assert e < TOL
    torch.cuda.synchronize()


@pytest.mark.parametrize("chunk", [16, 48])
def test_split_contractions(H, gpu, chunk):
    """Depths with few merges split their contractions (over me downward, over
    m3 upward) into chunks; forcing short chunks on a small problem exercises
    every split launch: solve, source solve and refinement against the oracle
    and against the unsplit passes."""
    say(f"split contractions, chunks >= {chunk}")
    pr = hi.helmholtz_bump(nleaf=(8, 8), p=12, q=10)
    op_o, C_o, f_o, grid = oracle_problem(pr)
    C, _ = library_inputs(pr)
    op = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q,
                                   mode=H.HPS_MIXED_SPLIT32)
    rng = np.random.default_rng(chunk)
    nrhs = 40
    f = rng.standard_normal((nrhs, op.n_bdry))
    s = rng.standard_normal((nrhs, op.N))
    s[:, op_o.boxes[0].Ie] = 0.0
    fd, sd = _t(f, gpu), _t(s, gpu)

    def run():
        info = {}
        u = op.solve(fd, refine=True, tol=1e-12, max_iter=20, info=info).cpu().numpy()
        w = op.solve_with_sources(fd, sd).cpu().numpy()
        return np.concatenate([u, w]), info["iters"]

    res = {}
    for c in (chunk, -1):
        H.tune_set("split_min_chunk", c)
        (a, it), (a2, _) = run(), run()
        assert np.array_equal(a, a2)
        res[c] = a
    H.tune_set("split_min_chunk", -1)
    u_o = hps.solve(op_o, f)
    e = max(rel_err(res[chunk][k], u_o[k]) for k in range(nrhs))
    d = rel_err(res[chunk], res[-1])
    say(f"  refined solve vs oracle {e:.2e} ({it} sweeps); split vs unsplit {d:.2e}")
    assert e < TOL and d < 1e-10
