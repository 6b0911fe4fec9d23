"""Learned leaf-DtN surrogate: kernels against the FP64 oracle network, training,
and what the trained network gains over the plain leaf build.

The surrogate's *accuracy* has no reference in the paper ("parity unpinned");
its training kernels are pinned by the FP64 oracle network (itself pinned by
finite differences), and its error is judged by the FP64 leaf solver.
"""
import numpy as np
import pytest

import hps_inputs as hi
from oracle import hps, mlp

from .helpers import library_inputs, rel_err, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def H(gpu):
    import paper_1307_2665_amd as H
    return H


def _t(x, dev):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=torch.float64, device=dev)


def _bf16(x):
    """Round FP32 values to BF16 (nearest even), returned as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    return (u.astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def _patches(p, q, h, fields, per_field, rng):
    """Coefficient samples (c11 = c22 = 1 + g/2, c = 1 + g') of random leaves of the given fields."""
    out = []
    xc = hps.cheb_points(p)
    for pr in fields:
        for _ in range(per_field):
            x0, y0 = rng.uniform(0, 1 - h, size=2)
            X = x0 + 0.5 * (xc + 1) * h
            Y = y0 + 0.5 * (xc + 1) * h
            xx, yy = np.meshgrid(X, Y)
            xy = np.stack([xx.ravel(), yy.ravel()], axis=1)[None]
            out.append(pr.coeffs_at(xy)[0])
    return np.array(out)


def test_gradients_match_fp64_oracle(H, gpu):
    p, q, hid, r = 6, 4, 48, 3
    h = 1.0 / 32
    rng = np.random.default_rng(0)
    C = _patches(p, q, h, [hi.sweep_field(6000 + i, p=p, q=q) for i in range(3)], 20, rng)
    n, m = C.shape[0], 4 * q
    mats = hps.leaf_matrices(p, q, h, h)
    T = np.array([hps.leaf_dtn(c, p, q, h, h, mats).T for c in C])
    lap = np.zeros((6, p * p))
    lap[0] = lap[2] = 1.0
    Tref = hps.leaf_dtn(lap, p, q, h, h, mats).T
    sg = H.Surrogate.create(p, q, h, h, hidden=hid, rank=r, seed=3)
    Cd, Td = _t(C, gpu), _t(T, gpu)
    sg.train(Cd, Td, epochs=1, batch=n, lr=0.0)      # fixes the normalisation only
    st = sg.state()
    L, G = sg.grad(Cd, Td)
    # FP64 oracle with the same BF16 weights, normalisation and targets.
    P = dict(W1=_bf16(st["W1"]), b1=st["b1"].astype(np.float64), W2=_bf16(st["W2"]),
             b2=st["b2"].astype(np.float64), W3=_bf16(st["W3"]), b3=st["b3"].astype(np.float64))
    feats = np.concatenate([C[:, 0], C[:, 2], C[:, 5]], axis=1)
    X = ((feats - st["mu"].astype(np.float64)) / st["sigma"].astype(np.float64)).astype(np.float32)
    Y = (T - Tref[None]) / st["out_scale"]
    Lo, Go = mlp.loss_and_grads(P, X.astype(np.float64), Y, m, r)
    say(f"loss gpu {L:.6e} oracle {Lo:.6e}")
    assert abs(L - Lo) < 2e-2 * Lo
    for k in mlp.PARAM_NAMES:
        e = np.max(np.abs(G[k].reshape(Go[k].shape) - Go[k])) / np.max(np.abs(Go[k]))
        say(f"  d{k}: rel err {e:.2e}")
        assert e < 5e-3, (k, e)


def test_training_reduces_loss(H, gpu):
    p, q = 12, 10
    h = 1.0 / 256
    rng = np.random.default_rng(1)
    C = _patches(p, q, h, [hi.sweep_field(6000 + i) for i in range(8)], 250, rng)
    Cd = _t(C, gpu)
    Td = H.leaf_dtn(Cd, h, h, p, q)
    sg = H.Surrogate.create(p, q, h, h, hidden=128, rank=8, seed=1)
    hist = sg.train(Cd, Td, epochs=30, batch=128, lr=2e-3, seed=2)
    say(f"loss history {hist[0]:.3e} -> {hist[-1]:.3e}")
    assert hist[-1] < 0.5 * hist[0]


@pytest.fixture(scope="module")
def trained(H, gpu):
    """Surrogate for the 256 x 256, p = 12, q = 10 sweep, trained on leaf solves of fields
    6000-6039 (500 random leaves each, 20k pairs)."""
    p, q = 12, 10
    h = 1.0 / 256
    rng = np.random.default_rng(6)
    C = _patches(p, q, h, [hi.sweep_field(6000 + i) for i in range(40)], 500, rng)
    Cd = _t(C, gpu)
    Td = H.leaf_dtn(Cd, h, h, p, q)
    sg = H.Surrogate.create(p, q, h, h, hidden=256, rank=16, seed=5)
    hist = sg.train(Cd, Td, epochs=40, batch=256, lr=1e-3, seed=7)
    say(f"trained: loss {hist[0]:.3e} -> {hist[-1]:.3e}")
    return sg


def test_surrogate_sweep_gain_and_error(H, gpu, trained, tmp_path):
    """Held-out field 5000 on 256 x 256 leaves: leaf stage time and solution error,
    surrogate vs the plain FP64 leaf build (both on this GPU)."""
    import torch
    pr = hi.sweep_field(5000)
    C, f = library_inputs(pr)
    Cd, fd = _t(C, gpu), _t(f, gpu)
    import time
    leaf_classes = ["leaf_assemble", "leaf_lu", "leaf_gemm", "mlp_infer"]

    def build(**kw):
        """(operator, leaf-stage ms from HIP events, wall ms of the whole build)."""
        torch.cuda.synchronize()
        H.prof_enable(leaf_classes)
        H.prof_reset()
        t0 = time.perf_counter()
        op = H.build_solution_operator(Cd, pr.box, pr.nleaf, pr.p, pr.q, **kw)
        torch.cuda.synchronize()
        wall = 1e3 * (time.perf_counter() - t0)
        leaf = sum(H.prof_query(c)["ms"] for c in leaf_classes)
        H.prof_enable([])
        return op, leaf, wall

    sk = dict(surrogate=trained, judge_samples=256, judge_tol=1e-6)
    build()                                         # warm-up (plans, memory cache)
    build(**sk)
    op_f, t_plain, w_plain = build()
    op_s, t_sur, w_sur = build(**sk)
    say(f"build wall time: plain {w_plain:.1f} ms, surrogate {w_sur:.1f} ms")
    u_f = op_f.solve(fd).cpu().numpy()
    u_s = op_s.solve(fd).cpu().numpy()
    err = rel_err(u_s, u_f)
    # The network-free baseline: every leaf DtN replaced by T_Laplace(h) (the
    # leaf operator is -a Lap u + c u, so c = 0 gives exactly T_Laplace).
    C0 = C.copy()
    C0[:, 5] = 0.0
    op_0 = H.build_solution_operator(_t(C0, gpu), pr.box, pr.nleaf, pr.p, pr.q)
    err0 = rel_err(op_0.solve(fd).cpu().numpy(), u_f)
    say(f"leaf stage (assembly, elimination, T products, inference): plain {t_plain:.2f} ms, "
        f"surrogate {t_sur:.2f} ms; u rel err: "
        f"surrogate {err:.2e}, T_Laplace-only {err0:.2e}; judged {op_s.n_judged} leaves, "
        f"worst {op_s.judge_worst:.2e}, fallback leaves {op_s.n_fallback_leaves}")
    assert op_s.n_judged == 256 and op_s.n_fallback_leaves == 0
    assert t_sur < 0.5 * t_plain
    assert w_sur < w_plain
    assert err < 1e-3 and err < 0.2 * err0
    # save / load round trip keeps predictions bit-identical
    path = tmp_path / "sur.bin"
    trained.save(path)
    again = H.Surrogate.load(path)
    a = trained.predict(Cd[:64])
    b = again.predict(Cd[:64])
    assert torch.equal(a, b)


def test_out_of_distribution_leaves_are_judged(H, gpu, trained):
    """c = 25 is far outside the training range [0, 2]: every leaf is flagged and
    re-solved by the FP64 leaf solver (replaced where above the tolerance)."""
    pr = hi.Problem("ood", [hi.ONE, hi.ZERO, hi.ONE, hi.ZERO, hi.ZERO, hi._const(25.0)],
                    nleaf=(256, 256), p=12, q=10, bc=[hi.cos_bc])
    C, f = library_inputs(pr)
    op_s = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q, surrogate=trained,
                                     judge_samples=64, judge_tol=1e-9)
    say(f"ood: judged {op_s.n_judged}, replaced {op_s.n_fallback_leaves}, "
        f"worst sampled {op_s.judge_worst:.2e}")
    assert op_s.n_judged == 256 * 256
    op_f = H.build_solution_operator(_t(C, gpu), pr.box, pr.nleaf, pr.p, pr.q)
    # every leaf above 1e-9 was replaced by its FP64 DtN, so the operators agree closely
    assert rel_err(op_s.export_root_dtn(), op_f.export_root_dtn()) < 1e-6


def test_tolerance_failure_rebuilds_every_leaf(H, gpu, trained):
    """A tolerance the network cannot meet fails the random sample: all leaves are rebuilt."""
    pr = hi.sweep_field(5001)
    C, f = library_inputs(pr)
    Cd = _t(C, gpu)
    op_s = H.build_solution_operator(Cd, pr.box, pr.nleaf, pr.p, pr.q, surrogate=trained,
                                     judge_samples=64, judge_tol=1e-13)
    assert op_s.n_fallback_leaves == 256 * 256
    op_f = H.build_solution_operator(Cd, pr.box, pr.nleaf, pr.p, pr.q)
    assert rel_err(op_s.export_root_dtn(), op_f.export_root_dtn()) < 1e-13
