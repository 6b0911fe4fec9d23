"""CPU tests of the C-ABI library: exported symbols and the host planner.

No device work happens here: these entry points are pure host code.  The
planner's tables and maps are compared with the oracle's independent
construction.
"""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import hps

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "hps.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hps_[a-z_0-9]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    import paper_1307_2665_amd as H
    names = _declared_symbols()
    assert len(names) >= 20
    lib = ctypes.CDLL(H._lib.LIB_PATH)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_mirrors_abi_names():
    import paper_1307_2665_amd as H
    for name in ("cheb_nodes", "gauss_nodes_grid", "boundary_ids", "leaf_dtn",
                 "build_solution_operator", "build_batch", "solve_batch"):
        assert callable(getattr(H, name))
    for meth in ("solve", "root_dtn_apply", "interface_residual", "solve_with_sources",
                 "export_S", "export_root_dtn", "export_leaf_dtn", "gauss_nodes",
                 "boundary_nodes"):
        assert hasattr(H.Operator, meth)


@pytest.mark.parametrize("nleaf,q,p", [((3, 2), 7, 9), ((4, 4), 14, 16), ((1, 5), 3, 4)])
def test_nodes_match_oracle(nleaf, q, p):
    import paper_1307_2665_amd as H
    box = (0.25, 1.5, -1.0, 0.5)
    g = hps.Grid(box, nleaf[0], nleaf[1], q)
    assert np.max(np.abs(H.cheb_nodes(box, nleaf, p) - g.cheb_xy(p))) < 1e-14
    assert np.max(np.abs(H.gauss_nodes_grid(box, nleaf, q) - g.node_xy())) < 1e-14
    assert np.array_equal(H.boundary_ids(nleaf, q), g.boundary(0, nleaf[0], 0, nleaf[1]))


@pytest.mark.parametrize("p,q", [(16, 14), (12, 10), (21, 20), (20, 18), (5, 3)])
def test_leaf_tables_reproduce_oracle_dtn(p, q):
    """T = P0 - P1 A_ii^-1 R from the planner's tables equals the oracle's L4 L3 L2 L1."""
    import paper_1307_2665_amd as H
    hx, hy = 0.125, 0.0625
    t = H.leaf_tables(p, q, hx, hy)
    rng = np.random.default_rng(p * 100 + q)
    coef = np.zeros((6, p * p))
    coef[0] = 1.0 + 0.3 * rng.random(p * p)
    coef[1] = 0.1 * rng.standard_normal(p * p)
    coef[2] = 1.0 + 0.3 * rng.random(p * p)
    coef[3] = 3.0 * rng.standard_normal(p * p)
    coef[4] = 3.0 * rng.standard_normal(p * p)
    coef[5] = rng.standard_normal(p * p)
    ref = hps.leaf_dtn(coef, p, q, hx, hy)
    # Rebuild the device-side formulas in NumPy from the planner's tables.
    pi = p - 2
    n = pi * pi
    Ji = t["Ji"]
    a = 1 + np.arange(n) % pi
    b = 1 + np.arange(n) // pi
    c = coef[:, Ji]
    dx = t["Dx"][np.ix_(a, a)]
    dy = t["Dy"][np.ix_(b, b)]
    same_b = (b[:, None] == b[None, :])
    same_a = (a[:, None] == a[None, :])
    A = (-2.0 * c[1][:, None] * dx * dy
         + same_b * (-c[0][:, None] * t["Dxx"][np.ix_(a, a)] + c[3][:, None] * dx)
         + same_a * (-c[2][:, None] * t["Dyy"][np.ix_(b, b)] + c[4][:, None] * dy)
         + np.diag(c[5]))
    G = t["G"]
    R = (-c[0][:, None] * G[0] - 2 * c[1][:, None] * G[1] - c[2][:, None] * G[2]
         + c[3][:, None] * G[3] + c[4][:, None] * G[4])
    T = t["P0"] - t["P1"] @ np.linalg.solve(A, R)
    assert np.max(np.abs(T - ref.T)) < 1e-11 * np.max(np.abs(ref.T))


@pytest.mark.parametrize("nleaf", [(4, 4), (3, 5), (7, 2), (1, 3)])
def test_merge_maps_match_oracle(nleaf):
    """Tree shape, J1/J2/J3 split and parent ordering agree with the oracle."""
    import paper_1307_2665_amd as H
    q = 3
    g = hps.Grid((0, 1, 0, 1), nleaf[0], nleaf[1], q)
    boxes = hps.build_tree(*nleaf)
    for b in boxes:
        b.Ie = g.boundary(b.i0, b.i1, b.j0, b.j1)
    info0 = H.plan_box(nleaf, q, 0)
    assert info0["n_boxes"] == len(boxes)
    for k, b in enumerate(boxes):
        pb = H.plan_box(nleaf, q, k)
        rec = pb["rec"]
        assert tuple(rec[:4]) == (b.i0, b.i1, b.j0, b.j1)
        assert rec[4] == b.level and rec[5] == b.parent
        if b.is_leaf:
            assert rec[6] == -1
            continue
        assert (rec[6], rec[7]) == b.children
        A, B = boxes[b.children[0]], boxes[b.children[1]]
        n = len(b.Ie)
        T_a = np.arange(len(A.Ie) ** 2, dtype=float).reshape(len(A.Ie), -1)
        T_b = -np.arange(len(B.Ie) ** 2, dtype=float).reshape(len(B.Ie), -1) - 1
        # Use the oracle merge only for its index bookkeeping (M is singular here).
        pos_a = {int(x): i for i, x in enumerate(A.Ie)}
        pos_b = {int(x): i for i, x in enumerate(B.Ie)}
        J3 = [int(x) for x in A.Ie if int(x) in pos_b]
        assert np.array_equal(pb["Ie"], b.Ie)
        assert np.array_equal(pb["Ii"], J3)
        assert np.array_equal(pb["a3"], [pos_a[x] for x in J3])
        assert np.array_equal(pb["b3"], [pos_b[x] for x in J3])
        exp = [pos_a[int(x)] if int(x) in pos_a else -pos_b[int(x)] - 1 for x in b.Ie]
        assert np.array_equal(pb["pmap"], exp)
        assert pb["sizes"][0] == n and pb["sizes"][1] == len(J3)
        del T_a, T_b


def test_invalid_arguments_are_rejected_on_host():
    import paper_1307_2665_amd as H
    with pytest.raises(H.HpsError) as e:
        H.leaf_tables(8, 10, 0.1, 0.1)           # q > p
    assert e.value.status == H.HPS_EINVAL
    with pytest.raises(H.HpsError) as e:
        H.leaf_tables(8, 8, 0.1, 0.1)            # q = p: singular merges
    assert e.value.status == H.HPS_EINVAL
    with pytest.raises(H.HpsError):
        H.leaf_tables(3, 2, 0.1, 0.1)            # p < 4
    with pytest.raises(H.HpsError):
        H.plan_box((0, 3), 4, 0)                 # empty grid


def test_tuning_cache_round_trip(tmp_path):
    """The tuning table's JSON cache loads, saves back the same entries, and
    malformed files or knob values are rejected (host code only)."""
    import json
    import paper_1307_2665_amd as H
    H.tune_reset()
    entries = [
        {"knob": 1, "name": "gemm", "key": [6, 6, 4, 11], "variant": 2, "ms": 0.5, "default_ms": 0.75,
         "all_ms": [0.75, 0.625, 0.5, 1.5, 2.0, 0.875, 0.625, 0.5625]},
        {"knob": 2, "name": "gj", "key": [10, 13, 0, 0], "variant": 9, "ms": 3.25, "default_ms": 4.5},
        {"knob": 0, "name": "leaf", "key": [196, 56, 0, 0], "variant": 4, "ms": 6.0, "default_ms": 6.0},
    ]
    src = tmp_path / "in.json"
    src.write_text('{\n  "format": "hps-tune-2",\n  "entries": [\n' +
                   ",\n".join("    " + json.dumps(e) for e in entries) + "\n  ]\n}\n")
    H.tune_load(src)
    out = tmp_path / "out.json"
    H.tune_save(out)
    got = json.loads(out.read_text())
    assert got["format"] == "hps-tune-2"
    key = lambda e: (e["knob"], tuple(e["key"]))
    assert sorted(((key(e), e["variant"]) for e in got["entries"])) == \
        sorted(((key(e), e["variant"]) for e in entries))
    # Every tile's time of a GEMM bucket survives the round trip.
    assert sorted(got["entries"], key=key) == sorted(entries, key=key)
    H.tune_reset()
    H.tune_save(out)
    assert json.loads(out.read_text())["entries"] == []
    bad = tmp_path / "bad.json"
    bad.write_text('{"entries": []}')
    with pytest.raises(H.HpsError) as e:
        H.tune_load(bad)
    assert e.value.status == H.HPS_EINVAL
    for knob, v in (("gemm_variant", 8), ("gj_variant", 3), ("leaf_variant", 5), ("nope", 0)):
        with pytest.raises(H.HpsError) as e:
            H.tune_set(knob, v)
        assert e.value.status == H.HPS_EINVAL


@pytest.mark.parametrize("p,q", [(12, 12), (8, 8), (6, 9)])
def test_build_refuses_q_not_below_p(p, q):
    """The build validates 1 <= q <= p - 1 before any device work: with q >= p
    every interior cross point carries a mode that no leaf sees (section 3.2,
    step 1), so the merge systems are singular (pinned on the oracle)."""
    import paper_1307_2665_amd as H
    C = np.zeros((4, 6, p * p))
    C[:, 0] = C[:, 2] = 1.0
    with pytest.raises(H.HpsError) as e:
        H.build_solution_operator(C, (0.0, 1.0, 0.0, 1.0), (2, 2), p, q)
    assert e.value.status == H.HPS_EINVAL
    assert "q" in str(e.value)


def test_tuning_cache_of_older_format_is_refused(tmp_path):
    import paper_1307_2665_amd as H
    old = tmp_path / "old.json"
    old.write_text('{"format": "hps-tune-1", "entries": []}')
    with pytest.raises(H.HpsError) as e:
        H.tune_load(old)
    assert e.value.status == H.HPS_EINVAL


def test_hbs_sizes_follow_the_documented_layout():
    """hps_hbs_sizes counts the blocks that include/hps.h lists (host code only),
    and sizes outside the limits are rejected."""
    import paper_1307_2665_amd as H
    for L, m, k in [(1, 16, 4), (3, 40, 12), (6, 160, 80), (14, 8, 2)]:
        nf, ni = H.hbs_sizes(L, m, k)
        leaves = (1 << L) * (m * m + 2 * m * k)
        parents = sum((1 << l) * 4 * k * k for l in range(1, L))
        b = sum((1 << l) * 4 * k * k for l in range(0, L))
        assert nf == leaves + parents + b
        inv = (1 << L) * (2 * m * k + m * m)
        inv += sum((1 << l) * (2 * 2 * k * k + 4 * k * k) for l in range(1, L)) + 4 * k * k
        assert ni == inv
    for L, m, k in [(0, 16, 4), (15, 16, 4), (3, 8, 9), (3, 16, 0), (2, 4000, 4)]:
        with pytest.raises(H.HpsError) as e:
            H.hbs_sizes(L, m, k)
        assert e.value.status == H.HPS_EINVAL
