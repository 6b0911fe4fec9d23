"""Pins of the FP64 surrogate-network oracle: central finite differences and
the closed form of a first Adam step."""
import numpy as np

from oracle import mlp


def _setup(seed=0, B=5, D=12, H=9, m=6, r=2):
    rng = np.random.default_rng(seed)
    P = mlp.init_params(D, H, 2 * m * r, rng)
    for k in ("b1", "b2", "b3"):
        P[k] = 0.1 * rng.standard_normal(P[k].shape)
    X = rng.standard_normal((B, D))
    Y = rng.standard_normal((B, m, m))
    return P, X, Y, m, r, rng


def test_gradients_match_central_differences():
    P, X, Y, m, r, rng = _setup()
    loss, G = mlp.loss_and_grads(P, X, Y, m, r)
    assert abs(loss - mlp.loss_only(P, X, Y, m, r)) < 1e-14
    eps = 1e-6
    for k in mlp.PARAM_NAMES:
        flat = P[k].reshape(-1)
        for idx in rng.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + eps
            lp = mlp.loss_only(P, X, Y, m, r)
            flat[idx] = old - eps
            lm = mlp.loss_only(P, X, Y, m, r)
            flat[idx] = old
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - G[k].reshape(-1)[idx]) < 1e-7 * max(1.0, abs(fd)), (k, idx)


def test_lowrank_output_layout():
    """U is the first m*r outputs row-major, V the rest (the layout the GPU uses)."""
    P, X, Y, m, r, rng = _setup()
    U, V, c = mlp.forward(P, X, m, r)
    o = c["o"]
    assert np.array_equal(U[1, 2], o[1, 2 * r:3 * r])
    assert np.array_equal(V[3, 0], o[3, m * r:m * r + r])


def test_first_adam_step_is_lr_times_sign():
    P = {k: np.array([1.0, -2.0]) for k in mlp.PARAM_NAMES}
    G = {k: np.array([0.3, -5.0]) for k in mlp.PARAM_NAMES}
    M = {k: np.zeros(2) for k in mlp.PARAM_NAMES}
    S = {k: np.zeros(2) for k in mlp.PARAM_NAMES}
    mlp.adam_step(P, G, M, S, 1, lr=0.01, eps=0.0)
    assert np.allclose(P["W1"], [1.0 - 0.01, -2.0 + 0.01], atol=1e-15)
