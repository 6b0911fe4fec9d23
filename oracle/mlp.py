"""FP64 oracle of the leaf-DtN surrogate network (not in the paper).

Test infrastructure only (see ``oracle/__init__.py``).

The surrogate replaces the leaf computation of section 3 for coefficient
fields of the form A u = -c11 u_11 - c22 u_22 + c u.  For one leaf:

  x  = ((c11, c22, c) at the p^2 Chebyshev nodes - mu) / sigma     (D = 3 p^2)
  h1 = tanh(W1 x + b1)                                              (H)
  h2 = tanh(W2 h1 + b2)                                             (H)
  o  = W3 h2 + b3                                                   (2 m r, m = 4q)
  U  = o[:m r] as m x r (row-major),  V = o[m r:] as m x r
  T  = T_ref + s U V^T

T_ref is the leaf DtN of the Laplace operator for the same leaf size and s a
fixed output scale.  Training minimises the mean over samples of
  L = (1/m^2) sum_ij (U V^T - Y)_ij^2,   Y = (T_exact - T_ref) / s.

Parity of the surrogate's *output* is unpinned by the paper (a learned map has
no closed form); these functions pin the GPU training kernels: forward values,
loss and every gradient, and they are pinned themselves by central finite
differences.
"""
from __future__ import annotations

import numpy as np

PARAM_NAMES = ("W1", "b1", "W2", "b2", "W3", "b3")


def init_params(D: int, H: int, O: int, rng: np.random.Generator) -> dict:
    """Uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) weights, zero biases."""
    def u(n_out, n_in):
        a = 1.0 / np.sqrt(n_in)
        return rng.uniform(-a, a, size=(n_out, n_in))
    return dict(W1=u(H, D), b1=np.zeros(H), W2=u(H, H), b2=np.zeros(H), W3=u(O, H),
                b3=np.zeros(O))


def forward(P: dict, X: np.ndarray, m: int, r: int):
    """X [B, D] (already normalised) -> U [B, m, r], V [B, m, r] and a cache."""
    a1 = X @ P["W1"].T + P["b1"]
    h1 = np.tanh(a1)
    a2 = h1 @ P["W2"].T + P["b2"]
    h2 = np.tanh(a2)
    o = h2 @ P["W3"].T + P["b3"]
    B = X.shape[0]
    U = o[:, :m * r].reshape(B, m, r)
    V = o[:, m * r:].reshape(B, m, r)
    return U, V, dict(X=X, h1=h1, h2=h2, o=o)


def loss_and_grads(P: dict, X: np.ndarray, Y: np.ndarray, m: int, r: int):
    """Mean loss over the batch and its gradient with respect to every parameter."""
    B = X.shape[0]
    U, V, c = forward(P, X, m, r)
    R = U @ V.transpose(0, 2, 1) - Y                     # [B, m, m]
    loss = float(np.sum(R * R) / (m * m) / B)
    g = 2.0 / (m * m) / B
    dU = g * R @ V                                       # dL/dU
    dV = g * R.transpose(0, 2, 1) @ U                    # dL/dV
    do = np.concatenate([dU.reshape(B, -1), dV.reshape(B, -1)], axis=1)
    grads = {}
    grads["W3"] = do.T @ c["h2"]
    grads["b3"] = do.sum(axis=0)
    dh2 = do @ P["W3"]
    da2 = dh2 * (1.0 - c["h2"] ** 2)
    grads["W2"] = da2.T @ c["h1"]
    grads["b2"] = da2.sum(axis=0)
    dh1 = da2 @ P["W2"]
    da1 = dh1 * (1.0 - c["h1"] ** 2)
    grads["W1"] = da1.T @ c["X"]
    grads["b1"] = da1.sum(axis=0)
    return loss, grads


def loss_only(P, X, Y, m, r) -> float:
    U, V, _ = forward(P, X, m, r)
    R = U @ V.transpose(0, 2, 1) - Y
    return float(np.sum(R * R) / (m * m) / X.shape[0])


def adam_step(P: dict, G: dict, M: dict, S: dict, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba), bias-corrected, in place."""
    for k in PARAM_NAMES:
        M[k] = b1 * M[k] + (1 - b1) * G[k]
        S[k] = b2 * S[k] + (1 - b2) * G[k] ** 2
        mh = M[k] / (1 - b1 ** t)
        sh = S[k] / (1 - b2 ** t)
        P[k] = P[k] - lr * mh / (np.sqrt(sh) + eps)
