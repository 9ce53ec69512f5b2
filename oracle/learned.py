"""Learned smoothness sensor, float64 reference (TEST INFRASTRUCTURE ONLY).

The paper uses the cell-vertex WENO sensor gamma_e (Sec. 3.2, eq. gamma); this
module defines a small network that predicts gamma_e from normalised
cell-plus-vertex Hermite data, trained on gamma_e of the method itself.  The
paper does not define it; the layout is this project's reading:

features (48 per cell), sigma_e = ||s^e||_e + 1e-12 sigma_ref (eq. snorm):
  * 4 vertex slots x 9 multi-indices 1 <= |k| <= 3 (order |k|, then
    decreasing first component): h_e^|k| (c_i[k] - D^k s^e(x_i)) / sigma_e,
    the mismatch between the vertex candidate (eq. taylorcand) and the cell's
    own Hermite data (eq. taylorsol) at its local vertex i; orders above p are 0;
  * 9 slots h_e^|k| D^k s^e(x_c) / sigma_e at the reference centroid x_c;
  * log10(sigma_e / sigma_ref), and the largest and the mean of the four
    per-vertex mismatch 2-norms.
network: 48 -> 64 -> 64 -> 1, GELU (erf form) after both hidden layers, a
sigmoid at the output, so gamma lies in [0, 1].  Loss: mean squared error
against the plain sensor; Adam.

Inference on the device rounds the inputs, the weights and both hidden
activations to bfloat16 (round to nearest even) and accumulates in float32;
``mlp_forward(..., bf16=True)`` rounds at the same points.  Training keeps the
activations unrounded (weights and inputs rounded), which is what
``mlp_loss_grad`` differentiates.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

from .basis import multi_indices
from .geometry import physical_derivatives, map_jacobian
from .method import element_seminorm_sq, hermite_at_vertices

N_FEAT = 48
N_HID = 64
SLOTS = multi_indices(2, 3)                       # the 9 multi-indices 1 <= |k| <= 3


# ---------------------------------------------------------------------------
# bfloat16 rounding (float64 -> float32 -> bfloat16, nearest even)
# ---------------------------------------------------------------------------
def bf16_round(x):
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    b = f.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------
def ref_centroid(ref):
    if ref.n_vert == 3:
        return np.array([[1.0 / 3.0, 1.0 / 3.0]])
    return np.zeros((1, ref.dim))


def cell_seminorm(sp, s):
    """n_e = ||s^e||_e of eq. (snorm) on the cell's semi-norm rule; [E]."""
    ref = sp.ref
    pts = ref.norm_pts
    J, _ = map_jacobian(sp.cell, sp.X, pts)
    W = ref.norm_w[None, :] * np.abs(np.linalg.det(J))
    Du = physical_derivatives(ref, sp.cell, sp.X, s, pts, sp.ks)
    return np.sqrt(element_seminorm_sq(sp, np.stack([Du[k] for k in sp.ks], axis=-1), W))


def features(sp, s, c, sigma_ref: float):
    """[E, 48] features of every cell; s [E, n_loc] sensor field, c [N_v, n_k]
    vertex candidates (eq. taylorcand), sigma_ref > 0 the reference scale."""
    if sp.ref.dim != 2:
        raise NotImplementedError("features are defined for two-dimensional meshes")
    E = sp.E
    ve = sp.mesh.cell_vertices.shape[1]
    if ve != 4:
        raise NotImplementedError("features are defined for quadrilaterals (four vertex slots)")
    sigma = cell_seminorm(sp, s) + 1e-12 * sigma_ref
    H = hermite_at_vertices(sp, s)                                   # [E, 4, n_k]
    Dc = physical_derivatives(sp.ref, sp.cell, sp.X, s, ref_centroid(sp.ref), sp.ks)
    out = np.zeros((E, N_FEAT))
    slot = {k: t for t, k in enumerate(SLOTS)}
    mis = np.zeros((E, 4, 9))
    for t, k in enumerate(sp.ks):
        scale = sp.h ** sum(k) / sigma
        for l in range(4):
            ci = c[sp.mesh.cell_vertices[:, l], t]
            mis[:, l, slot[k]] = scale * (ci - H[:, l, t])
        out[:, 36 + slot[k]] = scale * Dc[k][:, 0]
    out[:, :36] = mis.reshape(E, 36)
    norms = np.sqrt((mis * mis).sum(-1))                              # [E, 4]
    out[:, 45] = np.log10(sigma / sigma_ref)
    out[:, 46] = norms.max(1)
    out[:, 47] = norms.mean(1)
    return out


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def gelu(x):
    return 0.5 * x * (1.0 + erf(x / math.sqrt(2.0)))


def gelu_prime(x):
    return 0.5 * (1.0 + erf(x / math.sqrt(2.0))) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


def mlp_init(seed: int):
    """Weights N(0, 1/fan_in), zero biases."""
    rng = np.random.default_rng(seed)
    return {"W1": rng.normal(size=(N_FEAT, N_HID)) / math.sqrt(N_FEAT), "b1": np.zeros(N_HID),
            "W2": rng.normal(size=(N_HID, N_HID)) / math.sqrt(N_HID), "b2": np.zeros(N_HID),
            "w3": rng.normal(size=N_HID) / math.sqrt(N_HID), "b3": np.zeros(1)}


def bf16_weights(P):
    """The bfloat16 compute copies of the weight matrices (biases stay float32)."""
    Q = dict(P)
    for k in ("W1", "W2", "w3"):
        Q[k] = bf16_round(P[k])
    for k in ("b1", "b2", "b3"):
        Q[k] = np.asarray(P[k], np.float32).astype(np.float64)
    return Q


def mlp_forward(P, X, bf16: bool = False):
    """gamma [n] for features X [n, 48]; bf16=True rounds inputs, weights and
    the hidden activations as the device's inference does."""
    if bf16:
        P = bf16_weights(P)
        X = bf16_round(X)
    z1 = X @ P["W1"] + P["b1"]
    h1 = gelu(z1)
    if bf16:
        h1 = bf16_round(h1)
    z2 = h1 @ P["W2"] + P["b2"]
    h2 = gelu(z2)
    if bf16:
        h2 = bf16_round(h2)
    z3 = h2 @ P["w3"] + P["b3"][0]
    return sigmoid(z3)


def mlp_loss_grad(P, X, t):
    """Loss mean((gamma - t)^2) and its gradient with respect to every
    parameter, by the chain rule written out layer by layer."""
    n = X.shape[0]
    z1 = X @ P["W1"] + P["b1"]
    h1 = gelu(z1)
    z2 = h1 @ P["W2"] + P["b2"]
    h2 = gelu(z2)
    z3 = h2 @ P["w3"] + P["b3"][0]
    g = sigmoid(z3)
    loss = np.mean((g - t) ** 2)
    d3 = 2.0 * (g - t) / n * g * (1.0 - g)              # dL/dz3 [n]
    G = {"w3": h2.T @ d3, "b3": np.array([d3.sum()])}
    d2 = np.outer(d3, P["w3"]) * gelu_prime(z2)          # dL/dz2 [n, 64]
    G["W2"] = h1.T @ d2
    G["b2"] = d2.sum(0)
    d1 = (d2 @ P["W2"].T) * gelu_prime(z1)               # dL/dz1 [n, 64]
    G["W1"] = X.T @ d1
    G["b1"] = d1.sum(0)
    return loss, G


def adam_init(P):
    return {"t": 0, "m": {k: np.zeros_like(np.asarray(v, np.float64)) for k, v in P.items()},
            "v": {k: np.zeros_like(np.asarray(v, np.float64)) for k, v in P.items()}}


def adam_step(P, G, state, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """One Adam update (bias-corrected first and second moments)."""
    state["t"] += 1
    t = state["t"]
    out = {}
    for k in P:
        m = state["m"][k] = b1 * state["m"][k] + (1.0 - b1) * G[k]
        v = state["v"][k] = b2 * state["v"][k] + (1.0 - b2) * G[k] * G[k]
        mh = m / (1.0 - b1 ** t)
        vh = v / (1.0 - b2 ** t)
        out[k] = P[k] - lr * mh / (np.sqrt(vh) + eps)
    return out


def train_step(P, state, X, t, lr: float):
    """One training step as the device performs it: the gradient of the loss
    of the network with bfloat16-rounded weights and inputs (unrounded
    activations), applied by Adam to the float32 master weights."""
    loss, G = mlp_loss_grad(bf16_weights(P), bf16_round(X), t)
    return adam_step(P, G, state, lr), loss
