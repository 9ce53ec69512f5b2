"""Pins of the learned-sensor reference (oracle/learned.py): bfloat16 rounding
by its definition, GELU special values and identities, the hand-written
backward against central finite differences, Adam in closed form, the network
wiring by one-hot routing, and the features on polynomial data (exact vertex
candidates, analytic centroid derivatives), under rescaling of the data and
by slot position."""
import math

import numpy as np
import pytest
from scipy.stats import norm

import synth
from oracle import build_space
from oracle.method import vertex_candidates, hermite_at_vertices
from oracle.learned import (bf16_round, gelu, gelu_prime, sigmoid, mlp_init, mlp_forward, mlp_loss_grad,
                            adam_init, adam_step, features, cell_seminorm, N_FEAT, N_HID, SLOTS)


def test_bf16_rounding_by_definition():
    # 8 significant bits: the spacing above 1 is 2^-7; halfway cases go to the even mantissa
    x = np.array([1.0, 1 + 2 ** -8, 1 + 3 * 2 ** -8, 1 + 2 ** -8 + 2 ** -20, -(1 + 3 * 2 ** -8), 3.0, 2 ** -130])
    want = np.array([1.0, 1.0, 1 + 2 ** -6, 1 + 2 ** -7, -(1 + 2 ** -6), 3.0, 2 ** -130])
    assert np.array_equal(bf16_round(x), want)
    r = np.random.default_rng(0).normal(size=1000)
    q = bf16_round(r)
    assert np.all(np.abs(q - r) <= 2 ** -8 * np.abs(r))     # half a spacing 2^(e-7) <= 2^-8 |r|
    assert np.array_equal(bf16_round(q), q)                               # idempotent


def test_gelu_identities():
    x = np.linspace(-6, 6, 121)
    assert gelu(np.array([0.0]))[0] == 0.0
    assert np.allclose(gelu(x) - gelu(-x), x, atol=1e-15)
    assert np.allclose(gelu(x), x * norm.cdf(x), atol=1e-15, rtol=1e-13)   # x Phi(x)
    h = 1e-6
    assert np.allclose(gelu_prime(x), (gelu(x + h) - gelu(x - h)) / (2 * h), atol=1e-8)
    assert abs(sigmoid(np.array([0.0]))[0] - 0.5) < 1e-16


def test_backward_against_finite_differences():
    rng = np.random.default_rng(1)
    P = mlp_init(3)
    P["b1"] = rng.normal(size=N_HID) * 0.1
    P["b2"] = rng.normal(size=N_HID) * 0.1
    P["b3"] = np.array([0.2])
    X = rng.normal(size=(37, N_FEAT))
    t = rng.uniform(size=37)
    loss, G = mlp_loss_grad(P, X, t)
    h = 1e-6
    for key in P:
        flat = P[key].reshape(-1)
        idx = rng.choice(flat.size, min(12, flat.size), replace=False)
        for i in idx:
            Pp = {k: v.copy() for k, v in P.items()}
            Pm = {k: v.copy() for k, v in P.items()}
            Pp[key].reshape(-1)[i] += h
            Pm[key].reshape(-1)[i] -= h
            fd = (mlp_loss_grad(Pp, X, t)[0] - mlp_loss_grad(Pm, X, t)[0]) / (2 * h)
            an = G[key].reshape(-1)[i]
            assert abs(fd - an) <= 1e-6 * max(1e-3, abs(an)) + 1e-10, (key, i, fd, an)


def test_adam_closed_form():
    """Constant gradient: the bias-corrected moments equal g and g^2 at every
    step, so each step moves a parameter by lr g / (|g| + eps)."""
    P = {"a": np.array([1.0, -2.0, 0.5]), "b": np.array([0.0])}
    G = {"a": np.array([0.3, -1e-3, 5.0]), "b": np.array([-2.0])}
    st = adam_init(P)
    lr, eps = 1e-2, 1e-8
    Q = P
    for k in range(1, 6):
        Q = adam_step(Q, G, st, lr, eps=eps)
        for key in P:
            assert np.allclose(Q[key], P[key] - k * lr * G[key] / (np.abs(G[key]) + eps), rtol=0, atol=1e-12)


def test_network_wiring_by_one_hot_routing():
    """Feature 5 -> hidden 17 -> hidden 3 -> output: gamma = sigmoid(w gelu(gelu(x5) ...))."""
    P = {"W1": np.zeros((N_FEAT, N_HID)), "b1": np.zeros(N_HID), "W2": np.zeros((N_HID, N_HID)),
         "b2": np.zeros(N_HID), "w3": np.zeros(N_HID), "b3": np.array([0.25])}
    P["W1"][5, 17] = 2.0
    P["W2"][17, 3] = -1.5
    P["w3"][3] = 0.75
    P["b1"][17] = 0.1
    X = np.zeros((3, N_FEAT))
    X[:, 5] = [0.0, 1.0, -2.0]
    X[1, 6] = 9.0                      # a feature that is not routed
    want = 1.0 / (1.0 + np.exp(-(0.75 * gelu(-1.5 * gelu(2.0 * X[:, 5] + 0.1)) + 0.25)))
    assert np.allclose(mlp_forward(P, X), want, rtol=1e-14)
    # constant output when nothing is routed
    Z = {k: np.zeros_like(v) for k, v in P.items()}
    Z["b3"] = np.array([-1.0])
    assert np.allclose(mlp_forward(Z, np.random.default_rng(0).normal(size=(4, N_FEAT))), 1 / (1 + math.e))


def _poly_case(p, a=1.0, b=0.0):
    """A global polynomial of total degree p on a non-periodic 6 x 5 grid."""
    mesh = synth.quad_mesh(6, 5, periodic=(False, False))
    sp = build_space(mesh, p, 1)
    xn = sp.node_coords()
    x, y = xn[..., 0], xn[..., 1]
    coef = [0.3, -1.2, 0.7, 0.9, -0.4, 1.1, 0.5, -0.8, 0.6, 0.2]
    terms = [x, y, x * x, x * y, y * y, x ** 3, x * x * y, x * y * y, y ** 3]
    orders = [1, 1, 2, 2, 2, 3, 3, 3, 3]
    s = coef[0] + sum(c * t for c, t, o in zip(coef[1:], terms, orders) if o <= p)
    return mesh, sp, a * s + b, coef


def _interior(mesh):
    """Cells whose four vertices have full patches (no boundary vertex)."""
    cv = mesh.cell_vertices
    cnt = np.bincount(cv.ravel(), minlength=mesh.n_vertices)
    return np.nonzero((cnt[cv] == 4).all(1))[0]


@pytest.mark.parametrize("p", [1, 2, 3])
def test_features_on_polynomial_data(p):
    mesh, sp, s, coef = _poly_case(p)
    c = vertex_candidates(sp, s, synth.Params())
    F = features(sp, s, c, sigma_ref=1.0)
    inner = _interior(mesh)
    assert len(inner) >= 8
    # vertex candidates reproduce the polynomial's derivatives exactly
    assert np.abs(F[inner, :36]).max() < 1e-9
    assert np.abs(F[inner, 46:48]).max() < 1e-9
    # centroid slots: h^|k| D^k s(x_c) / sigma_e with the derivatives by hand
    xc = mesh.cell_coords.mean(1)
    x, y = xc[:, 0], xc[:, 1]
    c1, c2, c3, c4, c5, c6, c7, c8, c9 = coef[1:]
    D = {(1, 0): c1 + 2 * c3 * x + c4 * y, (0, 1): c2 + c4 * x + 2 * c5 * y,
         (2, 0): 2 * c3 + 0 * x, (1, 1): c4 + 0 * x, (0, 2): 2 * c5 + 0 * x}
    if p >= 3:
        D[(1, 0)] = D[(1, 0)] + 3 * c6 * x * x + 2 * c7 * x * y + c8 * y * y
        D[(0, 1)] = D[(0, 1)] + c7 * x * x + 2 * c8 * x * y + 3 * c9 * y * y
        D[(2, 0)] = D[(2, 0)] + 6 * c6 * x + 2 * c7 * y
        D[(1, 1)] = D[(1, 1)] + 2 * c7 * x + 2 * c8 * y
        D[(0, 2)] = D[(0, 2)] + 2 * c8 * x + 6 * c9 * y
        D.update({(3, 0): 6 * c6 + 0 * x, (2, 1): 2 * c7 + 0 * x, (1, 2): 2 * c8 + 0 * x, (0, 3): 6 * c9 + 0 * x})
    if p == 1:
        D = {(1, 0): c1 + 0 * x, (0, 1): c2 + 0 * x}
    sigma = cell_seminorm(sp, s) + 1e-12
    for t, k in enumerate(SLOTS):
        got = F[:, 36 + t]
        if k in D:
            want = sp.h ** sum(k) * D[k] / sigma
            assert np.allclose(got, want, rtol=1e-9, atol=1e-12), k
        else:
            assert np.all(got == 0.0), k
    assert np.allclose(F[:, 45], np.log10(sigma))


def test_features_invariant_under_rescaling_and_shift():
    mesh = synth.quad_mesh(7, 6)
    sp = build_space(mesh, 3, 1)
    s = synth.random_nodal((sp.E, sp.ref.n_loc), 5)
    c = vertex_candidates(sp, s, synth.Params())
    F = features(sp, s, c, sigma_ref=2.0)
    s2 = 3.5 * s - 1.25
    c2 = vertex_candidates(sp, s2, synth.Params())
    F2 = features(sp, s2, c2, sigma_ref=7.0)
    assert np.allclose(F, F2, rtol=1e-9, atol=1e-9)


def test_feature_slot_positions():
    """A perturbation of one candidate entry shows up in the slots of exactly
    the cells and local vertices that share that vertex, scaled by h^|k|/sigma."""
    mesh = synth.quad_mesh(5, 4)
    sp = build_space(mesh, 2, 1)
    s = synth.random_nodal((sp.E, sp.ref.n_loc), 7)
    H = hermite_at_vertices(sp, s)
    c = np.zeros((mesh.n_vertices, len(sp.ks)))
    for e in range(sp.E):
        for l in range(4):
            c[mesh.cell_vertices[e, l]] = H[e, l]          # candidates with no mismatch (last writer)
    F0 = features(sp, s, c, 1.0)
    v, t, delta = 7, 3, 0.01                                 # vertex 7, multi-index (1,1)
    c2 = c.copy()
    c2[v, t] += delta
    F1 = features(sp, s, c2, 1.0)
    sigma = cell_seminorm(sp, s) + 1e-12
    diff = F1 - F0
    k = sp.ks[t]
    slot = SLOTS.index(k)
    for e in range(sp.E):
        for l in range(4):
            want = (sp.h[e] ** sum(k) * delta / sigma[e]) if mesh.cell_vertices[e, l] == v else 0.0
            assert abs(diff[e, 9 * l + slot] - want) <= 1e-12 * max(1.0, abs(want))
    others = np.delete(np.arange(36), [9 * l + slot for l in range(4)])
    assert np.abs(diff[:, others]).max() < 1e-12
    assert np.abs(diff[:, 36:46]).max() < 1e-12
