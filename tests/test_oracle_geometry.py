"""Pins of the oracle's physical derivatives D^k u: exact on polynomial data the
space reproduces, and equal to finite differences through the inverse
bilinear map where the data is not polynomial."""
import math

import numpy as np
import pytest

import synth
from oracle import build_space
from oracle.basis import multi_indices
from oracle.geometry import physical_derivatives, map_points


def _poly(coefs, x, y, k=(0, 0)):
    """Value of D^k of sum c_ab x^a y^b."""
    out = np.zeros_like(x)
    for (a, b), c in coefs.items():
        if a < k[0] or b < k[1]:
            continue
        fa = math.factorial(a) // math.factorial(a - k[0])
        fb = math.factorial(b) // math.factorial(b - k[1])
        out = out + c * fa * fb * x ** (a - k[0]) * y ** (b - k[1])
    return out


def _rand_poly(deg, seed):
    rng = np.random.default_rng(seed)
    return {(a, n - a): rng.normal() for n in range(deg + 1) for a in range(n + 1)}


@pytest.mark.parametrize("cell,p,kind,jit", [
    (synth.TRI, 3, 1, 0.1), (synth.TRI, 2, 1, 0.1), (synth.QUAD, 3, 1, 0.0),
    (synth.QUAD, 2, 0, 0.1), (synth.QUAD, 2, 1, 0.1), (synth.QUAD, 1, 0, 0.1)])
def test_derivatives_exact_on_reproduced_polynomials(cell, p, kind, jit):
    mk = synth.tri_mesh if cell == synth.TRI else synth.quad_mesh
    mesh = mk(4, 4, jitter=jit, seed=7, periodic=(False, False))
    sp = build_space(mesh, p, kind)
    coefs = _rand_poly(p, 11)
    xn = sp.node_coords()
    u = _poly(coefs, xn[..., 0], xn[..., 1])
    pts = np.concatenate([sp.ref.vertices, sp.ref.vol_pts, sp.ref.norm_pts])
    D = physical_derivatives(sp.ref, sp.cell, sp.X, u, pts, multi_indices(2, p))
    xp = map_points(sp.cell, sp.X, pts)
    for k, val in D.items():
        ex = _poly(coefs, xp[..., 0], xp[..., 1], k)
        assert np.abs(val - ex).max() < 1e-9 * (1 + np.abs(ex).max()), k


def _invert_bilinear(X, x, y):
    """Newton inversion of the bilinear map of one cell (independent of the oracle's Jacobian code)."""
    xi = np.zeros(2)
    s = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], float)
    for _ in range(50):
        N = 0.25 * (1 + s[:, 0] * xi[0]) * (1 + s[:, 1] * xi[1])
        r = N @ X - np.array([x, y])
        dN = np.stack([0.25 * s[:, 0] * (1 + s[:, 1] * xi[1]), 0.25 * s[:, 1] * (1 + s[:, 0] * xi[0])], 1)
        Jm = X.T @ dN
        xi = xi - np.linalg.solve(Jm, r)
    return xi


def test_bilinear_second_derivatives_match_finite_differences():
    mesh = synth.quad_mesh(3, 3, jitter=0.2, seed=3, periodic=(False, False))
    sp = build_space(mesh, 2, 0)
    rng = np.random.default_rng(5)
    u = rng.normal(size=(sp.E, sp.ref.n_loc))          # arbitrary Q2 data: not polynomial in x
    e = 4
    Xe = sp.X[e]
    pt = np.array([[0.3, -0.2]])
    D = physical_derivatives(sp.ref, sp.cell, sp.X[e:e + 1], u[e:e + 1], pt, multi_indices(2, 2))
    x0 = map_points(sp.cell, sp.X[e:e + 1], pt)[0, 0]

    def f(x, y):
        xi = _invert_bilinear(Xe, x, y)
        return float(sp.ref.deriv(xi[None], (0, 0))[0] @ u[e])

    hh = 1e-3
    fd = {
        (1, 0): (f(x0[0] + hh, x0[1]) - f(x0[0] - hh, x0[1])) / (2 * hh),
        (0, 1): (f(x0[0], x0[1] + hh) - f(x0[0], x0[1] - hh)) / (2 * hh),
        (2, 0): (f(x0[0] + hh, x0[1]) - 2 * f(*x0) + f(x0[0] - hh, x0[1])) / hh ** 2,
        (0, 2): (f(x0[0], x0[1] + hh) - 2 * f(*x0) + f(x0[0], x0[1] - hh)) / hh ** 2,
        (1, 1): (f(x0[0] + hh, x0[1] + hh) - f(x0[0] + hh, x0[1] - hh)
                 - f(x0[0] - hh, x0[1] + hh) + f(x0[0] - hh, x0[1] - hh)) / (4 * hh * hh),
    }
    for k, v in fd.items():
        assert abs(D[k][0, 0] - v) < 1e-4 * (1 + abs(v)), (k, D[k][0, 0], v)
