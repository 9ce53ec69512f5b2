"""Pins of the oracle's HWENO limiter (Sec. 3: the cell-vertex reconstruction
overwrites u_h^e by u_h^{e,*}; Sec. 3.2: vertex candidates with corrected
cell averages).

* exact symbolic brute force (SymPy polynomials, exact cell integrals) of the
  reconstructed nodal values on a periodic 3 x 3 quad mesh, DG Q1..Q3;
* the corrected candidates preserve every cell average (conservation);
* polynomial data of the element degree and constant data are reproduced;
* the threshold selects the overwritten cells.
"""
import numpy as np
import pytest
import sympy as symp

import synth
from synth import Params
from oracle import build_space, nodal_interpolate, hweno_limit
from oracle.method import sensor_gamma
from tests.parity_helpers import rough_scalar, euler_state
from tests.test_oracle_sensor import _sympy_sensor, _sympy_tri_case, _lagrange_1d_sym, _box_integral, _R, xs, ys


def _cell_means(sp, u):
    from oracle.geometry import map_jacobian
    pts = sp.ref.norm_pts
    J, _ = map_jacobian(sp.cell, sp.X, pts)
    W = sp.ref.norm_w[None, :] * np.abs(np.linalg.det(J))
    return (W * (u @ sp.ref.deriv(pts, (0, 0)).T)).sum(1) / W.sum(1)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_sympy_brute_force_limiter(p):
    mesh = synth.quad_mesh(3, 3, periodic=(True, True))
    prm = Params()
    sp = build_space(mesh, p, 1)
    n1 = p + 1
    rng = np.random.default_rng(40 + p)
    u = rng.integers(-2, 3, size=(sp.E, n1 * n1)) / 8.0
    u[4, :] += 3.0
    u[4, 0] -= 6.0
    L = _lagrange_1d_sym([_R(x) for x in sp.ref.x1d])
    polys, boxes = [], []
    for e in range(sp.E):
        x0, x1 = _R(mesh.cell_coords[e, 0, 0]), _R(mesh.cell_coords[e, 1, 0])
        y0, y1 = _R(mesh.cell_coords[e, 0, 1]), _R(mesh.cell_coords[e, 3, 1])
        xi = 2 * (xs - (x0 + x1) / 2) / (x1 - x0)
        eta = 2 * (ys - (y0 + y1) / 2) / (y1 - y0)
        polys.append(symp.Poly(sum(_R(u[e, a + n1 * b]) * L[a](xi) * L[b](eta)
                                   for a in range(n1) for b in range(n1)), xs, ys))
        boxes.append((x0, x1, y0, y1))
    integ = lambda e, f: _box_integral(f, *boxes[e])
    _, _, oms, cls = _sympy_sensor(mesh, polys, p, integ, prm, parts=True)
    xn = sp.node_coords()
    ref = np.zeros_like(u)
    for e in range(sp.E):
        x0, x1, y0, y1 = boxes[e]
        area = (x1 - x0) * (y1 - y0)
        mean_u = integ(e, polys[e]) / area
        rec = polys[e] * _R(oms[e][0])
        for l, cl in enumerate(cls[e]):
            ubar = cl + symp.Poly(mean_u - integ(e, cl) / area, xs, ys)
            rec = rec + ubar * _R(oms[e][l + 1])
        for j in range(n1 * n1):
            ref[e, j] = float(rec.eval({xs: _R(xn[e, j, 0]), ys: _R(xn[e, j, 1])}))
    got = hweno_limit(sp, u, prm, threshold=2.0)
    assert np.abs(got - ref).max() < 1e-10 * (1 + np.abs(ref).max())
    assert np.abs(got - u).max() > 0.1                     # the limiter acts on this data


@pytest.mark.parametrize("p", [1, 2, 3])
def test_limiter_preserves_cell_averages(p):
    mesh = synth.quad_mesh(12, 10, jitter=0.0)
    sp = build_space(mesh, p, 1)
    u = rough_scalar(sp, 5)
    out = hweno_limit(sp, u, Params(), threshold=2.0)
    m0, m1 = _cell_means(sp, u), _cell_means(sp, out)
    assert np.abs(m1 - m0).max() < 1e-13 * np.abs(u).max()
    assert np.abs(out - u).max() > 1e-2


def test_limiter_preserves_cell_averages_euler():
    mesh = synth.quad_mesh(10, 9)
    sp = build_space(mesh, 3, 1, 4)
    U = sp.to_cells(euler_state(sp, k=200.0))
    out = hweno_limit(sp, U, Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0)), threshold=2.0)
    for v in range(4):
        assert np.abs(_cell_means(sp, out[v]) - _cell_means(sp, U[v])).max() < 1e-13 * np.abs(U[v]).max()


@pytest.mark.parametrize("p", [1, 2, 3])
def test_limiter_reproduces_polynomials(p):
    """Global polynomials of degree p: every candidate is the polynomial itself,
    so u_h^{e,*} = u_h^e on every cell (non-periodic mesh: no seam jump)."""
    mesh = synth.quad_mesh(9, 8, periodic=(False, False))
    sp = build_space(mesh, p, 1)
    rng = np.random.default_rng(p)
    coef = {(a, b): rng.normal() for a in range(p + 1) for b in range(p + 1 - a)}
    f = lambda x: sum(c * (x[..., 0] - 0.3) ** a * (x[..., 1] - 0.6) ** b for (a, b), c in coef.items())
    u = sp.to_cells(nodal_interpolate(sp, [f]))[0]
    out = hweno_limit(sp, u, Params(), threshold=2.0)
    assert np.abs(out - u).max() < 1e-10 * np.abs(u).max()
    const = np.full_like(u, 2.5)
    assert np.abs(hweno_limit(sp, const, Params(), threshold=2.0) - 2.5).max() < 1e-13


def test_limiter_threshold_selects_cells():
    mesh = synth.quad_mesh(13, 11)
    sp = build_space(mesh, 2, 1)
    u = rough_scalar(sp, 2)
    prm = Params()
    g = sensor_gamma(sp, u, prm)
    assert (g < 0.9).sum() >= 3 and (g >= 0.9).sum() >= 3
    assert np.array_equal(hweno_limit(sp, u, prm, threshold=0.0), u)
    out = hweno_limit(sp, u, prm, threshold=0.9)
    changed = np.abs(out - u).max(1) > 0
    assert not changed[g >= 0.9].any()
    assert changed[g < 0.9].all()
    full = hweno_limit(sp, u, prm, threshold=2.0)
    assert np.array_equal(out[g < 0.9], full[g < 0.9])


@pytest.mark.parametrize("p", [1, 2, 3])
def test_limiter_triangles_preserves_averages(p):
    """Jittered periodic triangles: the same construction (Taylor polynomials
    about the vertices, corrected averages, the sensor's weights)."""
    mesh = synth.tri_mesh(7, 6, jitter=0.1, seed=p)
    sp = build_space(mesh, p, 1)
    u = rough_scalar(sp, 4)
    out = hweno_limit(sp, u, Params(), threshold=2.0)
    m0, m1 = _cell_means_tri(sp, u), _cell_means_tri(sp, out)
    assert np.abs(m1 - m0).max() < 1e-13 * np.abs(u).max()
    assert np.abs(out - u).max() > 1e-2


@pytest.mark.parametrize("p", [1, 2, 3])
def test_limiter_triangles_reproduce_polynomials(p):
    mesh = synth.tri_mesh(6, 5, jitter=0.1, seed=7 + p, periodic=(False, False))
    sp = build_space(mesh, p, 1)
    rng = np.random.default_rng(10 + p)
    coef = {(a, b): rng.normal() for a in range(p + 1) for b in range(p + 1 - a)}
    f = lambda x: sum(c * (x[..., 0] - 0.4) ** a * (x[..., 1] - 0.7) ** b for (a, b), c in coef.items())
    u = sp.to_cells(nodal_interpolate(sp, [f]))[0]
    out = hweno_limit(sp, u, Params(), threshold=2.0)
    assert np.abs(out - u).max() < 1e-10 * np.abs(u).max()


def _cell_means_tri(sp, u):
    from oracle.geometry import map_jacobian
    pts = sp.ref.vol_pts
    J, _ = map_jacobian(sp.cell, sp.X, pts)
    W = sp.ref.vol_w[None, :] * np.abs(np.linalg.det(J))
    return (W * (u @ sp.ref.deriv(pts, (0, 0)).T)).sum(1) / W.sum(1)


def test_sympy_brute_force_limiter_triangles_p2():
    """Jittered periodic triangles, P2: the reconstructed nodal values with
    exact polynomials and exact cell integrals."""
    mesh, sp, u, polys, integ, prm, p = _sympy_tri_case()
    _, _, oms, cls = _sympy_sensor(mesh, polys, p, integ, prm, parts=True)
    xn = sp.node_coords()
    ref = np.zeros_like(u)
    one = symp.Poly(1, xs, ys)
    for e in range(sp.E):
        area = integ(e, one)
        mean_u = integ(e, polys[e]) / area
        rec = polys[e] * _R(oms[e][0])
        for l, cl in enumerate(cls[e]):
            rec = rec + (cl + symp.Poly(mean_u - integ(e, cl) / area, xs, ys)) * _R(oms[e][l + 1])
        for j in range(sp.ref.n_loc):
            ref[e, j] = float(rec.eval({xs: _R(xn[e, j, 0]), ys: _R(xn[e, j, 1])}))
    got = hweno_limit(sp, u, prm, threshold=2.0)
    assert np.abs(got - ref).max() < 1e-9 * (1 + np.abs(ref).max())
    assert np.abs(got - u).max() > 1e-2
