"""Pins of the oracle's cell-vertex WENO reconstruction and sensor (Sec. 3.2, eq. gamma).

* exact symbolic brute force (SymPy: symbolic interpolants, derivatives and
  integrals, no quadrature and no basis tables) on tiny periodic meshes;
* a closed form for 1D P1, where every quantity reduces to cell slopes;
* invariants fixed by the paper: linear weights recovered and gamma_e = 1 on
  polynomial data of the element degree, equal vertex weights 1/|C(x_i)| on
  uniform meshes, convex weights, gamma_e in [0, 1].
"""
import math

import numpy as np
import pytest
import sympy as symp

import synth
from synth import Params
from oracle import build_space
from oracle.method import vertex_candidates, cell_sensor
from oracle.basis import multi_indices


# ---------------------------------------------------------------------------
# SymPy brute force
# ---------------------------------------------------------------------------
xs, ys = symp.symbols("x y", real=True)


def _R(v):
    return symp.Rational(float(v))


def _sympy_sensor(mesh, polys, p, integrate, prm, parts=False):
    """gamma_e and vertex candidates computed with exact rational polynomials
    (sympy Poly in x, y): symbolic derivatives, exact integrals; only the
    square roots and the weights are taken in floating point.  parts: also
    the per-cell weights omega_l^e and vertex candidate polynomials (without
    their constant terms)."""
    ks = multi_indices(2, p)
    E, ve = mesh.cell_vertices.shape
    X = mesh.cell_coords
    hs = []
    for e in range(E):
        pts = [(_R(X[e, a, 0]), _R(X[e, a, 1])) for a in range(ve)]
        hs.append(max(((a[0] - b[0]) ** 2 + (a[1] - b[1]) ** 2) for a in pts for b in pts))  # h_e^2

    def D(f, k):
        for _ in range(k[0]):
            f = f.diff(xs)
        for _ in range(k[1]):
            f = f.diff(ys)
        return f

    # vertex stage: loop over vertices, patch = cells containing the vertex
    cand = {}
    for i in range(mesh.n_vertices):
        ents = [(e, lv) for e in range(E) for lv in range(ve) if mesh.cell_vertices[e, lv] == i]
        wts, hd = [], []
        for e, lv in ents:
            xi, yi = _R(X[e, lv, 0]), _R(X[e, lv, 1])
            vals = [D(polys[e], k).eval({xs: xi, ys: yi}) for k in ks]
            beta = math.sqrt(float(sum(hs[e] ** sum(k) * v ** 2 for k, v in zip(ks, vals))))
            wts.append(1 / (prm.eps_vertex + beta) ** 2)
            hd.append([float(v) for v in vals])
        tot = sum(wts)
        cand[i] = [sum(w * h[j] for w, h in zip(wts, hd)) / tot for j in range(len(ks))]

    def seminorm(e, f):
        return math.sqrt(float(sum(hs[e] ** (sum(k) - 1) * integrate(e, D(f, k) ** 2) for k in ks)))

    gam, oms, cls = [], [], []
    for e in range(E):
        ue = polys[e]
        cl = []
        for lv in range(ve):
            xi, yi = _R(X[e, lv, 0]), _R(X[e, lv, 1])
            c = cand[int(mesh.cell_vertices[e, lv])]
            expr = sum(_R(cj) * (xs - xi) ** k[0] * (ys - yi) ** k[1]
                       / (math.factorial(k[0]) * math.factorial(k[1])) for cj, k in zip(c, ks))
            cl.append(symp.Poly(expr, xs, ys))
        betas = [seminorm(e, ue)] + [seminorm(e, s) for s in cl]
        lin = [1 - ve * prm.lin_w_vertex] + [prm.lin_w_vertex] * ve
        wt = [g / (prm.eps_cell + b) ** 2 for g, b in zip(lin, betas)]
        om = [w / sum(wt) for w in wt]
        diff = sum(((ue - cl[l]) * _R(om[l + 1]) for l in range(ve)), symp.Poly(0, xs, ys))
        n0, d = betas[0], seminorm(e, diff)
        gam.append(1.0 if n0 == 0 else 1.0 - min(1.0, d / n0))
        oms.append(om)
        cls.append(cl)
    if parts:
        return np.array(gam), np.array([cand[i] for i in range(mesh.n_vertices)]), oms, cls
    return np.array(gam), np.array([cand[i] for i in range(mesh.n_vertices)])


def _lagrange_1d_sym(nodes):
    t = symp.Symbol("t")
    out = []
    for j, xj in enumerate(nodes):
        L = symp.Integer(1)
        for m, xm in enumerate(nodes):
            if m != j:
                L = L * (t - xm) / (xj - xm)
        out.append(symp.Lambda(t, symp.expand(L)))
    return out


def _box_integral(f, x0, x1, y0, y1):
    tot = symp.Integer(0)
    for (a, b), c in f.terms():
        tot += c * (x1 ** (a + 1) - x0 ** (a + 1)) / (a + 1) * (y1 ** (b + 1) - y0 ** (b + 1)) / (b + 1)
    return tot


def test_sympy_brute_force_quads_q2():
    """Uniform periodic 3x3 quads, CG Q2 (Gauss-Lobatto nodes -1, 0, 1), rough continuous data."""
    mesh = synth.quad_mesh(3, 3, periodic=(True, True))
    prm = Params()
    p = 2
    sp = build_space(mesh, p, 0)
    rng = np.random.default_rng(21)
    ug = rng.integers(-1, 2, size=sp.n_dof) / 8.0
    ug[4] += 4.0                                      # a spike so that some cells are troubled
    u = sp.to_cells(ug)[0]
    L = _lagrange_1d_sym([symp.Integer(-1), symp.Integer(0), symp.Integer(1)])
    polys, boxes = [], []
    for e in range(sp.E):
        x0, x1 = _R(mesh.cell_coords[e, 0, 0]), _R(mesh.cell_coords[e, 1, 0])
        y0, y1 = _R(mesh.cell_coords[e, 0, 1]), _R(mesh.cell_coords[e, 3, 1])
        xi = 2 * (xs - (x0 + x1) / 2) / (x1 - x0)
        eta = 2 * (ys - (y0 + y1) / 2) / (y1 - y0)
        polys.append(symp.Poly(sum(_R(u[e, a + 3 * b]) * L[a](xi) * L[b](eta)
                                   for a in range(3) for b in range(3)), xs, ys))
        boxes.append((x0, x1, y0, y1))

    g_sym, c_sym = _sympy_sensor(mesh, polys, p, lambda e, f: _box_integral(f, *boxes[e]), prm)
    c = vertex_candidates(sp, u, prm)
    g = cell_sensor(sp, u, c, prm)
    assert np.abs(c - c_sym).max() < 1e-9 * (1 + np.abs(c_sym).max())
    assert np.abs(g - g_sym).max() < 1e-10
    assert g.min() < 0.9          # the data is rough enough to exercise the sensor


@pytest.mark.parametrize("p", [1, 3])
def test_sympy_brute_force_dg_quads(p):
    """Uniform periodic 3x3 quads, DG Q_p at the Gauss-Legendre nodes (the
    benchmark's element at p = 3), rough discontinuous data: the nodes enter
    as the exact rationals of their float64 values."""
    mesh = synth.quad_mesh(3, 3, periodic=(True, True))
    prm = Params()
    sp = build_space(mesh, p, 1)
    n1 = p + 1
    rng = np.random.default_rng(30 + p)
    u = rng.integers(-2, 3, size=(sp.E, n1 * n1)) / 8.0
    u[4, :] += 3.0                                   # a jump cell
    u[4, 0] -= 6.0                                   # and a spike inside it, so that the sensor is active
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
    g_sym, c_sym = _sympy_sensor(mesh, polys, p, lambda e, f: _box_integral(f, *boxes[e]), prm)
    c = vertex_candidates(sp, u, prm)
    g = cell_sensor(sp, u, c, prm)
    assert np.abs(c - c_sym).max() < 1e-9 * (1 + np.abs(c_sym).max())
    assert np.abs(g - g_sym).max() < 1e-10
    assert g.min() < 0.9


def _sympy_tri_case():
    """Jittered periodic 3 x 3 x 2 triangles, P2, rough data: the mesh, space,
    nodal data, exact polynomials and an exact cell integral."""
    mesh = synth.tri_mesh(3, 3, jitter=0.15, seed=8, periodic=(True, True))
    prm = Params()
    p = 2
    sp = build_space(mesh, p, 1)
    rng = np.random.default_rng(22)
    u = rng.integers(-1, 2, size=(sp.E, 6)) / 8.0
    u[4] += 4.0
    mono = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2)]
    polys, maps = [], []
    for e in range(sp.E):
        P = [(_R(mesh.cell_coords[e, v, 0]), _R(mesh.cell_coords[e, v, 1])) for v in range(3)]
        # equispaced P2 nodes in the oracle's order: (i/2, j/2), j outer, i inner
        nodes = []
        for j in range(3):
            for i in range(3 - j):
                s, t = symp.Rational(i, 2), symp.Rational(j, 2)
                nodes.append((P[0][0] + s * (P[1][0] - P[0][0]) + t * (P[2][0] - P[0][0]),
                              P[0][1] + s * (P[1][1] - P[0][1]) + t * (P[2][1] - P[0][1])))
        V = symp.Matrix([[nx ** m[0] * ny ** m[1] for m in mono] for (nx, ny) in nodes])
        coef = V.LUsolve(symp.Matrix([_R(v) for v in u[e]]))
        polys.append(symp.Poly(sum(cf * xs ** m[0] * ys ** m[1] for cf, m in zip(coef, mono)), xs, ys))
        maps.append(P)

    s_, t_ = symp.symbols("s t")

    def integ(e, f):
        P = maps[e]
        xm = P[0][0] + s_ * (P[1][0] - P[0][0]) + t_ * (P[2][0] - P[0][0])
        ym = P[0][1] + s_ * (P[1][1] - P[0][1]) + t_ * (P[2][1] - P[0][1])
        det = abs((P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[2][0] - P[0][0]) * (P[1][1] - P[0][1]))
        g = symp.Poly(f.as_expr().subs({xs: xm, ys: ym}, simultaneous=True), s_, t_)
        tot = symp.Integer(0)
        for (a, b), cf in g.terms():       # int_T s^a t^b = a! b! / (a + b + 2)!
            tot += cf * symp.factorial(a) * symp.factorial(b) / symp.factorial(a + b + 2)
        return det * tot

    return mesh, sp, u, polys, integ, prm, p


def test_sympy_brute_force_jittered_triangles_p2():
    mesh, sp, u, polys, integ, prm, p = _sympy_tri_case()
    g_sym, c_sym = _sympy_sensor(mesh, polys, p, integ, prm)
    c = vertex_candidates(sp, u, prm)
    g = cell_sensor(sp, u, c, prm)
    assert np.abs(c - c_sym).max() < 1e-8 * (1 + np.abs(c_sym).max())
    assert np.abs(g - g_sym).max() < 1e-9
    assert g.min() < 0.9


# ---------------------------------------------------------------------------
# 1D P1 closed form
# ---------------------------------------------------------------------------
def test_closed_form_1d_p1():
    E = 7
    h = 1.0 / E
    mesh = synth.segment_mesh(E)
    sp = build_space(mesh, 1, 0)
    rng = np.random.default_rng(3)
    u = rng.normal(size=E)                 # CG P1 nodal values at the vertices
    prm = Params()
    s = (np.roll(u, -1) - u) / h           # slope of cell e
    eps = 1e-6
    # vertex i is shared by cells i-1 and i
    w_left = (eps + h * np.abs(np.roll(s, 1))) ** -2
    w_right = (eps + h * np.abs(s)) ** -2
    c = (w_left * np.roll(s, 1) + w_right * s) / (w_left + w_right)
    cl, cr = c, np.roll(c, -1)             # candidates at the left / right vertex of cell e
    b = [h * np.abs(s), h * np.abs(cl), h * np.abs(cr)]
    lin = [1 - 2e-3, 1e-3, 1e-3]
    wt = [g / (eps + bb) ** 2 for g, bb in zip(lin, b)]
    tot = sum(wt)
    d = h * np.abs(wt[1] / tot * (s - cl) + wt[2] / tot * (s - cr))
    gamma_ref = 1 - np.minimum(1, d / (h * np.abs(s)))

    uc = sp.to_cells(u)[0]
    cand = vertex_candidates(sp, uc, prm)
    assert np.allclose(cand[:, 0], c, rtol=1e-12, atol=1e-12)
    g = cell_sensor(sp, uc, cand, prm)
    assert np.allclose(g, gamma_ref, rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("cell,p,kind,jit", [
    (synth.QUAD, 2, 0, 0.0), (synth.QUAD, 2, 0, 0.1), (synth.QUAD, 3, 1, 0.0),
    (synth.QUAD, 1, 1, 0.1), (synth.TRI, 3, 1, 0.1), (synth.TRI, 2, 1, 0.0), (synth.SEG, 3, 0, 0.0)])
def test_polynomial_recovery(cell, p, kind, jit):
    """Global P_p data: every candidate equals u_h^e, so omega_l = linear weights and gamma_e = 1."""
    if cell == synth.SEG:
        mesh = synth.segment_mesh(6, periodic=False)
    else:
        mk = synth.tri_mesh if cell == synth.TRI else synth.quad_mesh
        mesh = mk(5, 4, jitter=jit, seed=2, periodic=(False, False))
    sp = build_space(mesh, p, kind)
    rng = np.random.default_rng(p)
    xn = sp.node_coords()
    u = np.zeros(xn.shape[:2])
    for (a, b) in [(i, n - i) for n in range(p + 1) for i in range(n + 1)]:
        if sp.ref.dim == 1 and b:
            continue
        u += rng.normal() * xn[..., 0] ** a * (xn[..., 1] ** b if sp.ref.dim == 2 else 1.0)
    prm = Params()
    c, omega_v, H, beta = vertex_candidates(sp, u, prm, return_weights=True)
    # candidates equal the exact derivatives at each vertex, from any cell of the patch
    pc, plv = sp.patch_cell, sp.patch_lv
    row = np.repeat(np.arange(len(sp.patch_ptr) - 1), np.diff(sp.patch_ptr))
    assert np.abs(H[pc, plv] - c[row]).max() < 1e-8 * (1 + np.abs(c).max())
    g, parts = cell_sensor(sp, u, c, prm, return_parts=True)
    assert np.abs(g - 1).max() < 1e-8
    ve = mesh.cell_vertices.shape[1]
    lin = np.array([1 - ve * 1e-3] + [1e-3] * ve)
    assert np.abs(parts["omega"] - lin).max() < 1e-8
    if jit == 0.0:
        # uniform mesh: equal vertex weights 1 / |C(x_i)|
        assert np.abs(omega_v - 1.0 / np.diff(sp.patch_ptr)[row]).max() < 1e-8


@pytest.mark.parametrize("cell,p", [(synth.QUAD, 2), (synth.TRI, 3), (synth.SEG, 2)])
def test_convex_weights_and_range(cell, p):
    if cell == synth.SEG:
        mesh = synth.segment_mesh(9)
    else:
        mk = synth.tri_mesh if cell == synth.TRI else synth.quad_mesh
        mesh = mk(5, 5, jitter=0.1, seed=4)
    sp = build_space(mesh, p, 1)
    u = synth.random_nodal((sp.E, sp.ref.n_loc), 9)
    prm = Params()
    c, om, H, beta = vertex_candidates(sp, u, prm, return_weights=True)
    assert (om >= 0).all()
    sums = np.add.reduceat(om, sp.patch_ptr[:-1])
    assert np.allclose(sums, 1.0, atol=1e-14)
    g, parts = cell_sensor(sp, u, c, prm, return_parts=True)
    assert (parts["omega"] >= 0).all() and np.allclose(parts["omega"].sum(1), 1.0, atol=1e-14)
    assert (g >= 0).all() and (g <= 1).all()


def test_patch_sizes():
    """Candidate counts (Sec. 3.2 remark): 2 per 1D vertex, 4 per quad vertex, 6 per structured-triangle vertex."""
    for mesh, expect in [(synth.segment_mesh(5), 2), (synth.quad_mesh(4, 3), 4), (synth.tri_mesh(4, 3), 6)]:
        sp = build_space(mesh, 1, 1)
        assert (np.diff(sp.patch_ptr) == expect).all()
