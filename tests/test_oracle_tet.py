"""Pins of the oracle on tetrahedra (DG P_p on the six-tetrahedra split of
boxes; the vertex-based candidates of a tetrahedron, four per cell, Sec. 3.2).

* the reference element: Kronecker property, exact derivatives of its
  monomials, the volume rule exact for total degree 2p + 1, faces on the
  faces;
* the mesh: positive volumes filling the box, conforming faces, closed cell
  surfaces, 24 cells at every vertex;
* exact symbolic brute force of the vertex candidates and the sensor (SymPy:
  symbolic Lagrange basis, derivatives and integrals over the tetrahedra);
* invariants: constant states, polynomials of the element degree (gamma_e = 1
  with complete and incomplete patches), conservation with the sensor and the
  shock-capturing weights active, the DG operator exact on polynomial data
  of the element degree;
* the closed form of the element semi-norm of a polynomial of degree <= 2
  (volume and central second moments of the cell) that the GPU sensor pass
  evaluates, against the oracle's volume-rule value.
"""
import math

import numpy as np
import pytest
import sympy as symp

import synth
from synth import Params
from oracle import build_space, residual, nodal_interpolate, apply_mass_inverse
from oracle.method import vertex_candidates, cell_sensor, face_geometry
from oracle.basis import multi_indices, RefTet


@pytest.mark.parametrize("p", [1, 2, 3])
def test_reftet_basics(p):
    ref = RefTet(p)
    assert ref.n_loc == (p + 1) * (p + 2) * (p + 3) // 6
    assert np.allclose(ref.deriv(ref.nodes, (0, 0, 0)), np.eye(ref.n_loc), atol=1e-12)
    rng = np.random.default_rng(p)
    pts = rng.dirichlet(np.ones(4), size=6)[:, 1:]
    for a, b, c in [mono for mono in [(p, 0, 0), (0, 1, p - 1), (1, 1, p - 2)] if min(mono) >= 0]:
        vals = ref.nodes[:, 0] ** a * ref.nodes[:, 1] ** b * ref.nodes[:, 2] ** c
        for m in [(1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0)]:
            got = ref.deriv(pts, m) @ vals
            ex = (math.perm(a, m[0]) * math.perm(b, m[1]) * math.perm(c, m[2])
                  * pts[:, 0] ** max(a - m[0], 0) * pts[:, 1] ** max(b - m[1], 0) * pts[:, 2] ** max(c - m[2], 0))
            assert np.allclose(got, ex, atol=1e-10)
    q, w = ref.vol_pts, ref.vol_w
    for a, b, c in [(0, 0, 0), (2 * p + 1, 0, 0), (p, 0, p + 1), (p, 1, p)]:
        ex = math.factorial(a) * math.factorial(b) * math.factorial(c) / math.factorial(a + b + c + 3)
        assert np.isclose((w * q[:, 0] ** a * q[:, 1] ** b * q[:, 2] ** c).sum(), ex, rtol=1e-12)
    for f in range(4):
        pf, wf = ref.face_points(f)
        bary = np.concatenate([1.0 - pf.sum(1, keepdims=True), pf], axis=1)
        assert np.abs(bary[:, f]).max() < 1e-14 and np.delete(bary, f, axis=1).min() > 0
        assert np.isclose(wf.sum(), 0.5)


def test_tet_mesh_and_faces():
    nx, ny, nz = 3, 4, 3
    m = synth.tet_mesh(nx, ny, nz, x1=1.5, z1=0.6)
    sp = build_space(m, 1, 1)
    X = m.cell_coords
    vol = np.linalg.det(np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=-1)) / 6
    assert vol.min() > 0 and np.isclose(vol.sum(), 1.5 * 1.0 * 0.6)
    assert (sp.nbr >= 0).all()
    assert np.all(sp.nbr[sp.nbr, sp.nbr_face] == np.arange(sp.E)[:, None])
    assert set(np.diff(sp.patch_ptr)) == {24}
    # closed surface of every cell: sum over faces of n * area = 0; areas from the edges
    tot = np.zeros((sp.E, 3))
    for f in range(4):
        n, J = face_geometry(sp, f)
        assert np.allclose(np.linalg.norm(n, axis=1), 1.0)
        tot += n * (J / 2)[:, None]
        c = [i for i in range(4) if i != f]
        area = 0.5 * np.linalg.norm(np.cross(X[:, c[1]] - X[:, c[0]], X[:, c[2]] - X[:, c[0]]), axis=1)
        assert np.allclose(J / 2, area)
        # outward: the opposite vertex lies behind the face
        assert np.all(((X[:, f] - X[:, c[0]]) * n).sum(1) < 0)
    assert np.abs(tot).max() < 1e-14


# ---------------------------------------------------------------------------
# SymPy brute force
# ---------------------------------------------------------------------------
xs, ys, zs = symp.symbols("x y z", real=True)


def _R(v):
    return symp.Rational(float(v))


def _tet_basis_sym(p):
    """Lagrange basis of RefTet in the reference coordinates, exact rationals."""
    r, s, t = symp.symbols("r s t")
    nodes = []
    for k in range(p + 1):
        for j in range(p + 1 - k):
            for i in range(p + 1 - j - k):
                nodes.append((symp.Rational(i, p), symp.Rational(j, p), symp.Rational(k, p)))
    mono = [(a, b, n - a - b) for n in range(p + 1) for a in range(n, -1, -1) for b in range(n - a, -1, -1)]
    V = symp.Matrix([[x ** a * y ** b * z ** c for a, b, c in mono] for x, y, z in nodes])
    C = V.inv()
    return [sum(C[i, j] * r ** a * s ** b * t ** c for i, (a, b, c) in enumerate(mono)) for j in range(len(nodes))], (r, s, t)


def _tet_integral(f, X):
    """int over the tetrahedron X [4][3] (rationals) of the polynomial f(x, y, z)."""
    r, s, t = symp.symbols("r s t")
    J = symp.Matrix([[X[k][d] - X[0][d] for k in (1, 2, 3)] for d in range(3)])
    sub = {v: X[0][d] + J[d, 0] * r + J[d, 1] * s + J[d, 2] * t for d, v in enumerate((xs, ys, zs))}
    g = symp.Poly(symp.expand(f.as_expr().subs(sub)), r, s, t)
    tot = symp.Integer(0)
    for (a, b, c), co in g.terms():
        tot += co * symp.factorial(a) * symp.factorial(b) * symp.factorial(c) / symp.factorial(a + b + c + 3)
    return tot * abs(J.det())


def _sympy_sensor_tet(mesh, polys, p, prm):
    ks = multi_indices(3, p)
    E, ve = mesh.cell_vertices.shape
    Xr = [[[_R(mesh.cell_coords[e, v, d]) for d in range(3)] for v in range(ve)] for e in range(E)]
    h2 = [max(sum((a[d] - b[d]) ** 2 for d in range(3)) for a in Xr[e] for b in Xr[e]) for e in range(E)]

    def D(f, k):
        for sv, n in zip((xs, ys, zs), k):
            for _ in range(n):
                f = f.diff(sv)
        return f

    cand = {}
    for i in range(mesh.n_vertices):
        ents = [(e, lv) for e in range(E) for lv in range(ve) if mesh.cell_vertices[e, lv] == i]
        wts, hd = [], []
        for e, lv in ents:
            pt = {xs: Xr[e][lv][0], ys: Xr[e][lv][1], zs: Xr[e][lv][2]}
            vals = [D(polys[e], k).eval(pt) for k in ks]
            beta = math.sqrt(float(sum(h2[e] ** sum(k) * v ** 2 for k, v in zip(ks, vals))))
            wts.append(1 / (prm.eps_vertex + beta) ** 2)
            hd.append([float(v) for v in vals])
        tot = sum(wts)
        cand[i] = [sum(w * h[j] for w, h in zip(wts, hd)) / tot for j in range(len(ks))]

    def seminorm(e, f):
        return math.sqrt(sum(float(h2[e] ** sum(k) * _tet_integral(D(f, k) ** 2, Xr[e])) for k in ks)
                         / float(h2[e]) ** 1.5)

    gam = []
    for e in range(E):
        cl = []
        for lv in range(ve):
            x0 = Xr[e][lv]
            c = cand[int(mesh.cell_vertices[e, lv])]
            expr = sum(_R(cj) * (xs - x0[0]) ** k[0] * (ys - x0[1]) ** k[1] * (zs - x0[2]) ** k[2]
                       / (math.factorial(k[0]) * math.factorial(k[1]) * math.factorial(k[2])) for cj, k in zip(c, ks))
            cl.append(symp.Poly(expr, xs, ys, zs))
        betas = [seminorm(e, polys[e])] + [seminorm(e, s) for s in cl]
        lin = [1 - ve * prm.lin_w_vertex] + [prm.lin_w_vertex] * ve
        wt = [g / (prm.eps_cell + b) ** 2 for g, b in zip(lin, betas)]
        om = [w / sum(wt) for w in wt]
        diff = sum(((polys[e] - cl[l]) * _R(om[l + 1]) for l in range(ve)), symp.Poly(0, xs, ys, zs))
        n0, d = betas[0], seminorm(e, diff)
        gam.append(1.0 if n0 == 0 else 1.0 - min(1.0, d / n0))
    return np.array(gam), np.array([cand[i] for i in range(mesh.n_vertices)])


@pytest.mark.parametrize("p", [1, 2])
def test_sympy_brute_force_dg_tet(p):
    """2 x 2 x 2 open boxes split into 48 tetrahedra (incomplete patches at the
    boundary), rough data with a jump cell and a spike inside it."""
    mesh = synth.tet_mesh(2, 2, 2, x1=1.0, y1=0.75, z1=0.5, periodic=(False, False, False))
    prm = Params()
    sp = build_space(mesh, p, 1)
    rng = np.random.default_rng(50 + p)
    u = rng.integers(-2, 3, size=(sp.E, sp.ref.n_loc)) / 8.0
    u[17, :] += 3.0
    u[17, 0] -= 6.0
    basis, (r, s, t) = _tet_basis_sym(p)
    polys = []
    for e in range(sp.E):
        X = [[_R(mesh.cell_coords[e, v, d]) for d in range(3)] for v in range(4)]
        J = symp.Matrix([[X[k][d] - X[0][d] for k in (1, 2, 3)] for d in range(3)])
        loc = J.inv() * symp.Matrix([xs - X[0][0], ys - X[0][1], zs - X[0][2]])
        sub = {r: loc[0], s: loc[1], t: loc[2]}
        polys.append(symp.Poly(symp.expand(sum(_R(u[e, j]) * basis[j].subs(sub) for j in range(sp.ref.n_loc))),
                               xs, ys, zs))
    g_sym, c_sym = _sympy_sensor_tet(mesh, polys, p, prm)
    c = vertex_candidates(sp, u, prm)
    g = cell_sensor(sp, u, c, prm)
    assert np.abs(c - c_sym).max() < 1e-9 * (1 + np.abs(c_sym).max())
    assert np.abs(g - g_sym).max() < 1e-10
    assert g.min() < 0.9


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p", [1, 2])
def test_constant_state_and_polynomials(p):
    sp = build_space(synth.tet_mesh(3, 3, 3), p, 1)
    U = np.full(sp.state_size(), -0.4)
    R, parts = residual(sp, U, Params(flux=synth.BURGERS, flux_param=(1.0, 0.5, -0.3, 0)), return_parts=True)
    assert np.abs(R).max() < 1e-14 and np.all(parts["gamma"] == 1.0)
    so = build_space(synth.tet_mesh(2, 2, 2, periodic=(False, False, False)), p, 1)
    rng = np.random.default_rng(8)
    co = rng.normal(size=(len(multi_indices(3, p)),))
    poly = lambda x: 0.2 + sum(c * x[..., 0] ** k[0] * x[..., 1] ** k[1] * x[..., 2] ** k[2]
                               for c, k in zip(co, multi_indices(3, p)))
    u = nodal_interpolate(so, [poly]).reshape(so.E, -1)
    g = cell_sensor(so, u, vertex_candidates(so, u, Params()), Params())
    assert np.all(np.abs(g - 1.0) < 1e-9)
    u2 = nodal_interpolate(so, [lambda x: poly(x) + 3.0 * x[..., 1] ** (p + 1)]).reshape(so.E, -1)
    assert cell_sensor(so, u2, vertex_candidates(so, u2, Params()), Params()).min() < 1 - 1e-6


def test_conservation_with_the_sensor_active():
    sp = build_space(synth.tet_mesh(3, 3, 3), 2, 1)
    rng = np.random.default_rng(3)
    U = nodal_interpolate(sp, [lambda x: np.sin(2 * np.pi * x[..., 2]) + 2.0 * (np.abs(x[..., 0] - 0.45) < 0.2)])
    U = U + 0.01 * rng.normal(size=U.shape)
    R, parts = residual(sp, U, Params(flux=synth.BURGERS, flux_param=(0.6, 1.0, 0.3, 0)), return_parts=True)
    assert parts["gamma"].min() < 0.9 and (parts["alpha"] != 1).any()
    assert abs(R.sum()) < 1e-13 * np.abs(R).sum()


@pytest.mark.parametrize("p", [1, 2])
def test_dg_operator_exact_on_polynomials(p):
    """Data of degree p and a linear flux: -M^{-1} R(u_h) equals -v . grad u
    exactly (to rounding) on every cell whose four neighbours exist (gamma_e =
    1, boundary faces dropped): the neighbours' traces equal the cell's own,
    so a mis-paired face point, a wrong normal or face Jacobian breaks it."""
    m = synth.tet_mesh(4, 4, 4, periodic=(False, False, False))
    sp = build_space(m, p, 1)
    a = np.array([0.3, -0.7, 0.5])
    v = np.array([1.0, 0.6, -0.8])
    q = 0.4 if p == 2 else 0.0
    U = nodal_interpolate(sp, [lambda x: x @ a + q * x[..., 0] * x[..., 2]])
    prm = Params(flux=synth.ADVECT_CONST, flux_param=tuple(v) + (0,), sensor=2, fixed_gamma=1.0)
    dU = -apply_mass_inverse(sp, residual(sp, U, prm, allow_boundary=True)).reshape(sp.E, -1)
    inner = (sp.nbr >= 0).all(1)
    xn = sp.node_coords()
    ex = -(v @ a + q * (v[0] * xn[..., 2] + v[2] * xn[..., 0]))
    assert inner.sum() == 216
    assert np.abs(dU[inner] - ex[inner]).max() < 1e-11


@pytest.mark.parametrize("p", [1, 2])
def test_closed_form_seminorm(p):
    """The element semi-norm (eq. snorm, d = 3) of a polynomial of degree <= 2
    on an affine cell in closed form, the form the GPU sensor pass evaluates:
    with g the gradient at the centroid, H the (constant) Hessian and
    M = |K| / 20 sum_i y_i y_i^T the central second moments (y_i the vertices
    about the centroid), ||p||^2 = h^-1 (|K| |g|^2 + tr(M H H)) + h |K| sum_{|k|=2} H_k^2.
    Checked against the oracle's volume-rule value on every cell of a sheared,
    stretched six-tetrahedra mesh with random Taylor data."""
    from oracle.method import element_seminorm_sq, taylor_derivatives
    from oracle.geometry import map_jacobian, map_points
    m = synth.tet_mesh(2, 2, 2, periodic=(False, False, False))
    L = np.array([[1.3, 0.4, -0.2], [0.1, 0.8, 0.3], [0.0, -0.25, 1.1]])
    assert np.linalg.det(L) > 0
    m.cell_coords[...] = m.cell_coords @ L.T
    sp = build_space(m, p, 1)
    ref = sp.ref
    J, _ = map_jacobian(sp.cell, sp.X, ref.norm_pts)
    W = ref.norm_w[None, :] * np.abs(np.linalg.det(J))
    xq = map_points(sp.cell, sp.X, ref.norm_pts)
    rng = np.random.default_rng(21)
    coef = rng.normal(size=(sp.E, len(sp.ks)))
    x0 = sp.X[:, 1]                                   # expansion point: a vertex
    want = element_seminorm_sq(sp, taylor_derivatives(sp, coef, xq, x0), W)
    idx = {tuple(k): i for i, k in enumerate(sp.ks)}
    vol = W.sum(1)
    yc = sp.X - sp.X.mean(1, keepdims=True)
    M = vol[:, None, None] / 20.0 * np.einsum("eia,eib->eab", yc, yc)
    H = np.zeros((sp.E, 3, 3))
    if p == 2:
        for a in range(3):
            for b in range(3):
                k = [0, 0, 0]
                k[a] += 1
                k[b] += 1
                H[:, a, b] = coef[:, idx[tuple(k)]]
    g = np.stack([coef[:, idx[(1, 0, 0)]], coef[:, idx[(0, 1, 0)]], coef[:, idx[(0, 0, 1)]]], 1)
    g = g + np.einsum("eab,eb->ea", H, sp.X.mean(1) - x0)
    h = sp.h
    s1 = vol * (g * g).sum(1) + np.einsum("eab,ebc,eca->e", M, H, H)
    s2 = sum(H[:, a, b] ** 2 for a in range(3) for b in range(a, 3))
    got = s1 / h + h * vol * s2
    assert np.allclose(got, want, rtol=1e-12, atol=0.0)


def test_euler_constant_state_and_conservation():
    """The Euler equations on tetrahedra (the 3D flux and HLL speeds are
    pinned on hexahedra by the exact reduction to 2D): a constant state has
    zero residual; with a density jump the sensor and the SC weights are
    active and every variable's residual sums to zero on a periodic mesh."""
    sp = build_space(synth.tet_mesh(3, 3, 3), 2, 1, n_var=5)
    prm = Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0))
    c = [1.2, 0.3, -0.2, 0.1, 2.5]
    U = nodal_interpolate(sp, [lambda x, v=v: v + 0.0 * x[..., 0] for v in c])
    assert np.abs(residual(sp, U, prm)).max() < 1e-13
    rho = lambda x: 1.0 + 2.0 * (np.abs(x[..., 1] - 0.45) < 0.2) + 0.3 * np.sin(2 * np.pi * x[..., 0]) * np.cos(2 * np.pi * x[..., 2])
    U = nodal_interpolate(sp, [rho, lambda x: 0.3 * rho(x), lambda x: -0.2 * rho(x), lambda x: 0.1 * rho(x),
                               lambda x: 2.0 + 0.5 * np.cos(2 * np.pi * x[..., 0])])
    R, parts = residual(sp, U, prm, return_parts=True)
    assert parts["gamma"].min() < 0.9 and (parts["alpha"] != 1).any()
    R = R.reshape(5, -1)
    assert np.all(np.abs(R.sum(1)) < 1e-12 * np.abs(R).sum(1))
