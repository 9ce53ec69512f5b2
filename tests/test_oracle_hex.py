"""Pins of the oracle on hexahedra (DG Q_p on boxes; the vertex-based
candidates of a cube, eight per cell, Sec. 3.2).

* the reference element: Kronecker property, exact derivatives of the
  element's monomials, exact volume rule, faces on the faces;
* connectivity and face geometry of a structured mesh against hand values;
* exact symbolic brute force of the vertex candidates and the sensor (SymPy,
  3 x 3 x 3 periodic cells, p = 1, 2);
* data that does not depend on z reduces the 3D DG residual to the 2D one on
  the quadrilateral mesh of its x-y cross-section, exactly (up to rounding):
  the Galerkin and interface terms by the z-weights of the nodes, the
  stabilisation additionally by the ratio of the cell diameters (eq. lostab);
* the Euler equations: data independent of one axis with no momentum along
  it reduces to the 2D Euler residual on the cross-section (both in-plane
  pairs), constant states, conservation;
* invariants: constant states, polynomials of the element degree (gamma_e = 1
  with complete and incomplete vertex patches), conservation, and the
  consistency of the DG operator at order p on smooth periodic data.
"""
import math

import numpy as np
import pytest
import sympy as symp

import synth
from synth import Params
from oracle import build_space, residual, nodal_interpolate, apply_mass_inverse
from oracle.method import vertex_candidates, cell_sensor, face_geometry
from oracle.basis import multi_indices, RefHex


# ---------------------------------------------------------------------------
# reference element, connectivity, geometry
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p", [1, 2, 3])
def test_refhex_basics(p):
    ref = RefHex(p, "gauss")
    assert np.allclose(ref.deriv(ref.nodes, (0, 0, 0)), np.eye(ref.n_loc), atol=1e-13)
    rng = np.random.default_rng(p)
    pts = rng.uniform(-1, 1, size=(7, 3))
    # d^m of x^a y^b z^c (a, b, c <= p) from the interpolant of its nodal values
    for a, b, c in [(p, 0, 1), (1, p, p), (p, p, p)]:
        vals = ref.nodes[:, 0] ** a * ref.nodes[:, 1] ** b * ref.nodes[:, 2] ** c
        for m in [(1, 0, 0), (0, 1, 1), (1, 1, 1), (min(a, 2), 0, 0)]:
            got = ref.deriv(pts, m) @ vals
            ex = (math.perm(a, m[0]) * math.perm(b, m[1]) * math.perm(c, m[2])
                  * pts[:, 0] ** max(a - m[0], 0) * pts[:, 1] ** max(b - m[1], 0) * pts[:, 2] ** max(c - m[2], 0))
            assert np.allclose(got, ex, atol=1e-11)
    # volume rule: exact for degree 2p + 1 per direction, weights sum to 8
    q = ref.vol_pts
    assert np.isclose(ref.vol_w.sum(), 8.0)
    assert np.isclose((ref.vol_w * q[:, 0] ** (2 * p) * q[:, 2] ** 2).sum(), 2 / (2 * p + 1) * 2 * 2 / 3)
    # faces: points on the face, opposite faces share the tangential parametrisation
    for f in range(6):
        pf, wf = ref.face_points(f)
        assert np.all(pf[:, f // 2] == (1.0 if f % 2 else -1.0))
        assert np.isclose(wf.sum(), 4.0)
        if f % 2 == 0:
            pg, _ = ref.face_points(f + 1)
            t = [a for a in range(3) if a != f // 2]
            assert np.array_equal(pf[:, t], pg[:, t])


def test_multi_indices_3d():
    ks = multi_indices(3, 2)
    assert ks == [(1, 0, 0), (0, 1, 0), (0, 0, 1), (2, 0, 0), (1, 1, 0), (1, 0, 1), (0, 2, 0), (0, 1, 1), (0, 0, 2)]
    for p in (1, 2, 3):
        assert len(multi_indices(3, p)) == (p + 1) * (p + 2) * (p + 3) // 6 - 1


def test_hex_connectivity_and_faces():
    nx, ny, nz = 4, 3, 5
    m = synth.hex_mesh(nx, ny, nz, x1=2.0, z1=0.5)
    sp = build_space(m, 1, 1)
    assert np.all(np.diff(sp.patch_ptr) == 8)
    cid = lambda i, j, k: (i % nx) + nx * ((j % ny) + ny * (k % nz))
    for (i, j, k) in [(0, 0, 0), (3, 2, 4), (1, 1, 2)]:
        e = cid(i, j, k)
        want = [cid(i - 1, j, k), cid(i + 1, j, k), cid(i, j - 1, k), cid(i, j + 1, k), cid(i, j, k - 1), cid(i, j, k + 1)]
        assert list(sp.nbr[e]) == want
        assert list(sp.nbr_face[e]) == [1, 0, 3, 2, 5, 4]
    hx, hy, hz = 2.0 / nx, 1.0 / ny, 0.5 / nz
    for f, (nrm, area) in enumerate([((-1, 0, 0), hy * hz), ((1, 0, 0), hy * hz), ((0, -1, 0), hx * hz),
                                     ((0, 1, 0), hx * hz), ((0, 0, -1), hx * hy), ((0, 0, 1), hx * hy)]):
        n, J = face_geometry(sp, f)
        assert np.allclose(n, nrm) and np.allclose(J, area / 4)
    assert np.allclose(sp.h, math.sqrt(hx * hx + hy * hy + hz * hz))


# ---------------------------------------------------------------------------
# SymPy brute force of the candidates and the sensor
# ---------------------------------------------------------------------------
xs, ys, zs = symp.symbols("x y z", real=True)


def _R(v):
    return symp.Rational(float(v))


def _lagrange_sym(nodes):
    t = symp.Symbol("t")
    out = []
    for j, xj in enumerate(nodes):
        L = symp.Integer(1)
        for m, xm in enumerate(nodes):
            if m != j:
                L = L * (t - xm) / (xj - xm)
        out.append(symp.Lambda(t, symp.expand(L)))
    return out


def _box_int(f, box):
    (x0, x1), (y0, y1), (z0, z1) = box
    tot = symp.Integer(0)
    for (a, b, c), co in f.terms():
        tot += (co * (x1 ** (a + 1) - x0 ** (a + 1)) / (a + 1) * (y1 ** (b + 1) - y0 ** (b + 1)) / (b + 1)
                * (z1 ** (c + 1) - z0 ** (c + 1)) / (c + 1))
    return tot


def _sympy_sensor_3d(mesh, polys, boxes, p, prm):
    ks = multi_indices(3, p)
    E, ve = mesh.cell_vertices.shape
    X = mesh.cell_coords
    h2 = [sum((b[1] - b[0]) ** 2 for b in boxes[e]) for e in range(E)]       # diam^2 of a box

    def D(f, k):
        for s, n in zip((xs, ys, zs), k):
            for _ in range(n):
                f = f.diff(s)
        return f

    cand = {}
    for i in range(mesh.n_vertices):
        ents = [(e, lv) for e in range(E) for lv in range(ve) if mesh.cell_vertices[e, lv] == i]
        wts, hd = [], []
        for e, lv in ents:
            pt = {xs: _R(X[e, lv, 0]), ys: _R(X[e, lv, 1]), zs: _R(X[e, lv, 2])}
            vals = [D(polys[e], k).eval(pt) for k in ks]
            beta = math.sqrt(float(sum(h2[e] ** sum(k) * v ** 2 for k, v in zip(ks, vals))))
            wts.append(1 / (prm.eps_vertex + beta) ** 2)
            hd.append([float(v) for v in vals])
        tot = sum(wts)
        cand[i] = [sum(w * h[j] for w, h in zip(wts, hd)) / tot for j in range(len(ks))]

    def seminorm(e, f):
        # sum_k h_e^{2|k| - 3} int |D^k f|^2, h_e^2 exact, h_e^{-3} in floating point
        return math.sqrt(sum(float(h2[e] ** sum(k) * _box_int(D(f, k) ** 2, boxes[e])) for k in ks)
                         / float(h2[e]) ** 1.5)

    gam = []
    for e in range(E):
        cl = []
        for lv in range(ve):
            x0 = [_R(X[e, lv, a]) for a in range(3)]
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
def test_sympy_brute_force_dg_hex(p):
    """3 x 3 x 3 periodic boxes (unequal sides), DG Q_p at the Gauss nodes
    (entering as the exact rationals of their float64 values), rough data with
    a jump cell and a spike inside it."""
    mesh = synth.hex_mesh(3, 3, 3, x1=1.5, z1=0.75)
    prm = Params()
    sp = build_space(mesh, p, 1)
    n1 = p + 1
    rng = np.random.default_rng(40 + p)
    u = rng.integers(-2, 3, size=(sp.E, n1 ** 3)) / 8.0
    u[13, :] += 3.0
    u[13, 0] -= 6.0
    L = _lagrange_sym([_R(x) for x in sp.ref.x1d])
    polys, boxes = [], []
    for e in range(sp.E):
        X = mesh.cell_coords[e]
        box = [(_R(X[0, a]), _R(X[6, a])) for a in range(3)]
        loc = [2 * (s - (b0 + b1) / 2) / (b1 - b0) for s, (b0, b1) in zip((xs, ys, zs), box)]
        polys.append(symp.Poly(sum(_R(u[e, a + n1 * b + n1 * n1 * c]) * L[a](loc[0]) * L[b](loc[1]) * L[c](loc[2])
                                   for a in range(n1) for b in range(n1) for c in range(n1)), xs, ys, zs))
        boxes.append(box)
    g_sym, c_sym = _sympy_sensor_3d(mesh, polys, boxes, p, prm)
    c = vertex_candidates(sp, u, prm)
    g = cell_sensor(sp, u, c, prm)
    assert np.abs(c - c_sym).max() < 1e-9 * (1 + np.abs(c_sym).max())
    assert np.abs(g - g_sym).max() < 1e-10
    assert g.min() < 0.9


# ---------------------------------------------------------------------------
# reduction to 2D
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("flux,fp", [(synth.ADVECT_CONST, (1.0, -0.6, 0.8, 0)), (synth.BURGERS, (1.0, 0.7, -0.4, 0))])
@pytest.mark.parametrize("p", [1, 2])
def test_z_independent_data_reduces_to_2d(flux, fp, p):
    nx, ny, nz = 4, 3, 3
    m3 = synth.hex_mesh(nx, ny, nz, x1=1.0, y1=0.75, z1=0.6)
    m2 = synth.quad_mesh(nx, ny, x1=1.0, y1=0.75)
    s3, s2 = build_space(m3, p, 1), build_space(m2, p, 1)
    g = lambda x: np.sin(2 * np.pi * x[..., 0]) + 0.7 * np.cos(2 * np.pi * x[..., 1] / 0.75) + 1.5 * (x[..., 0] > 0.5)
    U3 = nodal_interpolate(s3, [g])
    U2 = nodal_interpolate(s2, [g])
    pr = dict(flux=flux, flux_param=fp, sensor=2, sc_on=0)
    R3 = residual(s3, U3, Params(**pr, fixed_gamma=0.4)).reshape(s3.E, -1)
    R2g = residual(s2, U2, Params(**pr, fixed_gamma=1.0)).reshape(s2.E, -1)
    R2 = residual(s2, U2, Params(**pr, fixed_gamma=0.4)).reshape(s2.E, -1)
    stab = R2 - R2g
    n1 = p + 1
    w1 = np.polynomial.legendre.leggauss(n1)[1]
    hz = 0.6 / nz
    # nu_e = lambda_e h_e / (2p): the wave speed and the diameter of the box against the rectangle's
    scale = (np.linalg.norm(fp[:3]) * s3.h[0]) / (np.linalg.norm(fp[:2]) * s2.h[0])
    for e in range(s3.E):
        e2 = e % (nx * ny)
        for c in range(n1):
            blk = R3[e, c * n1 * n1:(c + 1) * n1 * n1]
            want = (R2g[e2] + scale * stab[e2]) * w1[c] * hz / 2
            assert np.abs(blk - want).max() <= 1e-12 * np.abs(R2).max(), (e, c)
    assert np.abs(stab).max() > 1e-3 * np.abs(R2).max()


def _euler_fields(a2):
    """rho, the two in-plane velocities and p of a smooth state with a density
    jump, as functions of the two in-plane coordinates (x, w) of axis a2."""
    L = {1: 0.75, 2: 0.6}[a2]
    rho = lambda x: 1.0 + 0.3 * np.sin(2 * np.pi * x[..., 0]) + 0.2 * np.cos(2 * np.pi * x[..., a2] / L) \
        + 0.5 * (x[..., 0] > 0.5)
    u = lambda x: 0.4 * np.cos(2 * np.pi * x[..., a2] / L)
    w = lambda x: 0.3 * np.sin(2 * np.pi * x[..., 0])
    pr = lambda x: 1.0 + 0.2 * np.sin(2 * np.pi * (x[..., 0] + x[..., a2] / L))
    return rho, u, w, pr


@pytest.mark.parametrize("kept", [1, 2])
@pytest.mark.parametrize("p", [1, 2])
def test_euler_reduces_to_2d(kept, p):
    """Euler data that does not depend on one axis, with no momentum along it:
    the 3D residual's density, energy and in-plane momenta are the 2D Euler
    residual on the cross-section (kept = 1: the x-y plane, z dropped; kept =
    2: the x-z plane, y dropped), weighted as for the scalar fluxes, and the
    dropped momentum's residual vanishes.  Pins where each flux component and
    the HLL wave speeds sit in 3D."""
    gam = 1.4
    nx, ny, nz = 4, 3, 3
    m3 = synth.hex_mesh(nx, ny, nz, x1=1.0, y1=0.75, z1=0.6)
    n2 = ny if kept == 1 else nz
    L2 = 0.75 if kept == 1 else 0.6
    m2 = synth.quad_mesh(nx, n2, x1=1.0, y1=L2)
    s3, s2 = build_space(m3, p, 1, n_var=5), build_space(m2, p, 1, n_var=4)
    rho, u, w, pr = _euler_fields(kept)
    En = lambda x: pr(x) / (gam - 1.0) + 0.5 * rho(x) * (u(x) ** 2 + w(x) ** 2)
    zero = lambda x: 0.0 * x[..., 0]
    m_u = lambda x: rho(x) * u(x)
    m_w = lambda x: rho(x) * w(x)
    if kept == 1:
        U3 = nodal_interpolate(s3, [rho, m_u, m_w, zero, En])
    else:
        U3 = nodal_interpolate(s3, [rho, m_u, zero, m_w, En])
    to2 = lambda f: (lambda x: f(np.stack([x[..., 0], x[..., 1], x[..., 1]], -1)))
    U2 = nodal_interpolate(s2, [to2(f) for f in (rho, m_u, m_w, En)])
    pp = dict(flux=synth.EULER, flux_param=(gam, 0, 0, 0), sensor=2, sc_on=0)
    R3 = residual(s3, U3, Params(**pp, fixed_gamma=0.4)).reshape(5, s3.E, -1)
    R2g = residual(s2, U2, Params(**pp, fixed_gamma=1.0)).reshape(4, s2.E, -1)
    R2 = residual(s2, U2, Params(**pp, fixed_gamma=0.4)).reshape(4, s2.E, -1)
    stab = R2 - R2g
    n1 = p + 1
    w1 = np.polynomial.legendre.leggauss(n1)[1]
    hd = (0.6 / nz) if kept == 1 else (0.75 / ny)      # side of the dropped axis
    scale = s3.h[0] / s2.h[0]                          # nu_e: the same wave speed, the box's diameter
    var3 = [0, 1, 2, 4] if kept == 1 else [0, 1, 3, 4]
    drop = 3 if kept == 1 else 2
    tol = 1e-12 * np.abs(R2).max()
    for e in range(s3.E):
        i, j, k = e % nx, (e // nx) % ny, e // (nx * ny)
        e2 = i + nx * (j if kept == 1 else k)
        blk = R3[:, e].reshape(5, n1, n1, n1)            # [v, c, b, a]
        for t in range(n1):
            got = blk[:, t] if kept == 1 else blk[:, :, t]   # the dropped axis' node index t
            want = (R2g[:, e2] + scale * stab[:, e2]).reshape(4, n1, n1) * w1[t] * hd / 2
            assert np.abs(got[var3] - want).max() <= tol, (e, t)
            assert np.abs(got[drop]).max() <= tol, (e, t)
    assert np.abs(stab).max() > 1e-3 * np.abs(R2).max()


def test_euler_constant_state_and_conservation():
    """A constant Euler state has zero residual; with a density jump the sensor
    and the SC weights are active and the residual sums to zero per variable
    on a periodic mesh."""
    gam = 1.4
    sp = build_space(synth.hex_mesh(3, 3, 3), 2, 1, n_var=5)
    c = [1.2, 0.3, -0.2, 0.1, 2.5]
    U = nodal_interpolate(sp, [lambda x, v=v: v + 0.0 * x[..., 0] for v in c])
    R = residual(sp, U, Params(flux=synth.EULER, flux_param=(gam, 0, 0, 0)))
    assert np.abs(R).max() < 1e-13
    rng = np.random.default_rng(4)
    rho = lambda x: 1.0 + 2.0 * (np.abs(x[..., 1] - 0.45) < 0.2) + 0.3 * np.sin(2 * np.pi * x[..., 0]) * np.cos(2 * np.pi * x[..., 2])
    U = nodal_interpolate(sp, [rho, lambda x: 0.3 * rho(x), lambda x: -0.2 * rho(x), lambda x: 0.1 * rho(x),
                               lambda x: 2.0 + 0.5 * np.cos(2 * np.pi * x[..., 0])])
    U = U + 0.002 * rng.normal(size=U.shape)
    R, parts = residual(sp, U, Params(flux=synth.EULER, flux_param=(gam, 0, 0, 0)), return_parts=True)
    assert parts["gamma"].min() < 0.9 and (parts["alpha"] != 1).any()
    R = R.reshape(5, -1)
    assert np.all(np.abs(R.sum(1)) < 1e-12 * np.abs(R).sum(1))


# ---------------------------------------------------------------------------
# invariants
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p", [1, 2])
def test_constant_state_and_polynomials(p):
    m = synth.hex_mesh(3, 4, 3)
    sp = build_space(m, p, 1)
    U = np.full(sp.state_size(), 0.37)
    R, parts = residual(sp, U, Params(flux=synth.BURGERS, flux_param=(1.0, 0.5, -0.3, 0)), return_parts=True)
    assert np.abs(R).max() < 1e-14 and np.all(parts["gamma"] == 1.0)
    # a polynomial of total degree p on an open mesh (incomplete patches at the boundary)
    mo = synth.hex_mesh(3, 3, 2, periodic=(False, False, False))
    so = build_space(mo, p, 1)
    rng = np.random.default_rng(5)
    co = rng.normal(size=(len(multi_indices(3, p)),))
    poly = lambda x: 0.3 + sum(c * x[..., 0] ** k[0] * x[..., 1] ** k[1] * x[..., 2] ** k[2]
                               for c, k in zip(co, multi_indices(3, p)))
    u = nodal_interpolate(so, [poly]).reshape(so.E, -1)
    c = vertex_candidates(so, u, Params())
    g = cell_sensor(so, u, c, Params())
    assert np.all(np.abs(g - 1.0) < 1e-9)
    # one degree more: not all cells smooth
    poly2 = lambda x: poly(x) + 4.0 * x[..., 0] ** (p + 1) * x[..., 2]
    u2 = nodal_interpolate(so, [poly2]).reshape(so.E, -1)
    assert cell_sensor(so, u2, vertex_candidates(so, u2, Params()), Params()).min() < 1 - 1e-6


def test_conservation_with_the_sensor_active():
    m = synth.hex_mesh(4, 3, 3)
    sp = build_space(m, 2, 1)
    rng = np.random.default_rng(9)
    U = nodal_interpolate(sp, [lambda x: np.sin(2 * np.pi * x[..., 0]) * np.cos(2 * np.pi * x[..., 2])
                               + 2.0 * (np.abs(x[..., 1] - 0.45) < 0.2)])
    U = U + 0.01 * rng.normal(size=U.shape)
    R, parts = residual(sp, U, Params(flux=synth.BURGERS, flux_param=(1.0, 0.5, 0.25, 0)), return_parts=True)
    assert parts["gamma"].min() < 0.9 and (parts["alpha"] != 1).any()
    assert abs(R.sum()) < 1e-13 * np.abs(R).sum()


@pytest.mark.parametrize("p,ns", [(1, (8, 12)), (2, (4, 8))])
def test_dg_operator_consistency_rate(p, ns):
    """-M^{-1} R(u_h) of smooth periodic data against -v . grad u at the nodes
    (gamma_e = 1: no stabilisation): the error falls like h^p (measured rates
    0.91 for p = 1 from 8 to 12 cells per direction, 2.3 for p = 2 from 4 to 8;
    a mis-paired or mis-oriented face leaves an error that does not fall)."""
    v = (1.0, 0.6, -0.8)
    f = lambda x: np.sin(2 * np.pi * x[..., 0]) * np.cos(2 * np.pi * (x[..., 1] + x[..., 2]))
    df = lambda x: (2 * np.pi * np.cos(2 * np.pi * x[..., 0]) * np.cos(2 * np.pi * (x[..., 1] + x[..., 2])) * v[0]
                    - 2 * np.pi * np.sin(2 * np.pi * x[..., 0]) * np.sin(2 * np.pi * (x[..., 1] + x[..., 2]))
                    * (v[1] + v[2]))
    errs = []
    for n in ns:
        sp = build_space(synth.hex_mesh(n, n, n), p, 1)
        U = nodal_interpolate(sp, [f])
        prm = Params(flux=synth.ADVECT_CONST, flux_param=v + (0,), sensor=2, fixed_gamma=1.0)
        dU = -apply_mass_inverse(sp, residual(sp, U, prm))
        ex = -df(sp.node_coords()).ravel()
        errs.append(np.abs(dU - ex).max() / np.abs(ex).max())
    rate = math.log(errs[0] / errs[1]) / math.log(ns[1] / ns[0])
    assert rate > p - 0.3, (errs, rate)
