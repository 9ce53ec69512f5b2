"""Closed-form pins of the oracle's interface terms, shock-capturing indicators
and wave speeds, computed in the tests from the definitions with the test's
own polynomials and Gauss rules (not through the oracle's bases or rules).

* DG interface pairing (Sec. 2.1, the DG form with an interface flux): for a
  global polynomial of degree p the traces agree on every face, so on every
  interior cell the DG residual of linear advection is the Galerkin
  projection of div f(u) and M^{-1} R equals v . grad u at the nodes.  A face
  trace of the neighbour taken at the wrong point breaks the equality.
* Preliminary SC weights (eq. alpha_prelim with the pointwise semi-norm of
  eq. pointsnorm): alpha~_q = (sum_k h_e^{2|k|} |D^k u(x_q)|^2)^{1/2}, h_e the
  cell diameter, written out for known quadratics; alpha_q of eq. alphaq from
  the test's own Gauss weights.
* Low-order viscosity (eq. lostab): nu_e = lambda_e h_e / (2p) with the Euler
  wave speed |v| + c of a constant cell state.
* The dissipation of the low-order term: with SC off,
  u . (R(gamma=0) - R(gamma=1)) = sum_e nu_e int_K |grad u_h|^2, integrated
  here from the analytic gradient of per-cell polynomials.
"""
import math

import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space, residual, apply_mass_inverse
from oracle.method import sc_weights, sensor_gamma


def _poly2d(rng, p):
    """A random polynomial of total degree p: value and gradient callables."""
    C = {(i, j): rng.uniform(-1, 1) for i in range(p + 1) for j in range(p + 1 - i)}

    def val(x, y):
        return sum(c * x ** i * y ** j for (i, j), c in C.items())

    def grad(x, y):
        gx = sum(c * i * x ** (i - 1) * y ** j for (i, j), c in C.items() if i > 0)
        gy = sum(c * j * x ** i * y ** (j - 1) for (i, j), c in C.items() if j > 0)
        return gx + 0 * x, gy + 0 * y
    return val, grad


@pytest.mark.parametrize("cell,p", [(synth.QUAD, 1), (synth.QUAD, 2), (synth.QUAD, 3),
                                    (synth.TRI, 1), (synth.TRI, 2), (synth.TRI, 3)])
def test_dg_interior_residual_of_global_polynomial(cell, p):
    rng = np.random.default_rng(10 + p)
    if cell == synth.QUAD:
        mesh = synth.quad_mesh(5, 4, 0.0, 1.25, 0.0, 0.8, periodic=(False, False))
    else:
        mesh = synth.tri_mesh(5, 4, 0.0, 1.0, 0.0, 1.0, jitter=0.12, seed=3, periodic=(False, False))
    sp = build_space(mesh, p, 1)
    val, grad = _poly2d(rng, p)
    xn = sp.node_coords()
    U = val(xn[..., 0], xn[..., 1]).ravel()
    v = (0.7, -0.4)
    prm = Params(flux=synth.ADVECT_CONST, flux_param=(v[0], v[1], 0, 0))
    R, parts = residual(sp, U, prm, return_parts=True, allow_boundary=True)
    assert parts["gamma"].min() > 1.0 - 1e-9         # a global polynomial is smooth
    L = apply_mass_inverse(sp, R).reshape(sp.E, -1)
    gx, gy = grad(xn[..., 0], xn[..., 1])
    want = v[0] * gx + v[1] * gy
    interior = (sp.nbr >= 0).all(axis=1)
    assert interior.sum() >= 6
    err = np.abs(L[interior] - want[interior]).max()
    assert err < 1e-11 * max(1.0, np.abs(want).max()), err


def test_pointwise_indicator_segment_p2():
    """1D DG P2, cells of length h = 0.25: alpha~_q = sqrt(h^2 u'(x_q)^2 + h^4 u''^2)."""
    E, h = 5, 0.25
    mesh = synth.segment_mesh(E, 0.0, E * h)
    sp = build_space(mesh, 2, 1)
    rng = np.random.default_rng(7)
    c1 = np.array([1.0, 1.2, 30.0, -1.0, 40.0]) + rng.uniform(-0.5, 0.5, E)
    c2, c0 = rng.uniform(-2, 2, E), rng.uniform(-1, 1, E)
    xc = (np.arange(E) + 0.5) * h
    xn = sp.node_coords()[..., 0]
    u = c0[:, None] + c1[:, None] * (xn - xc[:, None]) + c2[:, None] * (xn - xc[:, None]) ** 2
    gamma = sensor_gamma(sp, u, Params())
    assert (gamma < 0.9).sum() >= 2                   # kinks between the cells
    alpha, parts = sc_weights(sp, u, gamma, Params(), return_parts=True)
    g = np.sqrt(3.0 / 5.0)
    xi, wq = np.array([-g, 0.0, g]), np.array([5.0, 8.0, 5.0]) / 9.0
    xq = xc[:, None] + 0.5 * h * xi[None, :]
    d1 = c1[:, None] + 2 * c2[:, None] * (xq - xc[:, None])
    d2 = 2 * c2[:, None] + 0 * xq
    atil = np.sqrt(h ** 2 * d1 ** 2 + h ** 4 * d2 ** 2)
    assert np.allclose(parts["atil"], atil, rtol=1e-12, atol=0)
    # eq. alphaq on the active cells, with the test's own 3-point Gauss rule
    f = (1.0 - gamma)[:, None] * d1 ** 2
    W = wq[None, :] * 0.5 * h
    act = gamma < 0.9
    want = atil * ((W * f).sum(1) / (W * atil * f).sum(1))[:, None]
    assert np.allclose(alpha[act], want[act], rtol=1e-12, atol=0)
    assert (alpha[~act] == 1.0).all()


def test_pointwise_indicator_rectangle_q2():
    """2D DG Q2 on hx x hy rectangles (h_e = sqrt(hx^2 + hy^2)):
    alpha~_q = sqrt(h^2 |grad u|^2 + h^4 (u_xx^2 + u_xy^2 + u_yy^2)) at the Gauss points."""
    nx, ny, hx, hy = 4, 3, 0.3, 0.2
    mesh = synth.quad_mesh(nx, ny, 0.0, nx * hx, 0.0, ny * hy)
    sp = build_space(mesh, 2, 1)
    rng = np.random.default_rng(11)
    E = nx * ny
    A = rng.uniform(-2, 2, (E, 6))          # per-cell quadratic about the cell centre
    X = mesh.cell_coords
    xc, yc = X[:, :, 0].mean(1), X[:, :, 1].mean(1)

    def cellpoly(x, y):
        X_, Y_ = x - xc[:, None], y - yc[:, None]
        return (A[:, 0, None] * X_ + A[:, 1, None] * Y_ + A[:, 2, None] * X_ * X_ + A[:, 3, None] * X_ * Y_
                + A[:, 4, None] * Y_ * Y_ + 3.0 * (np.arange(E) % 2)[:, None])
    xn = sp.node_coords()
    u = cellpoly(xn[..., 0], xn[..., 1])
    gamma = sensor_gamma(sp, u, Params())
    _, parts = sc_weights(sp, u, gamma, Params(), return_parts=True)
    g = np.sqrt(3.0 / 5.0)
    xi = np.array([-g, 0.0, g])
    qx = np.tile(xi, 3)                      # x fastest, as the collocated nodes
    qy = np.repeat(xi, 3)
    Xq, Yq = 0.5 * hx * qx[None, :], 0.5 * hy * qy[None, :]
    ux = A[:, 0, None] + 2 * A[:, 2, None] * Xq + A[:, 3, None] * Yq
    uy = A[:, 1, None] + A[:, 3, None] * Xq + 2 * A[:, 4, None] * Yq
    he = math.hypot(hx, hy)
    sec = (2 * A[:, 2]) ** 2 + A[:, 3] ** 2 + (2 * A[:, 4]) ** 2
    atil = np.sqrt(he ** 2 * (ux ** 2 + uy ** 2) + he ** 4 * sec[:, None])
    # the oracle's quadrature points in its own order: match by position
    pts = sp.ref.vol_pts
    order = [int(np.argmin((qx - a) ** 2 + (qy - b) ** 2)) for a, b in pts]
    assert np.allclose(parts["atil"], atil[:, order], rtol=1e-12, atol=0)


def test_euler_viscosity_of_constant_cells():
    """eq. lostab: nu_e = (|v| + sqrt(gamma p / rho)) h_e / (2p) on cells holding
    constant states (DG Q2 on 3 x 3 squares of side 1/3)."""
    n, p, gas = 3, 2, 1.4
    mesh = synth.quad_mesh(n, n)
    sp = build_space(mesh, p, 1, 4)
    rng = np.random.default_rng(5)
    rho, pr = rng.uniform(0.2, 2.0, n * n), rng.uniform(0.1, 3.0, n * n)
    vx, vy = rng.uniform(-1, 1, n * n), rng.uniform(-1, 1, n * n)
    En = pr / (gas - 1) + 0.5 * rho * (vx ** 2 + vy ** 2)
    nl = (p + 1) ** 2
    U = np.stack([np.repeat(c[:, None], nl, axis=1) for c in (rho, rho * vx, rho * vy, En)]).ravel()
    _, parts = residual(sp, U, Params(flux=synth.EULER, flux_param=(gas, 0, 0, 0)), return_parts=True)
    lam = np.hypot(vx, vy) + np.sqrt(gas * pr / rho)
    he = math.sqrt(2.0) / n
    assert np.allclose(parts["lam"], lam, rtol=1e-13, atol=0)
    assert np.allclose(parts["nu"], lam * he / (2 * p), rtol=1e-13, atol=0)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_low_order_dissipation_equals_viscous_energy(p):
    """eq. stab with SC off: u . (R(gamma=0) - R(gamma=1)) = sum_e nu_e int_K |grad u_h|^2,
    nu_e = |v| h_e / (2p), on hx x hy rectangles with per-cell polynomials of
    degree p (the interface terms cancel in the difference)."""
    nx, ny, hx, hy = 4, 3, 0.25, 0.4
    mesh = synth.quad_mesh(nx, ny, 0.0, nx * hx, 0.0, ny * hy)
    sp = build_space(mesh, p, 1)
    E = nx * ny
    rng = np.random.default_rng(20 + p)
    polys = [_poly2d(rng, p) for _ in range(E)]
    xn = sp.node_coords()
    U = np.stack([polys[e][0](xn[e, :, 0], xn[e, :, 1]) for e in range(E)]).ravel()
    v = (0.6, 0.8)
    base = dict(flux=synth.ADVECT_CONST, flux_param=(v[0], v[1], 0, 0), sc_on=0, sensor=2)
    R0 = residual(sp, U, Params(fixed_gamma=0.0, **base))
    R1 = residual(sp, U, Params(fixed_gamma=1.0, **base))
    lhs = U @ (R0 - R1)
    gx, gw = np.polynomial.legendre.leggauss(p + 3)
    X = mesh.cell_coords
    nu = math.hypot(*v) * math.hypot(hx, hy) / (2 * p)
    rhs = 0.0
    for e in range(E):
        x0, y0 = X[e, 0]
        xs, ys = x0 + 0.5 * hx * (gx + 1), y0 + 0.5 * hy * (gx + 1)
        XX, YY = np.meshgrid(xs, ys, indexing="xy")
        WW = np.outer(gw, gw) * 0.25 * hx * hy
        ux, uy = polys[e][1](XX, YY)
        rhs += nu * (WW * (ux * ux + uy * uy)).sum()
    assert abs(lhs - rhs) <= 1e-12 * rhs, (lhs, rhs)
