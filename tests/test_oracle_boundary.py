"""Pins of the oracle's 1D Euler equations, boundary data and high-degree
bases (the shock-tube and blast-wave runs of Sec. 5.4: an inflow end,
reflecting walls, degrees up to 32 on eight elements).

* the Lagrange basis at degree 16-32: the Kronecker property, the top
  derivative in closed form p! / prod_{i != j} (x_j - x_i), and exact
  reproduction of monomials with their derivatives;
* the 1D Euler flux and wave speed from primitive variables (the paper's
  flux written with rho, v, p); HLL consistency;
* a reflecting wall equals the periodic mirror-extended domain, and an inflow
  end equals a domain extended by one cell holding the inflow state (DG, a
  fixed gamma so that only the flux terms are compared);
* free streams: a constant state with matching inflow data, and gas at rest
  between walls, give R = 0 (CG and DG);
* walls at both ends conserve mass and energy (CG and DG, the plain sensor);
* on a domain with ends, a global polynomial of degree p has gamma = 1 in
  every cell (the vertex patches at the ends take only the cells present);
* a smooth 1D Euler wave converges at order p + 1 with DG.
"""
import math

import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space, nodal_interpolate, residual, rk3_step
from oracle.basis import Lagrange1D, gauss_legendre, gauss_lobatto
from oracle.method import flux, numerical_flux, wave_speed, sensor_gamma

G = 1.4


# ---------------------------------------------------------------------------
# bases at high degree
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p", [16, 24, 32])
@pytest.mark.parametrize("rule", ["gauss", "lobatto"])
def test_lagrange_high_degree(p, rule):
    x = (gauss_legendre if rule == "gauss" else gauss_lobatto)(p + 1)[0]
    L = Lagrange1D(x)
    assert np.abs(L(x) - np.eye(p + 1)).max() < 1e-12
    xs = np.linspace(-1.0, 1.0, 11)
    top = np.array([math.factorial(p) / np.prod(x[j] - np.delete(x, j)) for j in range(p + 1)])
    got = L(xs, p)
    assert np.abs(got - top[None, :]).max() <= 1e-9 * np.abs(top).max()
    assert np.abs(L(xs, p + 1)).max() == 0.0
    for k in range(7):
        for m in range(k + 1):
            Lm = L(xs, m)
            val = Lm @ x ** k
            exact = math.factorial(k) / math.factorial(k - m) * xs ** (k - m)
            scale = np.abs(Lm).sum(1).max()
            assert np.abs(val - exact).max() <= 1e-13 * scale, (k, m)


# ---------------------------------------------------------------------------
# 1D Euler flux
# ---------------------------------------------------------------------------
def _cons(rho, v, p):
    return np.array(synth.euler1d_conserved(rho, v, p, G), np.float64)


EULER1 = Params(flux=synth.EULER, flux_param=(G, 0, 0, 0))


def test_euler1d_flux_and_speed():
    rho, v, p = 1.3, -0.45, 2.2
    U = _cons(rho, v, p)[:, None]
    x = np.zeros((1, 1))
    E = p / (G - 1) + 0.5 * rho * v * v
    F = flux(EULER1, U, x)[..., 0]
    assert np.allclose(F[:, 0], [rho * v, rho * v * v + p, v * (E + p)], rtol=1e-15, atol=0)
    assert wave_speed(EULER1, U, x)[0] == pytest.approx(abs(v) + math.sqrt(G * p / rho), rel=1e-15)
    for n in (-1.0, 1.0):
        Fs = numerical_flux(EULER1, U, U, np.full((1, 1), n), x)
        assert np.allclose(Fs[:, 0], n * F[:, 0], rtol=1e-15, atol=1e-15)


def _smooth_state(sp, seed):
    rng = np.random.default_rng(seed)
    a, b, ph = rng.uniform(0.1, 0.3, 3)
    prim = [lambda x: 1.0 + a * np.sin(2 * np.pi * x[..., 0] + ph),
            lambda x: b * np.cos(2 * np.pi * x[..., 0]),
            lambda x: 1.0 + b * np.cos(4 * np.pi * x[..., 0] + ph)]
    return nodal_interpolate(sp, [lambda x, c=c: np.asarray(
        synth.euler1d_conserved(prim[0](x), prim[1](x), prim[2](x), G))[c] for c in range(3)])


# ---------------------------------------------------------------------------
# walls and inflow against extended domains (DG, fixed gamma)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("p", [2, 5])
def test_wall_equals_mirror_domain(p):
    N = 6
    sp = build_space(synth.segment_mesh(N, 0.0, 1.0, periodic=False), p, 1, 3)
    U = sp.to_cells(_smooth_state(sp, 3))
    prm = Params(flux=synth.EULER, flux_param=(G, 0, 0, 0), sensor=2, fixed_gamma=0.5,
                 bc=(synth.BC_WALL, synth.BC_WALL))
    R = residual(sp, U.ravel(), prm).reshape(3, N, p + 1)
    sp2 = build_space(synth.segment_mesh(2 * N, 0.0, 2.0, periodic=True), p, 1, 3)
    M = U[:, ::-1, ::-1].copy()                    # x -> 2 - x: cells and nodes reversed
    M[1] = -M[1]
    U2 = np.concatenate([U, M], axis=1)
    prm2 = Params(flux=synth.EULER, flux_param=(G, 0, 0, 0), sensor=2, fixed_gamma=0.5)
    R2 = residual(sp2, U2.ravel(), prm2).reshape(3, 2 * N, p + 1)
    assert np.abs(R - R2[:, :N]).max() <= 1e-12 * np.abs(R).max()
    # a sign slip in the mirror or the boundary term shows here
    assert np.abs(R[:, 0]).max() > 1e-3


@pytest.mark.parametrize("p", [1, 4])
def test_inflow_equals_extended_domain(p):
    N = 5
    h = 1.0 / N
    u_in = _cons(1.0, 0.75, 1.0)
    sp = build_space(synth.segment_mesh(N, 0.0, 1.0, periodic=False), p, 1, 3)
    U = sp.to_cells(_smooth_state(sp, 5))
    base = dict(flux=synth.EULER, flux_param=(G, 0, 0, 0), sensor=2, fixed_gamma=0.3)
    prm = Params(**base, bc=(synth.BC_INFLOW, synth.BC_OUTFLOW), bc_state=(tuple(u_in) + (0.0,), (0, 0, 0, 0)))
    R = residual(sp, U.ravel(), prm).reshape(3, N, p + 1)
    spx = build_space(synth.segment_mesh(N + 1, -h, 1.0, periodic=False), p, 1, 3)
    Ux = np.concatenate([np.broadcast_to(u_in[:, None, None], (3, 1, p + 1)), U], axis=1)
    prmx = Params(**base, bc=(synth.BC_OUTFLOW, synth.BC_OUTFLOW))
    Rx = residual(spx, Ux.ravel(), prmx).reshape(3, N + 1, p + 1)
    assert np.abs(R - Rx[:, 1:]).max() <= 1e-12 * np.abs(R).max()


# ---------------------------------------------------------------------------
# free streams and conservation (CG and DG, plain sensor)
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("p", [3, 8])
def test_free_streams(kind, p):
    mesh = synth.segment_mesh(7, periodic=False)
    sp = build_space(mesh, p, kind, 3)
    u_in = _cons(0.9, 0.6, 1.1)
    U = nodal_interpolate(sp, [lambda x, c=c: np.full(x.shape[:-1], u_in[c]) for c in range(3)])
    prm = Params(flux=synth.EULER, flux_param=(G, 0, 0, 0), bc=(synth.BC_INFLOW, synth.BC_OUTFLOW),
                 bc_state=(tuple(u_in) + (0.0,), (0, 0, 0, 0)))
    assert np.abs(residual(sp, U, prm)).max() <= 1e-13 * np.abs(u_in).max()
    rest = _cons(1.2, 0.0, 0.8)
    U = nodal_interpolate(sp, [lambda x, c=c: np.full(x.shape[:-1], rest[c]) for c in range(3)])
    prm = Params(flux=synth.EULER, flux_param=(G, 0, 0, 0), bc=(synth.BC_WALL, synth.BC_WALL))
    assert np.abs(residual(sp, U, prm)).max() <= 1e-13 * np.abs(rest).max()


@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("p", [2, 6])
def test_walls_conserve_mass_and_energy(kind, p):
    mesh = synth.segment_mesh(9, periodic=False)
    sp = build_space(mesh, p, kind, 3)
    U = _smooth_state(sp, 11)
    R = residual(sp, U, synth.blast_wave_params()).reshape(3, -1)
    scale = np.abs(R).max()
    assert scale > 1e-2
    assert abs(R[0].sum()) <= 1e-13 * scale * R.shape[1]
    assert abs(R[2].sum()) <= 1e-13 * scale * R.shape[1]
    # the momentum balance is the wall pressure force: gas at rest with the
    # pressure 1 + 0.3 x^2 (interpolated exactly) gives sum R_m = p(1) - p(0)
    Ur = nodal_interpolate(sp, [lambda x, c=c: np.asarray(synth.euler1d_conserved(
        1.0 + 0.2 * np.sin(2 * np.pi * x[..., 0]), 0.0, 1.0 + 0.3 * x[..., 0] ** 2, G))[c] for c in range(3)])
    Rr = residual(sp, Ur, synth.blast_wave_params()).reshape(3, -1)
    assert Rr[1].sum() == pytest.approx(0.3, abs=1e-12)


# ---------------------------------------------------------------------------
# sensor at the ends of a domain
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("kind", [0, 1])
@pytest.mark.parametrize("p", [3, 6])
def test_global_polynomial_is_smooth_up_to_the_ends(kind, p):
    mesh = synth.segment_mesh(8, periodic=False)
    sp = build_space(mesh, p, kind, 1)
    c = np.random.default_rng(p).normal(size=p + 1)
    U = nodal_interpolate(sp, [lambda x: np.polynomial.polynomial.polyval(2 * x[..., 0] - 1, c)])
    g = sensor_gamma(sp, sp.to_cells(U)[0], Params(flux=synth.ADVECT_CONST, bc=(synth.BC_OUTFLOW,
                                                                                   synth.BC_OUTFLOW)))
    assert np.abs(g - 1.0).max() < 1e-8
    # the same data on the periodic mesh is not a global polynomial across the wrap
    spp = build_space(synth.segment_mesh(8), p, kind, 1)
    Up = nodal_interpolate(spp, [lambda x: np.polynomial.polynomial.polyval(2 * x[..., 0] - 1, c)])
    gp = sensor_gamma(spp, spp.to_cells(Up)[0], Params(flux=synth.ADVECT_CONST))
    assert gp.min() < 1.0 - 1e-5


# ---------------------------------------------------------------------------
# convergence of a smooth 1D Euler wave (DG)
# ---------------------------------------------------------------------------
def test_euler1d_dg_convergence():
    """An entropy wave rho = 1 + 0.2 sin(2 pi (x - t)), v = 1, p = 1 on a
    periodic line, DG P2, to t = 0.05: errors fall at about order 3."""
    p, T = 2, 0.05
    errs = []
    for N in (12, 24):
        sp = build_space(synth.segment_mesh(N), p, 1, 3)

        def state(t):
            return nodal_interpolate(sp, [lambda x, c=c: np.asarray(synth.euler1d_conserved(
                1.0 + 0.2 * np.sin(2 * np.pi * (x[..., 0] - t)), 1.0, 1.0, G))[c] for c in range(3)])
        U = state(0.0)
        steps = int(np.ceil(T / (0.1 / N)))
        dt = T / steps
        for _ in range(steps):
            U = rk3_step(sp, U, dt, EULER1)
        errs.append(np.abs(U - state(T)).max())
    rate = np.log2(errs[0] / errs[1])
    assert rate > p + 0.5, errs


# ---------------------------------------------------------------------------
# 2D meshes with boundary faces (one kind and state per face)
# ---------------------------------------------------------------------------
from oracle.method import boundary_faces  # noqa: E402

EULER2 = dict(flux=synth.EULER, flux_param=(G, 0, 0, 0))


def _cons2(rho, vx, vy, p):
    return np.array([rho, rho * vx, rho * vy, p / (G - 1) + 0.5 * rho * (vx * vx + vy * vy)])


def _euler2_smooth(sp, seed):
    rng = np.random.default_rng(seed)
    a, b, ph = rng.uniform(0.1, 0.3, 3)

    def prim(x):
        X, Y = x[..., 0], x[..., 1]
        return (1.0 + a * np.sin(2 * np.pi * X + ph) * np.cos(2 * np.pi * Y),
                b * np.cos(2 * np.pi * X) + 0.1, b * np.sin(2 * np.pi * Y),
                1.0 + b * np.cos(2 * np.pi * (X + Y) + ph))
    return nodal_interpolate(sp, [lambda x, c=c: _cons2(*prim(x))[c] for c in range(4)])


@pytest.mark.parametrize("p", [1, 3])
def test_2d_wall_equals_mirror_domain(p):
    """Walls at x = 0 and x = 1 (periodic in y) against the periodic domain
    [0, 2] x [0, 1] holding the state and its mirror image (DG quads, fixed
    gamma)."""
    N, M = 4, 3
    sp = build_space(synth.quad_mesh(N, M, periodic=(False, True)), p, 1, 4)
    cells, _ = boundary_faces(sp)
    U = sp.to_cells(_euler2_smooth(sp, 2))
    base = dict(EULER2, sensor=2, fixed_gamma=0.4)
    R = residual(sp, U.ravel(), Params(**base, bc_face_kind=np.full(len(cells), synth.BC_WALL))).reshape(4, N * M, -1)
    sp2 = build_space(synth.quad_mesh(2 * N, M, 0.0, 2.0, periodic=(True, True)), p, 1, 4)
    n1 = p + 1
    U2 = np.zeros((4, 2 * N * M, n1 * n1))
    for j in range(M):
        for i in range(N):
            src = U[:, i + N * j].reshape(4, n1, n1)               # [v, b, a]
            U2[:, i + 2 * N * j] = src.reshape(4, -1)
            mir = src[:, :, ::-1].copy()                             # x -> 2 - x: node a -> p - a
            mir[1] = -mir[1]
            U2[:, (2 * N - 1 - i) + 2 * N * j] = mir.reshape(4, -1)
    R2 = residual(sp2, U2.ravel(), Params(**base)).reshape(4, 2 * N * M, -1)
    own = np.array([i + 2 * N * j for j in range(M) for i in range(N)])
    assert np.abs(R - R2[:, own]).max() <= 1e-12 * np.abs(R).max()


@pytest.mark.parametrize("cell", ["quad", "tri"])
@pytest.mark.parametrize("p", [2, 3])
def test_2d_free_streams_and_wall_conservation(cell, p):
    mesh = synth.quad_mesh(4, 3, periodic=(False, False)) if cell == "quad" else \
        synth.tri_mesh(4, 3, jitter=0.1, seed=5, periodic=(False, False))
    sp = build_space(mesh, p, 1, 4)
    nb = len(boundary_faces(sp)[0])
    st = _cons2(0.9, 0.5, -0.3, 1.1)
    U = nodal_interpolate(sp, [lambda x, c=c: np.full(x.shape[:-1], st[c]) for c in range(4)])
    kinds = np.where(np.arange(nb) % 2 == 0, synth.BC_INFLOW, synth.BC_OUTFLOW)
    prm = Params(**EULER2, bc_face_kind=kinds, bc_face_state=np.tile(st, (nb, 1)))
    assert np.abs(residual(sp, U, prm)).max() <= 1e-13 * np.abs(st).max()
    rest = _cons2(1.2, 0.0, 0.0, 0.8)
    U = nodal_interpolate(sp, [lambda x, c=c: np.full(x.shape[:-1], rest[c]) for c in range(4)])
    walls = Params(**EULER2, bc_face_kind=np.full(nb, synth.BC_WALL))
    assert np.abs(residual(sp, U, walls)).max() <= 1e-13 * np.abs(rest).max()
    # walls all round conserve mass and energy (plain sensor, smooth data)
    R = residual(sp, _euler2_smooth(sp, 4), walls).reshape(4, -1)
    scale = np.abs(R).max()
    assert scale > 1e-2
    assert abs(R[0].sum()) <= 1e-12 * scale * R.shape[1]
    assert abs(R[3].sum()) <= 1e-12 * scale * R.shape[1]


def test_boundary_face_order():
    """Boundary faces come in ascending (cell, local face) order: the order in
    which boundary data are given, on both sides of the library boundary."""
    sp = build_space(synth.tri_mesh(3, 3, jitter=0.1, seed=2, periodic=(False, True)), 1, 1)
    c, f = boundary_faces(sp)
    key = c * 8 + f
    assert len(c) == 2 * 3 and np.all(np.diff(key) > 0)
    assert np.all(sp.nbr[c, f] < 0) and (sp.nbr < 0).sum() == len(c)
