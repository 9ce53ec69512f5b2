"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only builds *inputs*: mesh descriptions (cell -> vertex ids and
unwrapped vertex coordinates), continuous initial-data functions u0(x) and
parameter sets.  It contains none of the method's arithmetic (no basis, no
quadrature, no sensor, no flux discretisation); interpolating u0 at the nodes
of a finite element space is done by whoever owns that space.

Mesh description convention (used by both the oracle and the C library):

* ``cell_vertices`` int32 [E, v_e]: topological vertex ids after periodic
  identification, counter-clockwise for 2D cells.
* ``cell_coords`` float64 [E, v_e, dim]: the *unwrapped* physical coordinates
  of each cell's vertices (a cell on a periodic seam keeps its own geometric
  position; only the vertex ids wrap).
* quads: local vertices (x0,y0),(x1,y0),(x1,y1),(x0,y1) of the logical cell;
  triangles: each logical square (i,j) is split along its (i,j)-(i+1,j+1)
  diagonal into (v00,v10,v11) and (v00,v11,v01); segments: (left, right).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEG, TRI, QUAD, HEX, TET = 1, 2, 3, 4, 5
CG, DG = 0, 1
ADVECT_CONST, ADVECT_ROT, BURGERS, KPP, EULER = 0, 1, 2, 3, 4
# boundary data at the two ends of a non-periodic 1D domain
BC_NONE, BC_OUTFLOW, BC_WALL, BC_INFLOW = 0, 1, 2, 3


@dataclass
class MeshDesc:
    dim: int
    cell: int
    n_vertices: int
    cell_vertices: np.ndarray  # int32 [E, v_e]
    cell_coords: np.ndarray    # float64 [E, v_e, dim]
    periodic: tuple = (1, 1)
    shape: tuple = ()          # logical (nx,), (nx, ny) or (nx, ny, nz), informative only

    @property
    def n_cells(self) -> int:
        return int(self.cell_vertices.shape[0])


def segment_mesh(n: int, x0: float = 0.0, x1: float = 1.0, periodic: bool = True) -> MeshDesc:
    h = (x1 - x0) / n
    i = np.arange(n)
    left = i
    right = (i + 1) % n if periodic else i + 1
    nv = n if periodic else n + 1
    cv = np.stack([left, right], axis=1).astype(np.int32)
    xl = x0 + i * h
    cc = np.stack([xl, xl + h], axis=1)[:, :, None].astype(np.float64)
    return MeshDesc(1, SEG, nv, cv, cc, (int(periodic), 0), (n,))


def _grid_vertices(nx, ny, x0, x1, y0, y1, jitter, seed, periodic):
    hx = (x1 - x0) / nx
    hy = (y1 - y0) / ny
    px, py = periodic
    nvx = nx if px else nx + 1
    nvy = ny if py else ny + 1
    jit = np.zeros((nvy, nvx, 2))
    if jitter > 0:
        rng = np.random.default_rng(seed)
        # one draw per canonical vertex, row-major (x fastest), x then y
        jit = rng.uniform(-jitter, jitter, size=(nvy, nvx, 2))
        jit[..., 0] *= hx
        jit[..., 1] *= hy
        if not px:
            jit[:, 0, 0] = 0.0
            jit[:, -1, 0] = 0.0
        if not py:
            jit[0, :, 1] = 0.0
            jit[-1, :, 1] = 0.0

    def vid(i, j):
        ii = i % nx if px else i
        jj = j % ny if py else j
        return ii + nvx * jj

    def pos(i, j):
        ii = i % nx if px else i
        jj = j % ny if py else j
        return np.stack([x0 + i * hx + jit[jj, ii, 0], y0 + j * hy + jit[jj, ii, 1]], axis=-1)

    return vid, pos, nvx * nvy


def quad_mesh(nx: int, ny: int, x0=0.0, x1=1.0, y0=0.0, y1=1.0, jitter: float = 0.0,
              seed: int = 0, periodic=(True, True)) -> MeshDesc:
    vid, pos, nv = _grid_vertices(nx, ny, x0, x1, y0, y1, jitter, seed, periodic)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    corners = [(i, j), (i + 1, j), (i + 1, j + 1), (i, j + 1)]
    cv = np.stack([vid(a, b) for a, b in corners], axis=1).astype(np.int32)
    cc = np.stack([pos(a, b) for a, b in corners], axis=1).astype(np.float64)
    return MeshDesc(2, QUAD, nv, cv, cc, tuple(int(p) for p in periodic), (nx, ny))


def tri_mesh(nx: int, ny: int, x0=0.0, x1=1.0, y0=0.0, y1=1.0, jitter: float = 0.0,
             seed: int = 0, periodic=(True, True)) -> MeshDesc:
    vid, pos, nv = _grid_vertices(nx, ny, x0, x1, y0, y1, jitter, seed, periodic)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    v00, v10, v11, v01 = (i, j), (i + 1, j), (i + 1, j + 1), (i, j + 1)
    E = nx * ny
    cv = np.empty((2 * E, 3), np.int32)
    cc = np.empty((2 * E, 3, 2), np.float64)
    for t, tri in enumerate([(v00, v10, v11), (v00, v11, v01)]):
        cv[t::2] = np.stack([vid(a, b) for a, b in tri], axis=1)
        cc[t::2] = np.stack([pos(a, b) for a, b in tri], axis=1)
    return MeshDesc(2, TRI, nv, cv, cc, tuple(int(p) for p in periodic), (nx, ny))


def hex_mesh(nx: int, ny: int, nz: int, x0=0.0, x1=1.0, y0=0.0, y1=1.0, z0=0.0, z1=1.0,
             periodic=(True, True, True)) -> MeshDesc:
    """Structured mesh of congruent axis-aligned boxes, cell e = i + nx (j + ny k).
    Local vertices: the bottom face (z = z_k) counter-clockwise from (i, j),
    then the top face in the same order.  Coordinates are unwrapped per cell
    (a cell across a periodic boundary keeps its own box)."""
    hx, hy, hz = (x1 - x0) / nx, (y1 - y0) / ny, (z1 - z0) / nz
    px, py, pz = periodic
    nvx, nvy, nvz = (nx if px else nx + 1), (ny if py else ny + 1), (nz if pz else nz + 1)

    def vid(i, j, k):
        return ((i % nx if px else i) + nvx * ((j % ny if py else j) + nvy * (k % nz if pz else k)))

    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    i, j, k = i.ravel(), j.ravel(), k.ravel()
    corners = [(0, 0, 0), (1, 0, 0), (1, 1, 0), (0, 1, 0), (0, 0, 1), (1, 0, 1), (1, 1, 1), (0, 1, 1)]
    cv = np.stack([vid(i + a, j + b, k + c) for a, b, c in corners], axis=1).astype(np.int32)
    cc = np.stack([np.stack([x0 + (i + a) * hx, y0 + (j + b) * hy, z0 + (k + c) * hz], axis=-1)
                   for a, b, c in corners], axis=1).astype(np.float64)
    return MeshDesc(3, HEX, nvx * nvy * nvz, cv, cc, tuple(int(q) for q in periodic), (nx, ny, nz))


def tet_mesh(nx: int, ny: int, nz: int, x0=0.0, x1=1.0, y0=0.0, y1=1.0, z0=0.0, z1=1.0,
             periodic=(True, True, True)) -> MeshDesc:
    """Each box of hex_mesh split into six tetrahedra around its diagonal from
    the lowest to the highest corner (the same split in every box, so the
    faces match across boxes); cell 6 box + t; every tetrahedron positively
    oriented (vertices 1, 2 swapped where needed)."""
    h = hex_mesh(nx, ny, nz, x0, x1, y0, y1, z0, z1, periodic)
    paths = [(1, 2), (1, 5), (3, 2), (3, 7), (4, 5), (4, 7)]     # corners between 0 and 6
    E = h.n_cells
    cv = np.empty((6 * E, 4), np.int32)
    cc = np.empty((6 * E, 4, 3), np.float64)
    for t, (a, b) in enumerate(paths):
        loc = [0, a, b, 6]
        X = h.cell_coords[:, loc]
        det = np.linalg.det(np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=-1))
        if det[0] < 0:
            loc = [0, b, a, 6]
        cv[t::6] = h.cell_vertices[:, loc]
        cc[t::6] = h.cell_coords[:, loc]
    return MeshDesc(3, TET, h.n_vertices, cv, cc, h.periodic, h.shape)


# ---------------------------------------------------------------------------
# Parameters of the method (defaults are the values the paper states)
# ---------------------------------------------------------------------------
@dataclass
class Params:
    flux: int = ADVECT_CONST
    flux_param: tuple = (1.0, 0.0, 0.0, 0.0)  # const velocity (vx, vy) / gas gamma
    eps_vertex: float = 1e-6
    eps_cell: float = 1e-6
    r: int = 2
    q_sensor: float = 1.0
    q_beta: float = 1.0
    lin_w_vertex: float = 1e-3
    sc_on: int = 1
    c_gamma: float = 0.9
    lambda_global: float = 0.0
    sensor: int = 0          # 0 plain HWENO sensor, 2 fixed gamma
    fixed_gamma: float = 1.0
    # 1D domains with ends: the kind at the left and right end (BC_*) and the
    # exterior state of an inflow end (conserved variables)
    bc: tuple = (BC_NONE, BC_NONE)
    bc_state: tuple = ((0.0, 0.0, 0.0, 0.0), (0.0, 0.0, 0.0, 0.0))
    # 2D meshes with boundary faces: the kind (BC_*) and exterior state of each
    # boundary face, in ascending (cell, local face) order ([n_bfaces], [n_bfaces, n_var])
    bc_face_kind: object = None
    bc_face_state: object = None


# ---------------------------------------------------------------------------
# Initial data (continuous functions of the physical coordinates)
# ---------------------------------------------------------------------------
def u0_config1(x):
    """Unit square pulse on [0.2,0.4] plus a cos^2 hump on [0.6,0.8]."""
    x = np.asarray(x)
    pulse = ((x >= 0.2) & (x <= 0.4)).astype(float)
    hump = np.where((x >= 0.6) & (x <= 0.8), np.cos(5 * np.pi * (x - 0.7)) ** 2, 0.0)
    return pulse + hump


def config2_bodies(seed: int = 1002):
    """Centres of the slotted cylinder, cone and hump (radius 0.15)."""
    rng = np.random.default_rng(seed)
    a0 = rng.uniform(0, 2 * np.pi)
    out = []
    for k in range(3):
        ang = a0 + k * 2 * np.pi / 3 + np.deg2rad(rng.uniform(-10, 10))
        rad = 0.25 + rng.uniform(-0.02, 0.02)
        out.append((0.5 + rad * np.cos(ang), 0.5 + rad * np.sin(ang)))
    return out


def u0_config2(x, y, seed: int = 1002):
    R = 0.15
    (cx1, cy1), (cx2, cy2), (cx3, cy3) = config2_bodies(seed)
    u = np.zeros(np.broadcast(x, y).shape)
    # slotted cylinder: slot of width R/3 pointing at the domain centre,
    # running from the rim through 70% of the diameter
    dx, dy = x - cx1, y - cy1
    r1 = np.hypot(dx, dy)
    tx, ty = 0.5 - cx1, 0.5 - cy1
    tn = math.hypot(tx, ty)
    tx, ty = tx / tn, ty / tn
    along = dx * tx + dy * ty          # towards the centre
    across = -dx * ty + dy * tx
    slot = (np.abs(across) <= R / 6) & (along >= R - 1.4 * R)
    u = np.where((r1 <= R) & ~slot, 1.0, u)
    r2 = np.hypot(x - cx2, y - cy2)
    u = np.where(r2 <= R, 1.0 - r2 / R, u)
    r3 = np.hypot(x - cx3, y - cy3)
    u = np.where(r3 <= R, np.cos(np.pi * r3 / (2 * R)) ** 2, u)
    return u


def u0_kpp(x, y):
    return np.where(np.hypot(x, y) <= 1.0, 3.5 * np.pi, 0.25 * np.pi)


def euler_quadrants(seed: int = 1004):
    """(rho, vx, vy, p) for the NE, NW, SW, SE quadrants."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(4):
        rho = rng.uniform(0.1, 1.5)
        p = rng.uniform(0.03, 1.5)
        vx, vy = rng.uniform(-1, 1, size=2)
        out.append((rho, vx, vy, p))
    return out


def _periodic_step(s, k):
    """Smooth periodic indicator of [0.5, 1) on the unit period; k sets the sharpness."""
    return 0.5 * (1.0 + np.tanh(-k * np.sin(2 * np.pi * s)))


def euler_state_config4(x, y, seed: int = 1004, gas_gamma: float = 1.4, smooth_k: float | None = None):
    """Conserved variables (rho, rho*vx, rho*vy, rho*E) of the four-quadrant data.

    With ``smooth_k=None`` the data is piecewise constant (quadrant split at
    (0.5, 0.5) on the unit periodic square); with a value, the quadrant
    indicators are smoothed periodic steps of sharpness ``smooth_k`` (used as a
    synthetic mid-run state whose discontinuities span a few cells).
    """
    q = euler_quadrants(seed)
    if smooth_k is None:
        hx = (np.asarray(x) % 1.0 >= 0.5).astype(float)
        hy = (np.asarray(y) % 1.0 >= 0.5).astype(float)
    else:
        hx = _periodic_step(np.asarray(x), smooth_k)
        hy = _periodic_step(np.asarray(y), smooth_k)
    w = [hx * hy, (1 - hx) * hy, (1 - hx) * (1 - hy), hx * (1 - hy)]
    rho = sum(wq * qq[0] for wq, qq in zip(w, q))
    vx = sum(wq * qq[1] for wq, qq in zip(w, q))
    vy = sum(wq * qq[2] for wq, qq in zip(w, q))
    p = sum(wq * qq[3] for wq, qq in zip(w, q))
    E = p / (gas_gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy)
    return np.stack([rho, rho * vx, rho * vy, E])


@dataclass
class Instance:
    n: int
    p: int
    flux: int
    velocity: tuple
    rects: list = field(default_factory=list)   # (x0, x1, y0, y1, value)
    gauss: tuple = (0.5, 0.5, 0.5, 1.0, 0.05)   # (cx, cy, amplitude, ..., sigma)


def config5_instances(seed: int = 1005, count: int = 64):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        u = rng.uniform()
        n = int(np.clip(8 * round(8 * 8 ** u), 64, 512))
        p = int(rng.integers(1, 4))
        flux = ADVECT_CONST if rng.uniform() < 0.5 else BURGERS
        th = rng.uniform(0, 2 * np.pi)
        rects = []
        for _r in range(int(rng.integers(1, 5))):
            a, b = np.sort(rng.uniform(0, 1, 2))
            c, d = np.sort(rng.uniform(0, 1, 2))
            rects.append((a, b, c, d, rng.uniform()))
        g = (rng.uniform(0, 1), rng.uniform(0, 1), rng.uniform(0.5, 1.0), rng.uniform(0.02, 0.1))
        out.append(Instance(n, p, flux, (math.cos(th), math.sin(th)), rects, g))
    return out


def u0_instance(inst: Instance, x, y):
    u = np.zeros(np.broadcast(x, y).shape)
    for (a, b, c, d, v) in inst.rects:
        u = u + np.where((x >= a) & (x <= b) & (y >= c) & (y <= d), v, 0.0)
    cx, cy, amp, sig = inst.gauss
    dx = (x - cx + 0.5) % 1.0 - 0.5
    dy = (y - cy + 0.5) % 1.0 - 0.5
    return u + amp * np.exp(-(dx * dx + dy * dy) / (2 * sig * sig))


def instance_params(inst: Instance) -> "Params":
    """Method parameters of one ensemble instance (paper defaults, its flux)."""
    if inst.flux == ADVECT_CONST:
        return Params(flux=ADVECT_CONST, flux_param=(inst.velocity[0], inst.velocity[1], 0.0, 0.0))
    return Params(flux=BURGERS, flux_param=(1.0, 1.0, 0.0, 0.0))


def instance_case(inst: Instance, n: int = None, cfl: float = 0.1):
    """(mesh, p, params, nodal state [E * (p+1)^2], dt) of one ensemble instance:
    periodic n x n unit-square quads (n defaults to the instance's), the initial
    data sampled at the Gauss-Legendre nodes of each cell (node (a, b) at index
    a + (p+1) b), and dt = cfl * h / ((2p + 1) lambda_max) with lambda_max of
    the initial data (the explicit DG limit; the shock-capturing viscosity
    needs cfl well below 0.2)."""
    n = inst.n if n is None else n
    p = inst.p
    mesh = quad_mesh(n, n)
    g, _ = np.polynomial.legendre.leggauss(p + 1)
    h = 1.0 / n
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    xc = (ii.ravel() + 0.5) * h
    yc = (jj.ravel() + 0.5) * h
    gx, gy = np.meshgrid(g, g, indexing="xy")
    X = xc[:, None] + 0.5 * h * gx.ravel()[None, :]
    Y = yc[:, None] + 0.5 * h * gy.ravel()[None, :]
    U = u0_instance(inst, X, Y)
    prm = instance_params(inst)
    lam = 1.0 if inst.flux == ADVECT_CONST else float(np.sqrt(2.0) * np.abs(U).max())
    dt = cfl * h / ((2 * p + 1) * lam)
    return mesh, p, prm, U.ravel(), dt


def smooth_field(x, y, seed: int, modes: int = 3):
    """A seeded smooth periodic field on the unit square (sum of a few Fourier modes)."""
    rng = np.random.default_rng(seed)
    u = np.zeros(np.broadcast(x, y).shape)
    for _ in range(modes):
        kx, ky = rng.integers(-3, 4, 2)
        a = rng.normal()
        ph = rng.uniform(0, 2 * np.pi)
        u = u + a * np.cos(2 * np.pi * (kx * x + ky * y) + ph)
    return u


def random_nodal(shape, seed: int, scale: float = 1.0):
    """Seeded arbitrary nodal values (for tests that do not need a physical state)."""
    return np.random.default_rng(seed).uniform(-scale, scale, size=shape)


# ---------------------------------------------------------------------------
# One-dimensional Euler data (conserved variables rho, m = rho v, E), gamma 1.4
# ---------------------------------------------------------------------------
def euler1d_conserved(rho, v, p, gas_gamma: float = 1.4):
    """(rho, rho v, p / (gamma - 1) + rho v^2 / 2) from primitive values."""
    rho, v, p = np.broadcast_arrays(np.asarray(rho, np.float64), np.asarray(v, np.float64),
                                    np.asarray(p, np.float64))
    return rho, rho * v, p / (gas_gamma - 1.0) + 0.5 * rho * v * v


# ---------------------------------------------------------------------------
# Double Mach reflection (Sec. 5.4) on (0, 4) x (0, 1), gamma 1.4
# ---------------------------------------------------------------------------
def dmr_states(gas_gamma: float = 1.4):
    """Post-shock (L) and pre-shock (R) conserved states (rho, m_x, m_y, E):
    (rho, v_x, v_y, p) = (8, 8.25 cos 30deg, -8.25 sin 30deg, 116.5) and
    (1.4, 0, 0, 1)."""
    def cons(rho, vx, vy, p):
        return np.array([rho, rho * vx, rho * vy, p / (gas_gamma - 1.0) + 0.5 * rho * (vx * vx + vy * vy)])
    a = np.deg2rad(30.0)
    return cons(8.0, 8.25 * np.cos(a), -8.25 * np.sin(a), 116.5), cons(1.4, 0.0, 0.0, 1.0)


def dmr_shock_x(y, t):
    """x of the moving Mach 10 shock at height y and time t."""
    return 1.0 / 6.0 + (y + 20.0 * t) / np.sqrt(3.0)


def u0_dmr(x, y, gas_gamma: float = 1.4):
    """Initial data: the post-shock state left of the shock line, pre-shock
    right of it; conserved variables [4, ...]."""
    L, R = dmr_states(gas_gamma)
    left = np.asarray(x) < dmr_shock_x(np.asarray(y), 0.0)
    return np.where(left[None], L.reshape((4,) + (1,) * left.ndim), R.reshape((4,) + (1,) * left.ndim))


def dmr_boundary(mid, normal, t: float, gas_gamma: float = 1.4):
    """Kind and exterior state of each boundary face from its midpoint
    [nb, 2] and outward normal [nb, 2] at time t: the bottom is inflow of the
    post-shock state for x < 1/6 and a reflecting wall beyond; the left side
    inflow (post-shock); the right side outflow; the top inflow of the
    post-shock state left of the moving shock and the pre-shock state right
    of it.  Returns (kinds [nb] int32, states [nb, 4])."""
    L, R = dmr_states(gas_gamma)
    mid = np.asarray(mid, np.float64)
    n = np.asarray(normal, np.float64)
    kinds = np.full(len(mid), BC_INFLOW, np.int32)
    states = np.tile(L, (len(mid), 1))
    bottom, top, right = n[:, 1] < -0.7, n[:, 1] > 0.7, n[:, 0] > 0.7
    kinds[bottom & (mid[:, 0] >= 1.0 / 6.0)] = BC_WALL
    kinds[right] = BC_OUTFLOW
    states[top & (mid[:, 0] >= dmr_shock_x(1.0, t))] = R
    return kinds, states


def u0_modified_sod(x):
    """Modified Sod shock tube on (0, 1): (rho, v, p) = (1, 0.75, 1) left of
    x = 0.25, (0.125, 0, 0.1) right of it; conserved variables [3, ...]."""
    x = np.asarray(x, np.float64)
    left = x < 0.25
    return np.stack(euler1d_conserved(np.where(left, 1.0, 0.125), np.where(left, 0.75, 0.0),
                                      np.where(left, 1.0, 0.1)))


def modified_sod_params(flux_gamma: float = 1.4) -> Params:
    """Inflow of the left state at x = 0, reflecting wall at x = 1."""
    inflow = tuple(float(c) for c in euler1d_conserved(1.0, 0.75, 1.0, flux_gamma)) + (0.0,)
    return Params(flux=EULER, flux_param=(flux_gamma, 0.0, 0.0, 0.0), bc=(BC_INFLOW, BC_WALL),
                  bc_state=(inflow, (0.0, 0.0, 0.0, 0.0)))


def u0_blast_wave(x):
    """Woodward-Colella blast waves on (0, 1): rho = 1, v = 0, p = 1000 / 0.01 /
    100 on (0, 0.1) / [0.1, 0.9] / (0.9, 1); conserved variables [3, ...]."""
    x = np.asarray(x, np.float64)
    p = np.where(x < 0.1, 1000.0, np.where(x > 0.9, 100.0, 0.01))
    return np.stack(euler1d_conserved(np.ones_like(x), np.zeros_like(x), p))


def blast_wave_params(flux_gamma: float = 1.4) -> Params:
    """Reflecting walls at both ends."""
    return Params(flux=EULER, flux_param=(flux_gamma, 0.0, 0.0, 0.0), bc=(BC_WALL, BC_WALL))
