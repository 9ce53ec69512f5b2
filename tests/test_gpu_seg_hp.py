"""GPU parity: 1D elements of any degree (float64, one wave per cell) through
the C ABI vs the float64 oracle -- the Euler equations with an inflow end, a
reflecting wall or outflow (the shock-tube and blast-wave runs of Sec. 5.4),
degrees up to 32 on eight elements, CG and DG.

Tolerances.  The whole path is float64.  Where every derivative is well
conditioned (scalar data of degree <= 8, and states whose cells are constant
or hold one jump) the bar is 1e-9 of the largest entry for candidates, gamma,
alpha and the residual.  Degrees of 12 and more amplify the rounding of the
nodal data in the top derivatives (the scaled k-th derivative of a degree-p
Lagrange interpolant carries up to (2p)! / (2^p p!) times the data's
rounding, about 1e44 at p = 32): there the sensor of a smooth, non-constant
cell is set by rounding on both sides, so the high degrees are compared on
the shock-tube data and on whole runs by invariants and L1 distance.
"""
import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space, nodal_interpolate, residual as o_residual, rk3_step
from oracle.method import vertex_candidates as o_cand, sensor_gamma, sc_weights, projected_gradient
from tests.parity_helpers import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import cvw  # noqa: E402

ADV = Params(flux=synth.ADVECT_CONST, flux_param=(1.0, 0, 0, 0))


def sod(x, x0=0.3):
    """The modified shock tube's two states with the jump at x0 (inside a cell
    for the meshes here, so that one cell holds it)."""
    left = x < x0
    return np.stack(synth.euler1d_conserved(np.where(left, 1.0, 0.125), np.where(left, 0.75, 0.0),
                                            np.where(left, 1.0, 0.1)))


def _euler_case(space, p, N, x0=None, prm=None):
    """x0 None: the centre of the cell holding x = 0.3, so that its nodes
    straddle the jump at every degree."""
    if x0 is None:
        x0 = (np.floor(0.3 * N) + 0.5) / N
    mesh = synth.segment_mesh(N, periodic=False)
    sp = build_space(mesh, p, space, 3)
    U = nodal_interpolate(sp, [lambda x, c=c: sod(x[..., 0], x0)[c] for c in range(3)])
    return mesh, sp, U, prm or synth.modified_sod_params()


def _gpu_residual(mesh, p, space, prm, U):
    gm = cvw.Mesh(mesh, p, space)
    cp = cvw.make_params(prm, cvw.F64)
    ws = cvw.alloc_workspace(gm, cp, 0)
    u = torch.from_numpy(np.ascontiguousarray(U)).cuda()
    R = torch.empty_like(u)
    g = torch.empty(mesh.n_cells, dtype=torch.float64, device="cuda")
    cvw.residual(gm, cp, u, R, g, ws)
    assert cvw.poll_status(gm, ws) == 0
    return R.cpu().numpy(), g.cpu().numpy(), gm, cp, ws, u


# ---------------------------------------------------------------------------
# scalar data, periodic, degrees 4 and 8: candidates, gamma, alpha, residual
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("space", [0, 1])
@pytest.mark.parametrize("p,N", [(4, 33), (8, 17)])
def test_hp_scalar_sensor_and_residual(space, p, N):
    mesh = synth.segment_mesh(N)
    sp = build_space(mesh, p, space)
    U = nodal_interpolate(sp, [lambda x: np.sin(2 * np.pi * x[..., 0]) + (x[..., 0] > 0.63)])
    gm = cvw.Mesh(mesh, p, space)
    cp = cvw.make_params(ADV, cvw.F64)
    ws = cvw.alloc_workspace(gm, cp, 0)
    u = torch.from_numpy(U).cuda()
    cand = torch.empty((mesh.n_vertices, p), dtype=torch.float64, device="cuda")
    cvw.vertex_candidates(gm, cp, u, cand, ws)
    s = sp.to_cells(U)[0]
    c_o = o_cand(sp, s, ADV)
    # order k of a candidate sums (2/h)^k l_j^(k)(x_i) (s_j - s_0) over the
    # nodes with cancellation: each side's rounding is bounded by a few
    # (p + 1)^2 ulps of the sum of the magnitudes of its terms
    h = 1.0 / N
    mag = np.stack([np.abs(sp.ref.deriv(sp.ref.vertices[[lv]], (k,))[0]) @ np.abs(s - s[:, :1]).T * (2 / h) ** k
                    for lv in range(2) for k in range(1, p + 1)]).reshape(2, p, -1).max(axis=(0, 2))
    err = np.abs(cand.cpu().numpy() - c_o).max(axis=0)
    assert (err <= 8 * (p + 1) ** 2 * np.finfo(float).eps * mag).all(), (err, mag)
    g = torch.empty(mesh.n_cells, dtype=torch.float64, device="cuda")
    a = torch.empty((mesh.n_cells, p + 1), dtype=torch.float64, device="cuda")
    cvw.sensor(gm, cp, u, g, a, ws)
    g_o = sensor_gamma(sp, s, ADV)
    # gamma inherits that conditioning: at p = 8 the oracle itself moves gamma
    # by up to 5e-9 under a 4e-16 relative change of its input
    tol = 1e-9 if p <= 4 else 1e-7
    assert np.abs(g.cpu().numpy() - g_o).max() < tol
    assert (g_o < 0.5).any() and (g_o > 0.99).any()
    pg = None
    if space == 0:
        Uc = sp.to_cells(U)
        PGn = projected_gradient(sp, Uc)
        pg = np.einsum("qj,ejd->eqd", sp.ref.deriv(sp.ref.vol_pts, (0,)), PGn[0][sp.cell_dof])
    a_o = sc_weights(sp, s, g_o, ADV, pg)
    assert np.abs(a.cpu().numpy() - a_o).max() < tol * np.abs(a_o).max()
    R = torch.empty_like(u)
    cvw.residual(gm, cp, u, R, None, ws)
    assert cvw.poll_status(gm, ws) == 0
    assert rel_err(R.cpu().numpy(), o_residual(sp, U, ADV)) < 1e-9


# ---------------------------------------------------------------------------
# Euler, shock-tube data with ends, up to p = 32
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("space", [0, 1])
@pytest.mark.parametrize("p,N", [(1, 64), (2, 48), (4, 32), (8, 16), (16, 8), (32, 8)])
def test_hp_euler_shock_tube_residual(space, p, N):
    mesh, sp, U, prm = _euler_case(space, p, N)
    R, g, *_ = _gpu_residual(mesh, p, space, prm, U)
    R_o, parts = o_residual(sp, U, prm, return_parts=True)
    assert np.abs(g - parts["gamma"]).max() < 1e-9
    assert (parts["gamma"] < 0.5).sum() >= 1            # the cell of the jump is troubled
    assert rel_err(R, R_o) < 1e-9


@pytest.mark.parametrize("space", [0, 1])
@pytest.mark.parametrize("bc", ["walls", "outflow"])
def test_hp_euler_other_ends(space, bc):
    """Blast-wave data between two walls, and the shock tube with outflow at
    both ends, p = 3 (the degree the one-thread kernels would take for a
    scalar law: here the Euler equations route to the wave kernels)."""
    p, N = 3, 40
    if bc == "walls":
        mesh = synth.segment_mesh(N, periodic=False)
        sp = build_space(mesh, p, space, 3)
        U = nodal_interpolate(sp, [lambda x, c=c: synth.u0_blast_wave(x[..., 0])[c] for c in range(3)])
        prm = synth.blast_wave_params()
    else:
        mesh, sp, U, _ = _euler_case(space, p, N)
        prm = Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0), bc=(synth.BC_OUTFLOW, synth.BC_OUTFLOW))
    R, g, *_ = _gpu_residual(mesh, p, space, prm, U)
    R_o, parts = o_residual(sp, U, prm, return_parts=True)
    assert np.abs(g - parts["gamma"]).max() < 1e-9
    assert rel_err(R, R_o) < 1e-9


def test_hp_periodic_euler_and_scalar_ends():
    """A periodic 1D Euler state (smooth entropy wave, p = 5 DG) and scalar
    advection on a line with an inflow and an outflow end (p = 2 CG)."""
    mesh = synth.segment_mesh(24)
    sp = build_space(mesh, 5, 1, 3)
    U = nodal_interpolate(sp, [lambda x, c=c: np.asarray(synth.euler1d_conserved(
        1.0 + 0.2 * np.sin(2 * np.pi * x[..., 0]), 0.5, 1.0))[c] for c in range(3)])
    prm = Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0))
    R, g, *_ = _gpu_residual(mesh, 5, 1, prm, U)
    R_o, parts = o_residual(sp, U, prm, return_parts=True)
    assert np.abs(g - parts["gamma"]).max() < 1e-9
    assert rel_err(R, R_o) < 1e-9
    mesh = synth.segment_mesh(30, periodic=False)
    sp = build_space(mesh, 2, 0, 1)
    U = nodal_interpolate(sp, [lambda x: synth.u0_config1(x[..., 0])])
    prm = Params(flux=synth.ADVECT_CONST, flux_param=(1.0, 0, 0, 0), bc=(synth.BC_INFLOW, synth.BC_OUTFLOW),
                 bc_state=((0.5, 0, 0, 0), (0, 0, 0, 0)))
    R, g, *_ = _gpu_residual(mesh, 2, 0, prm, U)
    assert rel_err(R, o_residual(sp, U, prm)) < 1e-9


# ---------------------------------------------------------------------------
# whole runs
# ---------------------------------------------------------------------------
def _run(mesh, p, space, prm, U, dt, steps):
    gm = cvw.Mesh(mesh, p, space)
    cp = cvw.make_params(prm, cvw.F64)
    ws = cvw.alloc_workspace(gm, cp, 1)
    u = torch.from_numpy(np.ascontiguousarray(U)).cuda()
    cvw.step(gm, cp, u, dt, steps, ws)
    flags = cvw.poll_status(gm, ws)
    return u.cpu().numpy(), flags


@pytest.mark.parametrize("space", [0, 1])
def test_hp_shock_tube_run(space):
    """The modified shock tube (inflow at x = 0, wall at x = 1, jump at 0.25),
    p = 4 on 32 cells, 40 steps at CFL 0.1 / (2p + 1): L1 distance to the
    oracle's run below 1e-6 of the state's L1 norm per variable."""
    p, N, steps = 4, 32, 40
    mesh, sp, U, prm = _euler_case(space, p, N, x0=0.25)
    dt = 0.1 * (1.0 / N) / ((2 * p + 1) * 2.0)
    got, flags = _run(mesh, p, space, prm, U, dt, steps)
    assert flags == 0
    ref = np.asarray(U, np.float64).copy()
    for _ in range(steps):
        ref = rk3_step(sp, ref, dt, prm)
    d = np.abs(got - ref).reshape(3, -1).sum(1) / np.abs(ref).reshape(3, -1).sum(1)
    assert (d < 1e-6).all(), d
    assert np.abs(got - U).max() > 1e-3                  # the state moved


@pytest.mark.parametrize("space", [0, 1])
def test_hp_degree32_run_invariants(space):
    """p = 32 on eight elements (the paper's extreme case), a pressure pulse
    between walls, 10 steps of dt = 0.1 h / (lambda p^2): mass and energy stay
    constant to rounding, the density stays positive at the nodes, and the
    state stays within 1e-3 (L1, relative to the whole state) of the oracle's
    run."""
    p, N, steps = 32, 8, 10
    mesh = synth.segment_mesh(N, periodic=False)
    sp = build_space(mesh, p, space, 3)
    U = nodal_interpolate(sp, [lambda x, c=c: np.asarray(synth.euler1d_conserved(
        1.0, 0.0, np.where(np.abs(x[..., 0] - 0.5) < 0.2, 10.0, 1.0)))[c] for c in range(3)])
    prm = synth.blast_wave_params()
    dt = 0.1 * (1.0 / N) / (4.0 * p * p)                # explicit stability: dt ~ h / (lambda p^2)
    got, flags = _run(mesh, p, space, prm, U, dt, steps)
    assert flags == 0
    # totals with the exact mass matrix of the space
    from oracle.method import _cell_mass
    Me = _cell_mass(sp)

    def totals(V):
        Vc = sp.to_cells(V)
        return np.einsum("eij,vej->v", Me, Vc)
    t0, t1 = totals(U), totals(got)
    assert np.abs(t1[[0, 2]] - t0[[0, 2]]).max() < 1e-11 * np.abs(t0).max()
    assert sp.to_cells(got)[0].min() > 0
    ref = np.asarray(U, np.float64).copy()
    for _ in range(steps):
        ref = rk3_step(sp, ref, dt, prm)
    # relative to the whole state's L1 norm (the momentum starts at zero); the
    # oracle itself moves by up to 8e-6 under a 4e-16 change of its input here
    d = np.abs(got - ref).reshape(3, -1).sum(1) / np.abs(ref).sum()
    assert (d < 1e-3).all(), d
    assert np.abs(got - U).max() > 1e-2


# ---------------------------------------------------------------------------
# refusals (host checks before any launch)
# ---------------------------------------------------------------------------
def test_hp_refusals():
    mesh = synth.segment_mesh(8, periodic=False)
    gm = cvw.Mesh(mesh, 4, cvw.DG)
    u = torch.zeros(3 * 8 * 5, dtype=torch.float64, device="cuda")
    R = torch.empty_like(u)
    sod_p = synth.modified_sod_params()
    cases = [
        (cvw.make_params(sod_p, cvw.F32), cvw.EUNSUPPORTED, "float64"),
        (cvw.make_params(Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0)), cvw.F64), cvw.EINVAL, "boundary data"),
        (cvw.make_params(Params(flux=synth.ADVECT_CONST, bc=(synth.BC_WALL, synth.BC_OUTFLOW)), cvw.F64),
         cvw.EINVAL, "wall"),
        (cvw.make_params(Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0), bc=(synth.BC_INFLOW, synth.BC_WALL),
                                bc_state=((1.0, 0.0, -1.0, 0.0), (0, 0, 0, 0))), cvw.F64), cvw.EINVAL, "inflow"),
    ]
    lib = cvw.load()
    import ctypes as C
    for cp, code, word in cases:
        ws = torch.empty(max(cvw.workspace_bytes(gm, cp, 0), 256), dtype=torch.uint8, device="cuda")
        st = lib.cvw_residual(gm.handle, C.byref(cp), C.c_void_p(u.data_ptr()), C.c_void_p(R.data_ptr()), None,
                              C.c_void_p(ws.data_ptr()), ws.numel(), None)
        assert st == code, (word, st)
        assert word in lib.cvw_last_error().decode()
