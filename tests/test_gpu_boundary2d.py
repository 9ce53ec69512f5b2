"""GPU parity: DG quadrilaterals and triangles with boundary faces, each face
with its own kind (inflow state, reflecting wall, outflow) and exterior state
(the setting of the double Mach reflection run, Sec. 5.4), through the C ABI
vs the float64 oracle on the same float32-rounded inputs.

Bars as for the closed meshes: max |R_gpu - R_oracle| / max |R_oracle| <=
1e-5 per variable, cells with |gamma_e - 0.9| < 1e-4 (a float decision of
the shock-capturing switch) left out and counted; whole runs by their
conserved totals and their L1 distance to the oracle's run.
"""
import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space, rk3_step
from oracle import residual as o_residual
from oracle.method import boundary_faces, face_geometry, wave_speed
from tests.parity_helpers import rel_err, f32, euler_state, rough_scalar

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import cvw  # noqa: E402

G = 1.4
INFLOW = np.array([1.1, 0.3, 0.05, 0.9 / 0.4 + 0.5 * (0.3 ** 2 + 0.05 ** 2) / 1.1])


def _mesh(cell, nx=12, ny=9):
    if cell == "quad":
        return synth.quad_mesh(nx, ny, periodic=(False, False))
    return synth.tri_mesh(nx, ny, jitter=0.1, seed=7, periodic=(False, False))


def _side_kinds(sp, west=synth.BC_INFLOW, east=synth.BC_OUTFLOW, other=synth.BC_WALL):
    """Kind of every boundary face by its outward normal: x < 0 west, x > 0
    east, the rest (y faces) `other`."""
    cells, faces = boundary_faces(sp)
    kinds = np.empty(len(cells), np.int32)
    for b, (e, f) in enumerate(zip(cells, faces)):
        n = face_geometry(sp, f)[0][e]
        kinds[b] = west if n[0] < -0.7 else (east if n[0] > 0.7 else other)
    return kinds


def _run_residual(mesh, p, sp, prm, U):
    gm = cvw.Mesh(mesh, p, cvw.DG)
    assert gm.info["n_bfaces"] == len(boundary_faces(sp)[0])
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 0)
    u = torch.from_numpy(np.ascontiguousarray(U, np.float32)).cuda()
    R = torch.empty_like(u)
    cvw.residual(gm, cp, u, R, None, ws)
    assert cvw.poll_status(gm, ws) == 0
    return R.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("cell", ["quad", "tri"])
def test_boundary_face_export(cell):
    mesh = _mesh(cell, 5, 4)
    sp = build_space(mesh, 2, 1)
    gm = cvw.Mesh(mesh, 2, cvw.DG)
    c, f = boundary_faces(sp)
    assert np.array_equal(gm.export(cvw.EXPORT_BFACE).reshape(-1, 2), np.stack([c, f], 1))


@pytest.mark.parametrize("cell", ["quad", "tri"])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_euler_residual_with_boundary_faces(cell, p):
    mesh = _mesh(cell)
    sp = build_space(mesh, p, 1, 4)
    U = f32(euler_state(sp, k=6.0))
    kinds = _side_kinds(sp)
    prm = Params(flux=synth.EULER, flux_param=(G, 0, 0, 0), bc_face_kind=kinds,
                 bc_face_state=np.tile(INFLOW, (len(kinds), 1)))
    R = _run_residual(mesh, p, sp, prm, U)
    R_o, parts = o_residual(sp, U, prm, return_parts=True)
    keep = np.repeat(np.abs(parts["gamma"] - 0.9) >= 1e-4, sp.ref.n_loc)
    assert keep.mean() > 0.95
    R, R_o = R.reshape(4, -1), R_o.reshape(4, -1)
    for v in range(4):
        assert rel_err(R[v][keep], R_o[v][keep]) < 1e-5, v
    # the boundary terms matter: without them the residual differs
    R_x = o_residual(sp, U, Params(flux=synth.EULER, flux_param=(G, 0, 0, 0)), allow_boundary=True).reshape(4, -1)
    assert np.abs(R_x - R_o).max() > 1e-2 * np.abs(R_o).max()


@pytest.mark.parametrize("cell", ["quad", "tri"])
@pytest.mark.parametrize("p", [1, 3])
def test_scalar_residual_with_boundary_faces(cell, p):
    """Advection through an inflow (west) and outflow (east) boundary, the y
    faces outflow too (a wall on a scalar law is outflow)."""
    mesh = _mesh(cell)
    sp = build_space(mesh, p, 1)
    U = f32(rough_scalar(sp, 3)).ravel()
    kinds = _side_kinds(sp, other=synth.BC_WALL)
    prm = Params(flux=synth.ADVECT_CONST, flux_param=(1.0, 0.4, 0, 0), bc_face_kind=kinds,
                 bc_face_state=np.full((len(kinds), 1), 0.7))
    R = _run_residual(mesh, p, sp, prm, U)
    prm_o = Params(flux=synth.ADVECT_CONST, flux_param=(1.0, 0.4, 0, 0),
                   bc_face_kind=np.where(kinds == synth.BC_WALL, synth.BC_OUTFLOW, kinds),
                   bc_face_state=np.full((len(kinds), 1), 0.7))
    R_o, parts = o_residual(sp, U, prm_o, return_parts=True)
    keep = np.repeat(np.abs(parts["gamma"] - 0.9) >= 1e-4, sp.ref.n_loc)
    assert rel_err(R[keep], R_o[keep]) < 1e-5


@pytest.mark.parametrize("cell", ["quad", "tri"])
def test_walls_conserve_and_run_tracks_the_oracle(cell):
    """Euler between four walls, DG P2 on quads and on jittered triangles,
    10 steps in one cvw_step call:
    mass and energy totals constant to float32 rounding (the wall flux of
    both is zero), the state within 1 % (L1, per variable) of the oracle's
    run, as for the periodic trajectories."""
    p, steps, n = 2, 10, 10
    mesh = _mesh(cell, n, 8)
    sp = build_space(mesh, p, 1, 4)
    # smooth enough that the float64 run keeps density and pressure positive
    # on the 160 triangles (at k = 6 the density turns negative within 3 steps)
    U = f32(euler_state(sp, k=2.0))
    nb = len(boundary_faces(sp)[0])
    prm = Params(flux=synth.EULER, flux_param=(G, 0, 0, 0), bc_face_kind=np.full(nb, synth.BC_WALL))
    lam = wave_speed(prm, sp.to_cells(U), sp.node_coords()).max()
    dt = 0.1 * (1.0 / n) / ((2 * p + 1) * lam) / (2 if cell == "tri" else 1)
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 1)
    u = torch.from_numpy(np.ascontiguousarray(U, np.float32)).cuda()
    t0 = cvw.totals(gm, cp, u, ws, n_var=4)
    cvw.step(gm, cp, u, dt, steps, ws)
    assert cvw.poll_status(gm, ws) == 0
    t1 = cvw.totals(gm, cp, u, ws, n_var=4)
    for v in (0, 3):
        assert abs(t1[v] - t0[v]) <= 2e-6 * abs(t0[v]), (v, t0, t1)
    ref = np.asarray(U, np.float64).copy()
    for _ in range(steps):
        ref = rk3_step(sp, ref, dt, prm)
    got = u.cpu().numpy().astype(np.float64)
    d = np.abs(got - ref).reshape(4, -1).sum(1) / np.abs(ref).reshape(4, -1).sum(1)
    assert (d <= 1e-2).all(), d
    assert (np.abs(got - U).reshape(4, -1).sum(1) > 0).all()


@pytest.mark.parametrize("cell", ["quad", "tri"])
def test_single_open_cell(cell):
    """The degenerate open mesh: one quadrilateral (two triangles), every
    face but the triangles' diagonal on the boundary, every vertex patch one
    cell (two at the ends of the diagonal); Euler with outflow (west),
    inflow (east) and walls (south, north)."""
    mesh = _mesh(cell, 1, 1)
    sp = build_space(mesh, 2, 1, 4)
    U = f32(euler_state(sp, k=6.0))
    kinds = _side_kinds(sp, west=synth.BC_OUTFLOW, east=synth.BC_INFLOW)
    assert len(kinds) == 4
    prm = Params(flux=synth.EULER, flux_param=(G, 0, 0, 0), bc_face_kind=kinds,
                 bc_face_state=np.tile(INFLOW, (len(kinds), 1)))
    R = _run_residual(mesh, 2, sp, prm, U)
    R_o, parts = o_residual(sp, U, prm, return_parts=True)
    keep = np.repeat(np.abs(parts["gamma"] - 0.9) >= 1e-4, sp.ref.n_loc)
    R, R_o = R.reshape(4, -1), R_o.reshape(4, -1)
    for v in range(4):
        assert rel_err(R[v][keep], R_o[v][keep]) < 1e-5, v


def test_missing_boundary_data_is_refused():
    mesh = _mesh("quad", 6, 5)
    gm = cvw.Mesh(mesh, 2, cvw.DG)
    cp = cvw.make_params(Params(flux=synth.EULER, flux_param=(G, 0, 0, 0)))
    ws = cvw.alloc_workspace(gm, cp, 0)
    u = torch.zeros(4 * mesh.n_cells * 9, dtype=torch.float32, device="cuda")
    with pytest.raises(cvw.CvwError, match="boundary data"):
        cvw.residual(gm, cp, u, torch.empty_like(u), None, ws)
