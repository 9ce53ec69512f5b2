"""GPU parity: DG P1..P3 on jittered affine triangles (equispaced Lagrange
nodes, Stroud rule), HIP path through the C ABI vs the float64 oracle on
identical float32-rounded inputs.

The vertex pass and the sensor run in float64 on the device, so candidates
agree to the float32 rounding of the stored result (1e-6 of each multi-index
column) and gamma_e to 1e-5.  Residual: max |R_gpu - R_oracle| / max |R_oracle|
<= 1e-5 per variable; cells with |gamma_e - 0.9| < 1e-4 (a float decision of
the shock-capturing switch) are left out and counted.
"""
import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space, nodal_interpolate, residual as o_residual
from oracle.method import vertex_candidates as o_cand, cell_sensor as o_sensor, sc_weights as o_sc
from oracle.method import time_derivative, wave_speed, _cell_mass
from tests.parity_helpers import rel_err, f32, rough_scalar, euler_state, subset_ring

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import cvw  # noqa: E402

FLUXES = {
    "advect": Params(flux=synth.ADVECT_CONST, flux_param=(1.0, 0.5, 0, 0)),
    "rot": Params(flux=synth.ADVECT_ROT, flux_param=(0.5, 0.5, 1.0, 0)),
    "burgers": Params(flux=synth.BURGERS, flux_param=(1.0, 1.0, 0, 0)),
    "kpp": Params(flux=synth.KPP, lambda_global=1.0),
}
EULER = Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0))


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _mesh(nx=9, ny=7, seed=3):
    return synth.tri_mesh(nx, ny, jitter=0.1, seed=seed)


def _kpp_state(sp):
    xn = sp.node_coords()
    r = np.hypot(xn[..., 0] - 0.5, xn[..., 1] - 0.45)
    return (np.where(r <= 0.3, 3.5 * np.pi, 0.25 * np.pi)).ravel()


def test_connectivity_bit_exact():
    mesh = _mesh()
    sp = build_space(mesh, 2, 1)
    gm = cvw.Mesh(mesh, 2, cvw.DG)
    assert np.array_equal(gm.export(cvw.EXPORT_VTX_PTR), sp.patch_ptr)
    assert np.array_equal(gm.export(cvw.EXPORT_VTX_CELL), sp.patch_cell)
    assert np.array_equal(gm.export(cvw.EXPORT_VTX_LV), sp.patch_lv)
    assert np.array_equal(gm.export(cvw.EXPORT_NBR), sp.nbr.ravel())
    assert np.array_equal(gm.export(cvw.EXPORT_NBR_FACE), sp.nbr_face.ravel())
    assert set(np.diff(sp.patch_ptr)) == {6}


@pytest.mark.parametrize("p", [1, 2, 3])
def test_vertex_candidates(p):
    mesh = _mesh()
    sp = build_space(mesh, p, 1)
    u = f32(rough_scalar(sp, 1))
    prm = Params()
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 0)
    cand = torch.empty((mesh.n_vertices, len(sp.ks)), dtype=torch.float32, device="cuda")
    cvw.vertex_candidates(gm, cp, _dev(u), cand, ws)
    c_o = o_cand(sp, u, prm)
    got = cand.cpu().numpy()
    for t, k in enumerate(sp.ks):
        assert rel_err(got[:, t], c_o[:, t]) < 1e-6, k


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("sc_on", [1, 0])
def test_sensor_and_sc_weights(p, sc_on):
    mesh = _mesh()
    sp = build_space(mesh, p, 1)
    u = f32(rough_scalar(sp, 2) + _kpp_state(sp).reshape(sp.E, -1))
    prm = Params(sc_on=sc_on)
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 0)
    gam = torch.empty(sp.E, dtype=torch.float32, device="cuda")
    alpha = torch.empty((sp.E, len(sp.ref.vol_w)), dtype=torch.float32, device="cuda")
    cvw.sensor(gm, cp, _dev(u), gam, alpha, ws)
    c_o = o_cand(sp, u, prm)
    g_o, parts = o_sensor(sp, u, c_o, prm, return_parts=True)
    a_o = o_sc(sp, u, g_o, prm)
    g = gam.cpu().numpy()
    a = alpha.cpu().numpy()
    live = parts["n"] > 1e-6 * parts["n"].max()
    assert np.abs(g - g_o)[live].max() < 1e-5
    assert (g_o < 0.9).sum() >= 3
    ok = live & (np.abs(g_o - 0.9) >= 1e-4)
    assert np.abs(a - a_o)[ok].max() <= 1e-5 * np.abs(a_o).max()
    if not sc_on:
        assert np.all(a == 1.0)


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("flux", ["advect", "rot", "burgers", "kpp"])
def test_residual_scalar(p, flux):
    mesh = _mesh()
    sp = build_space(mesh, p, 1)
    prm = FLUXES[flux]
    U = f32(_kpp_state(sp) if flux == "kpp" else rough_scalar(sp, 3).ravel())
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 0)
    Ud = _dev(U)
    R = torch.empty_like(Ud)
    gam = torch.empty(sp.E, dtype=torch.float32, device="cuda")
    cvw.residual(gm, cp, Ud, R, gam, ws)
    R_o, parts = o_residual(sp, U, prm, return_parts=True)
    keep = np.repeat(np.abs(parts["gamma"] - 0.9) >= 1e-4, sp.ref.n_loc)
    assert keep.mean() > 0.9
    assert rel_err(R.cpu().numpy()[keep], R_o[keep]) < 1e-5


@pytest.mark.parametrize("p", [1, 2, 3])
def test_residual_euler(p):
    mesh = _mesh()
    sp = build_space(mesh, p, 1, 4)
    U = f32(euler_state(sp, k=6.0))
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(EULER)
    ws = cvw.alloc_workspace(gm, cp, 0)
    Ud = _dev(U)
    R = torch.empty_like(Ud)
    cvw.residual(gm, cp, Ud, R, None, ws)
    R_o, parts = o_residual(sp, U, EULER, return_parts=True)
    keep = np.repeat(np.abs(parts["gamma"] - 0.9) >= 1e-4, sp.ref.n_loc)
    R, R_o = R.cpu().numpy().reshape(4, -1), R_o.reshape(4, -1)
    for v in range(4):
        assert rel_err(R[v][keep], R_o[v][keep]) < 1e-5, v
    assert cvw.poll_status(gm, ws) == 0


@pytest.mark.parametrize("p", [1, 3])
def test_rk3_stages_and_step(p):
    """Each SSP-RK3 stage on the stage state the device stored (exact element
    mass inverse), then cvw_step equal to the stage sequence bit for bit."""
    mesh = _mesh()
    sp = build_space(mesh, p, 1)
    prm = FLUXES["kpp"]
    U = f32(_kpp_state(sp))
    dt = 0.1 * (1.0 / 9) / (2 * p + 1)
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 1)
    nk = len(sp.ks)
    cand = torch.zeros((mesh.n_vertices, nk), dtype=torch.float32, device="cuda")
    Un = _dev(U)
    cur = Un
    for (a0, b0) in ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0)):
        cvw.vertex_candidates(gm, cp, cur, cand, ws)
        out = torch.empty_like(Un)
        cvw.rk_stage(gm, cp, cur, cand, Un if a0 else None, out, dt, a0, b0, ws)
        us = cur.cpu().numpy().astype(np.float64)
        inc = b0 * dt * time_derivative(sp, us, prm)
        ref = a0 * U + b0 * us + inc
        uc = us.reshape(sp.E, -1)
        g_o = o_sensor(sp, uc, o_cand(sp, uc, prm), prm)
        near = np.repeat(np.abs(g_o - 0.9) < 1e-4, sp.ref.n_loc)
        err = np.abs(out.cpu().numpy().astype(np.float64) - ref)[~near].max()
        assert err <= 8 * np.finfo(np.float32).eps * np.abs(U).max() + 1e-5 * np.abs(inc).max()
        cur = out
    Ud = _dev(U)
    cvw.step(gm, cp, Ud, dt, 1, ws)
    assert torch.equal(Ud, cur)
    assert cvw.poll_status(gm, ws) == 0


def test_totals():
    mesh = _mesh()
    sp = build_space(mesh, 3, 1)
    U = f32(rough_scalar(sp, 4).ravel())
    gm = cvw.Mesh(mesh, 3, cvw.DG)
    cp = cvw.make_params(FLUXES["kpp"])
    ws = cvw.alloc_workspace(gm, cp, 1)
    t = cvw.totals(gm, cp, _dev(U), ws)
    ref = (_cell_mass(sp).sum(-1) * U.reshape(sp.E, -1)).sum()
    assert abs(t[0] - ref) <= 1e-6 * np.abs(U).max()


def test_full_size_config3_sampled_cells():
    """512 x 512 squares split into 524,288 jittered triangles on
    [-2,2] x [-2.5,1.5], DG P3, KPP: sampled cells (random, along the circle
    r = 1, at the periodic seams) against the oracle on the sub-mesh of their
    vertex rings."""
    n = 512
    mesh = synth.tri_mesh(n, n, -2.0, 2.0, -2.5, 1.5, jitter=0.1, seed=1003)
    p = 3
    gm = cvw.Mesh(mesh, p, cvw.DG)
    ref = build_space(synth.tri_mesh(1, 1, periodic=(False, False)), p, 1).ref
    X = mesh.cell_coords                                      # [E, 3, 2]
    lam = ref.nodes                                           # [10, 2] reference coords
    px = X[:, 0, None, 0] + (X[:, 1, None, 0] - X[:, 0, None, 0]) * lam[None, :, 0] \
        + (X[:, 2, None, 0] - X[:, 0, None, 0]) * lam[None, :, 1]
    py = X[:, 0, None, 1] + (X[:, 1, None, 1] - X[:, 0, None, 1]) * lam[None, :, 0] \
        + (X[:, 2, None, 1] - X[:, 0, None, 1]) * lam[None, :, 1]
    U = np.asarray(synth.u0_kpp(px, py), np.float32)          # [E, 10]
    prm = FLUXES["kpp"]
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 0)
    Ud = torch.from_numpy(U.reshape(-1)).cuda()
    R = torch.empty_like(Ud)
    cvw.residual(gm, cp, Ud, R, None, ws)
    R = R.cpu().numpy().reshape(-1, 10)
    E = mesh.n_cells
    cx, cy = X[:, :, 0].mean(1), X[:, :, 1].mean(1)
    rng = np.random.default_rng(0)
    ring = np.nonzero(np.abs(np.hypot(cx, cy) - 1.0) < 0.02)[0]
    cells = np.unique(np.concatenate([rng.choice(E, 16, replace=False), rng.choice(ring, 40, replace=False),
                                      [0, 1, 2 * n - 1, E - 1]]))
    sub, ids, pos = subset_ring(mesh, cells)
    sp = build_space(sub, p, 1)
    R_o, parts = o_residual(sp, U[ids].astype(np.float64).ravel(), prm, return_parts=True, allow_boundary=True)
    R_o = R_o.reshape(len(ids), 10)[pos]
    keep = np.abs(parts["gamma"][pos] - 0.9) >= 1e-4
    assert (parts["gamma"][pos] < 0.9).sum() >= 5
    assert rel_err(R[cells][keep], R_o[keep]) < 1e-5
