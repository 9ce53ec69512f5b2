"""GPU parity: 1D CG / DG elements through the C ABI vs the float64 oracle.

Float64 state (the 1D advection workload: 128 periodic cells, CG P2): the whole
path runs in float64, so the residual must agree to 1e-12 relative (sums of a
few dozen float64 terms).  Float32 state: 1e-5 as for the 2D paths.
"""
import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space, nodal_interpolate, residual as o_residual
from oracle.method import vertex_candidates as o_cand
from tests.parity_helpers import rel_err

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import cvw  # noqa: E402

ADV = Params(flux=synth.ADVECT_CONST, flux_param=(1.0, 0, 0, 0))
BUR = Params(flux=synth.BURGERS, flux_param=(1.0, 0, 0, 0))


def _state(sp, kind):
    if kind == "config1":
        return nodal_interpolate(sp, [lambda x: synth.u0_config1(x[..., 0])])
    return nodal_interpolate(sp, [lambda x: np.sin(2 * np.pi * x[..., 0]) + (x[..., 0] > 0.63)])


@pytest.mark.parametrize("space", [0, 1])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_seg_connectivity_and_candidates_f64(space, p):
    mesh = synth.segment_mesh(37)
    sp = build_space(mesh, p, space)
    U = _state(sp, "rough")
    gm = cvw.Mesh(mesh, p, space)
    if space == 0:
        assert np.array_equal(gm.export(cvw.EXPORT_CELL_DOF), sp.cell_dof.ravel())
    else:
        assert np.array_equal(gm.export(cvw.EXPORT_NBR), sp.nbr.ravel())
    cp = cvw.make_params(ADV, cvw.F64)
    ws = cvw.alloc_workspace(gm, cp, 0)
    cand = torch.empty((mesh.n_vertices, p), dtype=torch.float64, device="cuda")
    cvw.vertex_candidates(gm, cp, torch.from_numpy(U).cuda(), cand, ws)
    c_o = o_cand(sp, sp.to_cells(U)[0], ADV)
    assert rel_err(cand.cpu().numpy(), c_o) < 1e-12


@pytest.mark.parametrize("space", [0, 1])
@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("flux", ["advect", "burgers"])
def test_seg_residual_f64(space, p, flux):
    prm = ADV if flux == "advect" else BUR
    mesh = synth.segment_mesh(64)
    sp = build_space(mesh, p, space)
    U = _state(sp, "rough")
    gm = cvw.Mesh(mesh, p, space)
    cp = cvw.make_params(prm, cvw.F64)
    ws = cvw.alloc_workspace(gm, cp, 0)
    Ud = torch.from_numpy(U).cuda()
    R = torch.empty_like(Ud)
    gam = torch.empty(sp.E, dtype=torch.float64, device="cuda")
    cvw.residual(gm, cp, Ud, R, gam, ws)
    R_o, parts = o_residual(sp, U, prm, return_parts=True)
    assert (parts["gamma"] < 0.9).sum() >= 1
    assert np.abs(gam.cpu().numpy() - parts["gamma"]).max() < 1e-10
    assert rel_err(R.cpu().numpy(), R_o) < 1e-12


def test_config1_residual_full_size_f64():
    """128 periodic cells, CG P2, float64, pulse + cos^2 hump, constant advection."""
    mesh = synth.segment_mesh(128)
    sp = build_space(mesh, 2, 0)
    U = _state(sp, "config1")
    gm = cvw.Mesh(mesh, 2, cvw.CG)
    cp = cvw.make_params(ADV, cvw.F64)
    ws = cvw.alloc_workspace(gm, cp, 0)
    Ud = torch.from_numpy(U).cuda()
    R = torch.empty_like(Ud)
    cvw.residual(gm, cp, Ud, R, None, ws)
    R_o, parts = o_residual(sp, U, ADV, return_parts=True)
    assert (parts["gamma"] < 0.9).sum() >= 2
    assert rel_err(R.cpu().numpy(), R_o) < 1e-12
    alpha = torch.empty((sp.E, 3), dtype=torch.float64, device="cuda")
    gam = torch.empty(sp.E, dtype=torch.float64, device="cuda")
    cvw.sensor(gm, cp, Ud, gam, alpha, ws)
    assert np.abs(gam.cpu().numpy() - parts["gamma"]).max() < 1e-10
    assert np.abs(alpha.cpu().numpy() - parts["alpha"]).max() < 1e-10 * np.abs(parts["alpha"]).max()


@pytest.mark.parametrize("space", [0, 1])
def test_seg_residual_f32(space):
    mesh = synth.segment_mesh(50)
    sp = build_space(mesh, 3, space)
    U = _state(sp, "rough").astype(np.float32).astype(np.float64)
    gm = cvw.Mesh(mesh, 3, space)
    cp = cvw.make_params(BUR, cvw.F32)
    ws = cvw.alloc_workspace(gm, cp, 0)
    Ud = torch.from_numpy(U.astype(np.float32)).cuda()
    R = torch.empty_like(Ud)
    cvw.residual(gm, cp, Ud, R, None, ws)
    R_o, parts = o_residual(sp, U, BUR, return_parts=True)
    near = np.abs(parts["gamma"] - 0.9) < 1e-4
    keep = np.ones(R_o.size, bool)
    if space == 1:
        keep = np.repeat(~near, 4)
    else:
        keep[sp.cell_dof[near].ravel()] = False
    assert rel_err(R.cpu().numpy()[keep], R_o[keep]) < 1e-5
