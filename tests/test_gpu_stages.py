"""GPU parity of the Runge-Kutta stages on the CG paths (consistent mass,
inverted on the device by preconditioned CG) and the 1D DG path (exact
diagonal mass), through the C ABI vs the float64 oracle.

Each SSP-RK3 stage is compared on the stage state the device stored, so that
rounding of one stage is not propagated into the next:
    expected = a0 u_n + b0 u_s + b0 dt L(u_s),  L = -M^{-1} R  (oracle: sparse LU).
Bars: float64 1e-11 of the increment b0 dt L plus 4 ulp of |u|; float32 2e-5 of
the increment plus 8 ulp of |u| (the residual itself agrees to 1e-5 of max |R|,
and M^{-1} couples the DOFs).
"""
import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space, nodal_interpolate, rk3_step
from oracle.method import time_derivative, _cell_mass
from tests.parity_helpers import f32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import cvw  # noqa: E402

ADV = Params(flux=synth.ADVECT_CONST, flux_param=(1.0, 0, 0, 0))
BUR = Params(flux=synth.BURGERS, flux_param=(1.0, 0, 0, 0))
ROT = Params(flux=synth.ADVECT_ROT, flux_param=(0.5, 0.5, 1.0, 0.0), sc_on=0)
BUR2 = Params(flux=synth.BURGERS, flux_param=(1.0, 1.0, 0, 0), sc_on=0)
STAGES = ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0))


def _seg_state(sp):
    return nodal_interpolate(sp, [lambda x: np.sin(2 * np.pi * x[..., 0]) + (x[..., 0] > 0.63)])


def _quad_state(sp, seed):
    return f32(nodal_interpolate(sp, [lambda x: 0.1 * synth.smooth_field(x[..., 0], x[..., 1], seed)
                                      + 1.5 * ((x[..., 0] - 0.45) ** 2 + (x[..., 1] - 0.55) ** 2 < 0.07)]))


def _run_stages(sp, gm, prm, cp, U, dt, torch_dtype, nk, rel, ulps):
    ws = cvw.alloc_workspace(gm, cp, 0)
    eps = np.finfo(np.float64 if torch_dtype == torch.float64 else np.float32).eps
    cand = torch.zeros((gm.info["n_vertices"], nk), dtype=torch_dtype, device="cuda")
    Un = torch.from_numpy(U.astype(np.float64 if torch_dtype == torch.float64 else np.float32)).cuda()
    cur = Un
    worst = 0.0
    for (a0, b0) in STAGES:
        cvw.vertex_candidates(gm, cp, cur, cand, ws)
        out = torch.empty_like(Un)
        cvw.rk_stage(gm, cp, cur, cand, Un if a0 else None, out, dt, a0, b0, ws)
        us = cur.cpu().numpy().astype(np.float64)
        inc = b0 * dt * time_derivative(sp, us, prm)
        ref = a0 * U + b0 * us + inc
        err = np.abs(out.cpu().numpy().astype(np.float64) - ref).max()
        bar = ulps * eps * np.abs(U).max() + rel * np.abs(inc).max()
        worst = max(worst, err / bar)
        assert err <= bar, (a0, b0, err, np.abs(inc).max())
        cur = out
    assert cvw.poll_status(gm, ws) == 0
    return worst


@pytest.mark.parametrize("space", [0, 1])
@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("flux", ["advect", "burgers"])
def test_seg_stages_f64(space, p, flux):
    prm = ADV if flux == "advect" else BUR
    mesh = synth.segment_mesh(64)
    sp = build_space(mesh, p, space)
    U = _seg_state(sp)
    gm = cvw.Mesh(mesh, p, space)
    cp = cvw.make_params(prm, cvw.F64)
    dt = 0.1 / 64 / (2 * p + 1) / 2.0
    _run_stages(sp, gm, prm, cp, U, dt, torch.float64, p, 1e-11, 4)


@pytest.mark.parametrize("space", [0, 1])
def test_seg_stages_f32(space):
    p = 2
    mesh = synth.segment_mesh(64)
    sp = build_space(mesh, p, space)
    U = f32(_seg_state(sp))
    gm = cvw.Mesh(mesh, p, space)
    prm = Params(flux=synth.BURGERS, flux_param=(1.0, 0, 0, 0), sc_on=0)
    cp = cvw.make_params(prm, cvw.F32)
    dt = 0.1 / 64 / (2 * p + 1) / 2.0
    _run_stages(sp, gm, prm, cp, U, dt, torch.float32, p, 2e-5, 8)


@pytest.mark.parametrize("space", [0, 1])
def test_seg_config1_steps_f64(space):
    """Ten SSP-RK3 steps of the 1D advection workload (128 periodic cells, P2,
    float64) through cvw_step vs the oracle's rk3_step."""
    mesh = synth.segment_mesh(128)
    sp = build_space(mesh, 2, space)
    U = nodal_interpolate(sp, [lambda x: synth.u0_config1(x[..., 0])])
    gm = cvw.Mesh(mesh, 2, space)
    cp = cvw.make_params(ADV, cvw.F64)
    ws = cvw.alloc_workspace(gm, cp, 1)
    dt = 0.1 / 128 / 5
    Ud = torch.from_numpy(U.copy()).cuda()
    cvw.step(gm, cp, Ud, dt, 10, ws)
    Uo = U.copy()
    for _ in range(10):
        Uo = rk3_step(sp, Uo, dt, ADV)
    assert np.abs(Ud.cpu().numpy() - Uo).max() <= 1e-10 * np.abs(U).max()
    assert cvw.poll_status(gm, ws) == 0


@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("flux", ["rot", "burgers"])
def test_cg_quad_stages(p, flux):
    prm = ROT if flux == "rot" else BUR2
    mesh = synth.quad_mesh(13, 11, jitter=0.1, seed=7)
    sp = build_space(mesh, p, 0)
    U = _quad_state(sp, 3)
    gm = cvw.Mesh(mesh, p, cvw.CG)
    cp = cvw.make_params(prm)
    dt = 0.1 / 13 / (2 * p + 1) / 1.5
    nk = (p + 1) * (p + 2) // 2 - 1
    _run_stages(sp, gm, prm, cp, U, dt, torch.float32, nk, 2e-5, 8)


def test_cg_quad_step_is_the_stages_and_conserves():
    """cvw_step equals the stage sequence bit for bit, and keeps the total
    integral sum_I u_I int phi_I (the residual sums to zero)."""
    p = 2
    mesh = synth.quad_mesh(24, 24, jitter=0.1, seed=1002)
    sp = build_space(mesh, p, 0)
    U = f32(nodal_interpolate(sp, [lambda x: synth.u0_config2(x[..., 0], x[..., 1])]))
    gm = cvw.Mesh(mesh, p, cvw.CG)
    prm = Params(flux=synth.ADVECT_ROT, flux_param=(0.5, 0.5, 1.0, 0.0))
    cp = cvw.make_params(prm)
    dt = 0.1 / 24 / 5 / 1.5
    ws = cvw.alloc_workspace(gm, cp, 1)
    Ud = torch.from_numpy(U.astype(np.float32)).cuda()
    cvw.step(gm, cp, Ud, dt, 3, ws)
    V = torch.from_numpy(U.astype(np.float32)).cuda()
    cand = torch.zeros((mesh.n_vertices, 5), dtype=torch.float32, device="cuda")
    for _ in range(3):
        V1, V2 = torch.empty_like(V), torch.empty_like(V)
        for (us, un, uo, a0, b0) in ((V, None, V1, 0.0, 1.0), (V1, V, V2, 0.75, 0.25),
                                     (V2, V, V, 1.0 / 3.0, 2.0 / 3.0)):
            cvw.vertex_candidates(gm, cp, us, cand, ws)
            cvw.rk_stage(gm, cp, us, cand, un, uo, dt, a0, b0, ws)
    assert torch.equal(Ud, V)
    lump = np.bincount(sp.cell_dof.ravel(), _cell_mass(sp).sum(-1).ravel(), minlength=sp.n_dof)
    t0 = (lump * U).sum()
    t1 = (lump * Ud.cpu().numpy().astype(np.float64)).sum()
    assert abs(t1 - t0) <= 1e-5 * (lump * np.abs(U)).sum()
    assert cvw.poll_status(gm, ws) == 0
