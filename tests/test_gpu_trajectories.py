"""GPU: whole trajectories (many SSP-RK3 steps through cvw_step) against the
float64 oracle stepping from the same float32-rounded initial state.

The float32 state and the nonlinear sensor make trajectories drift apart by
rounding (a one-ulp change of a stored stage moves gamma_e of smooth cells
through third derivatives), so the comparison is by the L1 norm of the
difference relative to the L1 norm of the oracle's state, per variable, with
a bar of 1 %.  The 1D float64 workload is compared element by element.  The
full 64-instance ensemble is compared bit for bit with its instances stepped
one by one.
"""
import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space, nodal_interpolate, rk3_step
from oracle.method import wave_speed
from tests.parity_helpers import f32, euler_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import cvw  # noqa: E402


def _run_both(mesh, p, space, prm, U, dt, n_steps, nv=1, dtype=cvw.F32):
    sp = build_space(mesh, p, space, nv)
    gm = cvw.Mesh(mesh, p, space)
    cp = cvw.make_params(prm, dtype)
    ws = cvw.alloc_workspace(gm, cp, 1)
    tdt = torch.float64 if dtype == cvw.F64 else torch.float32
    u = torch.from_numpy(np.ascontiguousarray(U)).to(tdt).cuda()
    cvw.step(gm, cp, u, dt, n_steps, ws)
    assert cvw.poll_status(gm, ws) == 0
    Uo = np.asarray(U, np.float64).copy()
    for _ in range(n_steps):
        Uo = rk3_step(sp, Uo, dt, prm)
    return u.cpu().numpy().astype(np.float64), Uo


def _rel_l1(a, b, nv):
    a, b = a.reshape(nv, -1), b.reshape(nv, -1)
    return np.abs(a - b).sum(1) / np.abs(b).sum(1)


def test_config1_full_run_f64():
    """1D advection workload: 128 periodic cells, CG P2, float64, CFL 0.3
    (dt = 0.3 h / p), all 200 steps in one cvw_step call.  Element by element
    to 1e-4 of max |u|: the run itself is ill-conditioned (gamma_e of an
    exactly flat cell is 1, and near 0 for rounding noise, and the CG
    stabilisation of a flat cell next to the pulse's jump carries
    gamma_e P_h grad u), so that the oracle moves by 2e-2 under a 1e-15
    relative change of its initial data; the L1 bar is 1 %."""
    mesh = synth.segment_mesh(128)
    sp = build_space(mesh, 2, 0)
    U = nodal_interpolate(sp, [lambda x: synth.u0_config1(x[..., 0])])
    prm = Params(flux=synth.ADVECT_CONST, flux_param=(1.0, 0, 0, 0))
    got, ref = _run_both(mesh, 2, cvw.CG, prm, U, 0.3 * (1.0 / 128) / 2, 200, dtype=cvw.F64)
    assert np.abs(got - ref).max() <= 1e-4 * np.abs(ref).max()
    assert _rel_l1(got, ref, 1)[0] <= 1e-2


def test_dg_quad_euler_trajectory():
    """2D Euler, DG Q3 on 32 x 32 periodic quads, 20 steps, float32."""
    n, p = 32, 3
    mesh = synth.quad_mesh(n, n)
    sp = build_space(mesh, p, 1, 4)
    U = f32(euler_state(sp, k=6.0))
    prm = Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0))
    lam = wave_speed(prm, sp.to_cells(U), sp.node_coords()).max()
    dt = 0.1 * (1.0 / n) / ((2 * p + 1) * lam)
    got, ref = _run_both(mesh, p, cvw.DG, prm, U, dt, 20, nv=4)
    assert (_rel_l1(got, ref, 4) <= 1e-2).all(), _rel_l1(got, ref, 4)
    assert (_rel_l1(got, U, 4) > 0).all()        # the state moved


def test_cg_rotation_trajectory():
    """Solid-body rotation workload at 48 x 48 jittered Q2 cells, CG, 10 steps."""
    n, p = 48, 2
    mesh = synth.quad_mesh(n, n, jitter=0.1, seed=1002)
    sp = build_space(mesh, p, 0)
    U = f32(nodal_interpolate(sp, [lambda x: synth.u0_config2(x[..., 0], x[..., 1])]))
    prm = Params(flux=synth.ADVECT_ROT, flux_param=(0.5, 0.5, 1.0, 0.0))
    dt = 0.1 * (0.8 / n) / ((2 * p + 1) * 0.5 * np.sqrt(2.0))
    got, ref = _run_both(mesh, p, cvw.CG, prm, U, dt, 10)
    assert _rel_l1(got, ref, 1)[0] <= 1e-2


def test_tri_kpp_trajectory():
    """KPP workload at 32 x 32 squares split into 2048 jittered triangles, DG P3, 20 steps."""
    n, p = 32, 3
    mesh = synth.tri_mesh(n, n, -2.0, 2.0, -2.5, 1.5, jitter=0.1, seed=1003)
    sp = build_space(mesh, p, 1)
    U = f32(nodal_interpolate(sp, [lambda x: synth.u0_kpp(x[..., 0], x[..., 1])]))
    prm = Params(flux=synth.KPP, lambda_global=1.0)
    dt = 0.1 * (4.0 / n * 0.8) / (2 * p + 1)
    got, ref = _run_both(mesh, p, cvw.DG, prm, U, dt, 20)
    assert _rel_l1(got, ref, 1)[0] <= 1e-2


def test_full_ensemble_one_step_bitwise():
    """All 64 ensemble instances at their real sizes (64^2 .. 512^2 cells,
    41.6 M DOFs): one batched, graph-captured step equals each instance's own
    cvw_step bit for bit (both take the fused sensor pass)."""
    cases = []
    for inst in synth.config5_instances():
        mesh, p, prm, U, dt = synth.instance_case(inst)
        cases.append((cvw.Mesh(mesh, p, cvw.DG), cvw.make_params(prm), np.asarray(U, np.float32), dt))
    assert sum(c[2].size for c in cases) == 41609216
    singles = []
    for gm, cp, U, dt in cases:
        u = torch.from_numpy(U.copy()).cuda()
        ws = cvw.alloc_workspace(gm, cp, 1)
        cvw.step(gm, cp, u, dt, 1, ws)
        singles.append(u)
        del ws
    states = [torch.from_numpy(U.copy()).cuda() for _, _, U, _ in cases]
    b = cvw.Batch([(gm, cp, u, dt) for (gm, cp, _, dt), u in zip(cases, states)])
    ws = b.alloc_workspace()
    b.step(1, ws, use_graph=True)
    for k, (x, y) in enumerate(zip(states, singles)):
        assert torch.equal(x, y), k
    assert b.poll_status(ws) == 0
