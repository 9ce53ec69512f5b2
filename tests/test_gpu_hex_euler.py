"""GPU parity: the Euler equations on DG Q1 / Q2 hexahedra (periodic boxes),
HIP path through the C ABI vs the float64 oracle on identical float32-rounded
inputs.  The sensor field is the density; the SC weights and the viscosity
apply to all five variables; HLL at the faces.

Bars as for the scalar laws on hexahedra: residual max |R_gpu - R_oracle| per
variable <= 1e-5 of that variable's max |R_oracle| (cells with
|gamma_e - 0.9| < 1e-4 left out and counted), gamma_e to 1e-5, a stage to 8
ulp of |u| plus 1e-5 of the increment, ten SSP-RK3 steps within 1 % (L1) of
the oracle's run with every variable's total conserved to float32 rounding.
"""
import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space, rk3_step, residual as o_residual
from oracle.method import time_derivative, wave_speed
from tests.parity_helpers import rel_err, f32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import cvw  # noqa: E402

GAM = 1.4
PRM = Params(flux=synth.EULER, flux_param=(GAM, 0, 0, 0))


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _mesh(nx=5, ny=4, nz=3):
    return synth.hex_mesh(nx, ny, nz, x1=1.0, y1=0.8, z1=0.6)


def _state(sp, seed=0):
    """Smooth flow plus a ball of dense, high-pressure gas: [5, E, n_loc]."""
    xn = sp.node_coords()
    x, y, z = xn[..., 0], xn[..., 1], xn[..., 2]
    rng = np.random.default_rng(seed)
    a = rng.uniform(0.5, 1.5, size=3)
    ball = ((x - 0.45) ** 2 + (y - 0.4) ** 2 + (z - 0.3) ** 2) < 0.05
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x + a[0]) * np.cos(2 * np.pi * y / 0.8) + 1.0 * ball
    vx = 0.4 * np.cos(2 * np.pi * z / 0.6 + a[1])
    vy = -0.3 * np.sin(2 * np.pi * x)
    vz = 0.2 * np.sin(2 * np.pi * y / 0.8 + a[2])
    p = 1.0 + 0.2 * np.cos(2 * np.pi * (x + z / 0.6)) + 1.5 * ball
    En = p / (GAM - 1.0) + 0.5 * rho * (vx * vx + vy * vy + vz * vz)
    return np.stack([rho, rho * vx, rho * vy, rho * vz, En])


def _space(mesh, p):
    return build_space(mesh, p, 1, n_var=5)


@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("shape", [(5, 4, 3), (7, 3, 4)])
def test_residual(p, shape):
    mesh = _mesh(*shape)
    sp = _space(mesh, p)
    u = f32(_state(sp, 3))
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(PRM)
    ws = cvw.alloc_workspace(gm, cp, 0)
    R = torch.empty(u.size, dtype=torch.float32, device="cuda")
    gam = torch.empty(sp.E, dtype=torch.float32, device="cuda")
    cvw.residual(gm, cp, _dev(u), R, gam, ws)
    R_o, parts = o_residual(sp, u.ravel(), PRM, return_parts=True)
    keep = np.repeat(np.abs(parts["gamma"] - 0.9) >= 1e-4, sp.ref.n_loc)
    assert keep.mean() > 0.9
    assert (parts["gamma"] < 0.9).sum() >= 3 and (parts["alpha"] != 1).any()
    Rg = R.cpu().numpy().reshape(5, -1)
    Ro = R_o.reshape(5, -1)
    for v in range(5):
        assert rel_err(Rg[v][keep], Ro[v][keep]) < 1e-5, v
    assert np.abs(gam.cpu().numpy() - parts["gamma"]).max() < 1e-5
    assert cvw.poll_status(gm, ws) == 0


@pytest.mark.parametrize("p", [1, 2])
def test_constant_state(p):
    mesh = _mesh(3, 3, 3)
    sp = _space(mesh, p)
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(PRM)
    ws = cvw.alloc_workspace(gm, cp, 0)
    c = [1.2, 0.3, -0.2, 0.1, 2.5]
    u = torch.cat([torch.full((sp.E * sp.ref.n_loc,), v, dtype=torch.float32, device="cuda") for v in c])
    gam = torch.empty(sp.E, dtype=torch.float32, device="cuda")
    R = torch.empty_like(u)
    cvw.residual(gm, cp, u, R, gam, ws)
    assert torch.all(gam == 1.0)
    assert R.abs().max().item() < 1e-5


@pytest.mark.parametrize("p", [1, 2])
def test_rk_stage(p):
    mesh = _mesh()
    sp = _space(mesh, p)
    U = f32(_state(sp, 5)).ravel()
    Un = f32(U * (1.0 + 0.01 * np.sin(np.arange(U.size))))
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(PRM)
    ws = cvw.alloc_workspace(gm, cp, 0)
    cand = torch.empty((mesh.n_vertices, len(sp.ks)), dtype=torch.float32, device="cuda")
    dt = 1e-3
    for a0, b0 in ((0.0, 1.0), (0.75, 0.25)):
        cvw.vertex_candidates(gm, cp, _dev(U), cand, ws)
        out = torch.empty(U.size, dtype=torch.float32, device="cuda")
        cvw.rk_stage(gm, cp, _dev(U), cand, _dev(Un) if a0 else None, out, dt, a0, b0, ws)
        inc = b0 * dt * time_derivative(sp, U, PRM)
        ref = a0 * Un + b0 * U + inc
        err = np.abs(out.cpu().numpy().astype(np.float64) - ref).max()
        assert err <= 8 * np.finfo(np.float32).eps * np.abs(U).max() + 1e-5 * np.abs(inc).max(), (a0, b0)


@pytest.mark.parametrize("p", [1, 2])
def test_trajectory(p):
    """10 SSP-RK3 steps through cvw_step against the oracle's run."""
    mesh = _mesh(6, 5, 4)
    sp = _space(mesh, p)
    U = f32(_state(sp, 6)).ravel()
    lam = wave_speed(PRM, sp.to_cells(U), sp.node_coords()).max()
    dt = 0.1 * (0.6 / 4) / ((2 * p + 1) * lam)
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(PRM)
    ws = cvw.alloc_workspace(gm, cp, 1)
    u = _dev(U)
    cvw.step(gm, cp, u, dt, 10, ws)
    assert cvw.poll_status(gm, ws) == 0
    ref = U.copy()
    for _ in range(10):
        ref = rk3_step(sp, ref, dt, PRM)
    got = u.cpu().numpy().astype(np.float64)
    assert np.abs(got - ref).sum() / np.abs(ref).sum() <= 1e-2
    assert np.abs(got - U).max() > 1e-3
    w = np.tile(sp.ref.vol_w, sp.E)
    for v in range(5):
        g, u0 = got.reshape(5, -1)[v], U.reshape(5, -1)[v]
        assert abs((w * g).sum() - (w * u0).sum()) <= 1e-5 * (w * np.abs(u0)).sum() + 1e-6, v


@pytest.mark.parametrize("p", [1, 2])
def test_fixed_sensor_and_global_lambda(p):
    """The fixed sensor and a global wave speed: the viscosity takes the
    global speed, the faces keep HLL (as in the oracle)."""
    mesh = _mesh(4, 3, 3)
    sp = _space(mesh, p)
    prm = Params(flux=synth.EULER, flux_param=(GAM, 0, 0, 0), sensor=2, fixed_gamma=0.3, lambda_global=3.0)
    u = f32(_state(sp, 4))
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 0)
    R = torch.empty(u.size, dtype=torch.float32, device="cuda")
    cvw.residual(gm, cp, _dev(u), R, None, ws)
    Rg = R.cpu().numpy().reshape(5, -1)
    Ro = o_residual(sp, u.ravel(), prm).reshape(5, -1)
    for v in range(5):
        assert rel_err(Rg[v], Ro[v]) < 1e-5, v
