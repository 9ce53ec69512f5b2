"""GPU parity: DG on congruent axis-aligned quadrilaterals (HIP path through the
C ABI vs the float64 oracle on identical float32-rounded inputs).

Tolerances: the residual is compared as max |R_gpu - R_oracle| / max |R_oracle|
per variable <= 1e-5 (float32 arithmetic on O(10..100)-term sums with the
sensor and weights kept to ~1e-6 by float64 reductions).  gamma_e is compared
in absolute value (it lives in [0, 1]) on cells whose element semi-norm is not
at round-off level; the shock-capturing switch gamma_e < 0.9 is a float
decision, so cells with |gamma_e - 0.9| < 1e-4 are left out of the element-by-
element comparison and counted.
"""
import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space, nodal_interpolate, residual as o_residual, rk3_step
from oracle.method import vertex_candidates as o_cand, cell_sensor as o_sensor, sc_weights as o_sc
from tests.parity_helpers import rel_err, f32, rough_scalar, euler_state, subset_ring

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import cvw  # noqa: E402

EULER = Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0))
SCALARS = {
    "advect": Params(flux=synth.ADVECT_CONST, flux_param=(1.0, 0.5, 0, 0)),
    "burgers": Params(flux=synth.BURGERS, flux_param=(1.0, 1.0, 0, 0)),
    "kpp": Params(flux=synth.KPP, lambda_global=1.0),
}


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _setup(nx, ny, p, nv=1):
    mesh = synth.quad_mesh(nx, ny)
    sp = build_space(mesh, p, 1, nv)
    gm = cvw.Mesh(mesh, p, cvw.DG)
    return mesh, sp, gm


def test_connectivity_bit_exact():
    mesh, sp, gm = _setup(12, 10, 2)
    assert np.array_equal(gm.export(cvw.EXPORT_VTX_PTR), sp.patch_ptr)
    assert np.array_equal(gm.export(cvw.EXPORT_VTX_CELL), sp.patch_cell)
    assert np.array_equal(gm.export(cvw.EXPORT_VTX_LV), sp.patch_lv)
    assert np.array_equal(gm.export(cvw.EXPORT_NBR), sp.nbr.ravel())
    assert np.array_equal(gm.export(cvw.EXPORT_NBR_FACE), sp.nbr_face.ravel())
    assert gm.info["uniform"] == 1


@pytest.mark.parametrize("p", [1, 2, 3])
def test_vertex_candidates(p):
    mesh, sp, gm = _setup(13, 11, p)          # ragged: 143 cells / vertices
    u = f32(rough_scalar(sp, 1))
    prm = Params()
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 0)
    cand = torch.empty((mesh.n_vertices, len(sp.ks)), dtype=torch.float32, device="cuda")
    cvw.vertex_candidates(gm, cp, _dev(u), cand, ws)
    c_o = o_cand(sp, u, prm)
    # float32 bound per multi-index k: the derivative is a sum of n_loc products
    # of table entries and nodal values, so its rounding error scales with
    # sum_j |D^k phi_j(x_i)| max|u| (large for the third derivatives)
    h = 1.0 / 13, 1.0 / 11
    got = cand.cpu().numpy()
    for t, k in enumerate(sp.ks):
        cond = np.abs(sp.ref.deriv(sp.ref.vertices, k)).sum(1).max() * (2 / h[0]) ** k[0] * (2 / h[1]) ** k[1]
        bound = 64 * np.finfo(np.float32).eps * cond * np.abs(u).max()
        assert np.abs(got[:, t] - c_o[:, t]).max() < bound, (k, np.abs(got[:, t] - c_o[:, t]).max(), bound)
    assert rel_err(got[:, :2], c_o[:, :2]) < 1e-5


@pytest.mark.parametrize("p", [1, 2, 3])
def test_vertex_candidates_structured_waves(p):
    """128 x 128 periodic quads: the 64-vertex waves away from the periodic
    seam see their k-th patch cell at one corner for every vertex and take the
    vertex pass's variants with the mirroring fixed at compile time; waves
    holding a seam vertex take the run-time variant.  Same bound as above."""
    n = 128
    mesh, sp, gm = _setup(n, n, p)
    u = f32(rough_scalar(sp, 1))
    prm = Params()
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 0)
    cand = torch.empty((mesh.n_vertices, len(sp.ks)), dtype=torch.float32, device="cuda")
    cvw.vertex_candidates(gm, cp, _dev(u), cand, ws)
    c_o = o_cand(sp, u, prm)
    got = cand.cpu().numpy()
    h = 1.0 / n
    for t, k in enumerate(sp.ks):
        cond = np.abs(sp.ref.deriv(sp.ref.vertices, k)).sum(1).max() * (2 / h) ** (k[0] + k[1])
        bound = 64 * np.finfo(np.float32).eps * cond * np.abs(u).max()
        assert np.abs(got[:, t] - c_o[:, t]).max() < bound, (k, np.abs(got[:, t] - c_o[:, t]).max(), bound)
    assert rel_err(got[:, :2], c_o[:, :2]) < 1e-5


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("sc_on", [1, 0])
def test_sensor_and_sc_weights(p, sc_on):
    mesh, sp, gm = _setup(13, 11, p)
    u = f32(rough_scalar(sp, 2))
    prm = Params(sc_on=sc_on)
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 0)
    gam = torch.empty(sp.E, dtype=torch.float32, device="cuda")
    alpha = torch.empty((sp.E, sp.ref.n_loc), dtype=torch.float32, device="cuda")
    cvw.sensor(gm, cp, _dev(u), gam, alpha, ws)
    c_o = o_cand(sp, u, prm)
    g_o, parts = o_sensor(sp, u, c_o, prm, return_parts=True)
    a_o, ap = o_sc(sp, u, g_o, prm, return_parts=True)
    g = gam.cpu().numpy()
    a = alpha.cpu().numpy()
    live = parts["n"] > 1e-6 * parts["n"].max()
    assert np.abs(g - g_o)[live].max() < 2e-5
    assert (g_o < 0.9).sum() >= 3          # the data exercises the sensor
    near = np.abs(g_o - 0.9) < 1e-4
    ok = live & ~near
    assert np.abs(a - a_o)[ok].max() <= 1e-5 * np.abs(a_o).max()
    if sc_on == 0:
        assert (a == 1.0).all()


def _residual_case(nx, ny, p, prm, nv, U):
    mesh = synth.quad_mesh(nx, ny)
    sp = build_space(mesh, p, 1, nv)
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 0)
    Ud = _dev(U)
    R = torch.empty_like(Ud)
    gam = torch.empty(sp.E, dtype=torch.float32, device="cuda")
    cvw.residual(gm, cp, Ud, R, gam, ws)
    R_o, parts = o_residual(sp, U, prm, return_parts=True)
    return sp, R.cpu().numpy(), R_o, gam.cpu().numpy(), parts


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("flux", list(SCALARS))
def test_residual_scalar(p, flux):
    prm = SCALARS[flux]
    mesh = synth.quad_mesh(13, 11)
    sp = build_space(mesh, p, 1)
    if flux == "kpp":
        U = f32(2.0 + 2.5 * (rough_scalar(sp, 3) > 0.8)).ravel()
    else:
        U = f32(rough_scalar(sp, 3)).ravel()
    sp, R, R_o, g, parts = _residual_case(13, 11, p, prm, 1, U)
    keep = np.repeat(np.abs(parts["gamma"] - 0.9) >= 1e-4, sp.ref.n_loc)
    assert keep.mean() > 0.95
    assert rel_err(R[keep], R_o[keep]) < 1e-5


@pytest.mark.parametrize("p", [1, 2, 3])
def test_residual_euler(p):
    mesh = synth.quad_mesh(16, 12)
    sp = build_space(mesh, p, 1, 4)
    U = f32(euler_state(sp, k=6.0))
    sp, R, R_o, g, parts = _residual_case(16, 12, p, EULER, 4, U)
    assert (parts["gamma"] < 0.9).sum() >= 3
    keep = np.repeat(np.abs(parts["gamma"] - 0.9) >= 1e-4, sp.ref.n_loc)
    R = R.reshape(4, -1)
    R_o = R_o.reshape(4, -1)
    for v in range(4):
        assert rel_err(R[v][keep], R_o[v][keep]) < 1e-5, v


def test_residual_deterministic_and_gamma_out():
    mesh = synth.quad_mesh(16, 12)
    sp = build_space(mesh, 3, 1, 4)
    U = f32(euler_state(sp, k=6.0))
    gm = cvw.Mesh(mesh, 3, cvw.DG)
    cp = cvw.make_params(EULER)
    ws = cvw.alloc_workspace(gm, cp, 0)
    Ud = _dev(U)
    R1, R2 = torch.empty_like(Ud), torch.empty_like(Ud)
    cvw.residual(gm, cp, Ud, R1, None, ws)
    cvw.residual(gm, cp, Ud, R2, None, ws)
    assert torch.equal(R1, R2)


@pytest.mark.parametrize("p", [1, 3])
def test_mesh_in_caller_buffer_matches(p):
    """A mesh built into a caller-owned device buffer (cvw_mesh_plan /
    cvw_mesh_build_in) gives bitwise the residual of a library-allocated one."""
    mesh = synth.quad_mesh(16, 12)
    sp = build_space(mesh, p, 1, 4)
    U = _dev(f32(euler_state(sp, k=6.0)))
    cp = cvw.make_params(EULER)
    nbytes = cvw.mesh_plan(mesh, p, cvw.DG)
    buf = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
    ga = cvw.Mesh(mesh, p, cvw.DG)
    gb = cvw.Mesh(mesh, p, cvw.DG, device_buffer=buf)
    Ra, Rb = torch.empty_like(U), torch.empty_like(U)
    cvw.residual(ga, cp, U, Ra, None, cvw.alloc_workspace(ga, cp, 0))
    cvw.residual(gb, cp, U, Rb, None, cvw.alloc_workspace(gb, cp, 0))
    assert torch.equal(Ra, Rb)
    with pytest.raises(cvw.CvwError):
        cvw.Mesh(mesh, p, cvw.DG, device_buffer=buf[: nbytes // 2])


@pytest.mark.parametrize("flux", ["euler", "burgers"])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_wide_addressing_path_matches(p, flux, monkeypatch):
    """The 64-bit addressed cell pass (taken for states over 4 GiB) computes
    bitwise what the 32-bit buffer-addressed pass computes: residual, gamma
    and a stage update, forced here on a small mesh."""
    mesh = synth.quad_mesh(16, 12)
    if flux == "euler":
        sp = build_space(mesh, p, 1, 4)
        U = f32(euler_state(sp, k=6.0))
        prm = EULER
    else:
        sp = build_space(mesh, p, 1)
        U = f32(rough_scalar(sp, 3))
        prm = SCALARS["burgers"]
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 0)
    Ud = _dev(U)
    cand = torch.empty((mesh.n_vertices, len(sp.ks)), dtype=torch.float32, device="cuda")
    cvw.vertex_candidates(gm, cp, Ud, cand, ws)

    def run():
        R = torch.empty_like(Ud)
        g = torch.empty(sp.E, dtype=torch.float32, device="cuda")
        cvw.residual(gm, cp, Ud, R, g, ws)
        S = torch.empty_like(Ud)
        cvw.rk_stage(gm, cp, Ud, cand, Ud, S, 1e-4, 0.75, 0.25, ws)
        torch.cuda.synchronize()
        return R, g, S

    a = run()
    monkeypatch.setenv("CVW_WIDE_ADDRESSING", "1")
    b = run()
    monkeypatch.delenv("CVW_WIDE_ADDRESSING")
    for x, y in zip(a, b):
        assert torch.equal(x, y)


@pytest.mark.parametrize("sensor", ["fixed", "plain"])
@pytest.mark.parametrize("p", [1, 2, 3])
def test_rk3_stages_match_oracle(p, sensor):
    """The three SSP-RK3 stages (Shu-Osher form), SC off, stable dt.  Each
    stage is compared with the oracle on the stage state the device actually
    stored (float32), so that one-ulp differences of a stored stage state are
    not propagated into the next stage: the plain sensor of smooth p = 3 cells
    reacts to such differences through third derivatives of the rounding.
    Bar per stage: 8 ulp of |U| plus 1e-5 of the stage increment b0 dt L."""
    from oracle.method import wave_speed, time_derivative
    mesh = synth.quad_mesh(12, 12)
    sp = build_space(mesh, p, 1, 4)
    U = f32(euler_state(sp, k=6.0))
    prm = Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0), sc_on=0,
                 sensor=2 if sensor == "fixed" else 0, fixed_gamma=0.5)
    lam = wave_speed(prm, sp.to_cells(U), sp.node_coords()).max()
    dt = 0.1 * (1.0 / 12) / ((2 * p + 1) * lam)     # inside the SSP-RK3 / DG stability region
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 0)
    nk = (p + 1) * (p + 2) // 2 - 1
    cand = torch.zeros((mesh.n_vertices, nk), dtype=torch.float32, device="cuda")
    Un = _dev(U)
    cur = Un
    for (a0, b0) in ((0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0)):
        if sensor == "plain":
            cvw.vertex_candidates(gm, cp, cur, cand, ws)
        out = torch.empty_like(Un)
        cvw.rk_stage(gm, cp, cur, cand, Un if a0 else None, out, dt, a0, b0, ws)
        us = cur.cpu().numpy().astype(np.float64)
        inc = b0 * dt * time_derivative(sp, us, prm)
        ref = a0 * U + b0 * us + inc
        err = np.abs(out.cpu().numpy().astype(np.float64) - ref).max()
        assert err <= 8 * np.finfo(np.float32).eps * np.abs(U).max() + 1e-5 * np.abs(inc).max(), (a0, b0)
        cur = out
    assert cvw.poll_status(gm, ws) == 0


@pytest.mark.parametrize("sensor", ["fixed", "plain"])
def test_step_is_the_three_stages(sensor):
    """cvw_step equals, bit for bit, the stage-by-stage sequence through the
    public entry points (same kernels, same order)."""
    p = 3
    mesh = synth.quad_mesh(12, 12)
    sp = build_space(mesh, p, 1, 4)
    U = f32(euler_state(sp, k=6.0))
    prm = Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0),
                 sensor=2 if sensor == "fixed" else 0, fixed_gamma=0.5)
    dt = 2e-4
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 1)
    Ud = _dev(U)
    cvw.step(gm, cp, Ud, dt, 2, ws)
    cand = torch.zeros((mesh.n_vertices, 9), dtype=torch.float32, device="cuda")
    V = _dev(U)
    for _ in range(2):
        V1, V2 = torch.empty_like(V), torch.empty_like(V)
        for (us, un, uo, a0, b0) in ((V, None, V1, 0.0, 1.0), (V1, V, V2, 0.75, 0.25),
                                     (V2, V, V, 1.0 / 3.0, 2.0 / 3.0)):
            if sensor == "plain":
                cvw.vertex_candidates(gm, cp, us, cand, ws)
            cvw.rk_stage(gm, cp, us, cand, un, uo, dt, a0, b0, ws)
    assert torch.equal(Ud, V)
    assert cvw.poll_status(gm, ws) == 0


def test_totals_conserved_over_steps():
    from oracle.method import wave_speed
    mesh = synth.quad_mesh(32, 32)
    sp = build_space(mesh, 3, 1, 4)
    U = f32(euler_state(sp, k=6.0))
    lam = wave_speed(EULER, sp.to_cells(U), sp.node_coords()).max()
    dt = 0.2 * (1.0 / 32) / (3 * lam)
    gm = cvw.Mesh(mesh, 3, cvw.DG)
    cp = cvw.make_params(EULER)
    ws = cvw.alloc_workspace(gm, cp, 1)
    Ud = _dev(U)
    t0 = cvw.totals(gm, cp, Ud, ws, n_var=4)
    # oracle integral of the same state (diagonal collocated mass = Gauss weights;
    # the device uses the weights rounded to float32, hence rtol 1e-6)
    ref = (U.reshape(4, sp.E, -1) * sp.ref.vol_w[None, None, :]).sum((1, 2)) * (1.0 / 32) ** 2 / 4
    assert np.allclose(t0, ref, rtol=1e-6, atol=0)
    cvw.step(gm, cp, Ud, dt, 10, ws)
    t1 = cvw.totals(gm, cp, Ud, ws, n_var=4)
    assert np.all(np.abs(t1 - t0) <= 2e-6 * np.abs(t0).max())
    assert cvw.poll_status(gm, ws) == 0


def test_status_flags_negative_density():
    mesh = synth.quad_mesh(8, 8)
    sp = build_space(mesh, 2, 1, 4)
    U = f32(euler_state(sp, k=6.0)).reshape(4, -1)
    U[0, 5] = -0.5
    gm = cvw.Mesh(mesh, 2, cvw.DG)
    cp = cvw.make_params(EULER)
    ws = cvw.alloc_workspace(gm, cp, 0)
    Ud = _dev(U.ravel())
    R = torch.empty_like(Ud)
    cvw.residual(gm, cp, Ud, R, None, ws)
    flags = cvw.poll_status(gm, ws)
    assert flags & 2
    assert cvw.poll_status(gm, ws) == 0     # cleared


def test_error_paths():
    mesh = synth.quad_mesh(8, 8)
    gm = cvw.Mesh(mesh, 2, cvw.DG)
    cp = cvw.make_params(Params(flux=synth.ADVECT_ROT, flux_param=(0.5, 0.5, 1.0, 0)))
    ws = cvw.alloc_workspace(gm, cp, 0)
    u = torch.zeros(64 * 9, device="cuda")
    R = torch.empty_like(u)
    with pytest.raises(cvw.CvwError) as ei:
        cvw.residual(gm, cp, u, R, None, ws)
    assert ei.value.status == cvw.EUNSUPPORTED
    cp = cvw.make_params(Params())
    with pytest.raises(cvw.CvwError) as ei:
        cvw.residual(gm, cp, u, R, None, ws[:16])
    assert ei.value.status == cvw.EINVAL
    with pytest.raises(cvw.CvwError) as ei:
        cvw.residual(gm, cp, u, u, None, ws)
    assert ei.value.status == cvw.EINVAL
    # the binding checks element type and length before the call
    with pytest.raises(TypeError):
        cvw.residual(gm, cp, u.double(), R.double(), None, ws)
    with pytest.raises(ValueError):
        cvw.residual(gm, cp, u[:10], R, None, ws)


def test_full_size_config4_sampled_cells():
    """1024^2 DG Q3 Euler (the benchmark workload, same launch): sampled cells
    against the oracle evaluated on the sub-mesh of their vertex rings."""
    n = 1024
    mesh = synth.quad_mesh(n, n)
    gm = cvw.Mesh(mesh, 3, cvw.DG)
    # state on the device, built cell-row by cell-row from the oracle's node positions
    sp_small = build_space(synth.quad_mesh(1, 1, periodic=(False, False)), 3, 1)
    ref_nodes = sp_small.ref.nodes                                  # [16, 2] reference coords
    h = 1.0 / n
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    xc = (ii.ravel() + 0.5) * h
    yc = (jj.ravel() + 0.5) * h
    X = xc[:, None] + 0.5 * h * ref_nodes[None, :, 0]
    Y = yc[:, None] + 0.5 * h * ref_nodes[None, :, 1]
    U = np.asarray(synth.euler_state_config4(X, Y, smooth_k=400.0), np.float32)   # [4, E, 16]
    cp = cvw.make_params(EULER)
    ws = cvw.alloc_workspace(gm, cp, 0)
    Ud = torch.from_numpy(U.reshape(-1)).cuda()
    R = torch.empty_like(Ud)
    cvw.residual(gm, cp, Ud, R, None, ws)
    R = R.cpu().numpy().reshape(4, n * n, 16)
    rng = np.random.default_rng(0)
    edge = np.nonzero((np.abs(xc - 0.5) < 3 * h) | (np.abs(yc - 0.5) < 3 * h))[0]
    cells = np.unique(np.concatenate([rng.choice(n * n, 24, replace=False), rng.choice(edge, 40, replace=False),
                                      [0, n - 1, n * n - 1]]))
    sub, ids, pos = subset_ring(mesh, cells)
    sp = build_space(sub, 3, 1, 4)
    Us = U[:, ids, :].astype(np.float64)
    R_o, parts = o_residual(sp, Us.ravel(), EULER, return_parts=True, allow_boundary=True)
    R_o = R_o.reshape(4, len(ids), 16)[:, pos, :]
    keep = np.abs(parts["gamma"][pos] - 0.9) >= 1e-4
    assert (parts["gamma"][pos] < 0.9).sum() >= 5
    for v in range(4):
        assert rel_err(R[v, cells][keep], R_o[v][keep]) < 1e-5, v
