"""GPU parity of the fused sensor pass (structured periodic DG quadrilateral
grids): gamma_e of eq. gamma against the float64 oracle, against the two-pass
path (vertex candidates through the workspace), on ragged tiles and the
smallest periodic grid, and the stage with a supplied gamma.

Bars as in the other DG quadrilateral tests: gamma to 2e-5 in absolute value on
cells whose element semi-norm is not at round-off level; residuals to 1e-5 of
max |R| per variable, cells within 1e-4 of the shock-capturing switch left out.
"""
import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space, residual as o_residual
from oracle.method import vertex_candidates as o_cand, cell_sensor as o_sensor
from tests.parity_helpers import rel_err, f32, rough_scalar, euler_state, subset_ring

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import cvw  # noqa: E402

EULER = Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0))


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _gamma(gm, prm, U, E):
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 0)
    g = torch.empty(E, dtype=torch.float32, device="cuda")
    cvw.sensor(gm, cp, _dev(U), g, None, ws)
    return g.cpu().numpy()


def _oracle_gamma(sp, s, prm):
    g, parts = o_sensor(sp, s, o_cand(sp, s, prm), prm, return_parts=True)
    return g, parts["n"] > 1e-6 * parts["n"].max()


def test_grid_detection():
    gm = cvw.Mesh(synth.quad_mesh(13, 11), 2, cvw.DG)
    assert (gm.info["grid_nx"], gm.info["grid_ny"]) == (13, 11)
    gm = cvw.Mesh(synth.quad_mesh(13, 11), 2, cvw.CG)
    assert gm.info["grid_nx"] == 0


@pytest.mark.parametrize("p", [1, 2, 3])
@pytest.mark.parametrize("nx,ny", [(3, 3), (13, 11), (17, 35), (40, 33)])
def test_gamma_matches_oracle(p, nx, ny):
    mesh = synth.quad_mesh(nx, ny)
    sp = build_space(mesh, p, 1)
    u = f32(rough_scalar(sp, 2))
    gm = cvw.Mesh(mesh, p, cvw.DG)
    assert gm.info["grid_nx"] == nx
    g = _gamma(gm, Params(), u, sp.E)
    g_o, live = _oracle_gamma(sp, u, Params())
    assert np.abs(g - g_o)[live].max() < 2e-5
    if nx * ny > 100:
        assert (g_o < 0.9).sum() >= 3


@pytest.mark.parametrize("p", [1, 2, 3])
def test_gamma_euler_density(p):
    mesh = synth.quad_mesh(24, 20)
    sp = build_space(mesh, p, 1, 4)
    U = f32(euler_state(sp, k=6.0))
    gm = cvw.Mesh(mesh, p, cvw.DG)
    g = _gamma(gm, EULER, U, sp.E)
    g_o, live = _oracle_gamma(sp, U.reshape(4, sp.E, -1)[0], EULER)
    assert np.abs(g - g_o)[live].max() < 2e-5
    assert (g_o < 0.9).sum() >= 3


@pytest.mark.parametrize("p", [1, 3])
def test_fused_and_twopass_agree(p, monkeypatch):
    """Both paths of eq. gamma (fused; vertex candidates through the workspace)
    against the oracle and each other; residual of the Euler state too."""
    mesh = synth.quad_mesh(21, 18)
    sp = build_space(mesh, p, 1, 4)
    U = f32(euler_state(sp, k=6.0))
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(EULER)
    Ud = _dev(U)

    def run():
        ws = cvw.alloc_workspace(gm, cp, 0)        # the two-pass path needs room for the candidates
        g = torch.empty(sp.E, dtype=torch.float32, device="cuda")
        R = torch.empty_like(Ud)
        cvw.sensor(gm, cp, Ud, g, None, ws)
        cvw.residual(gm, cp, Ud, R, None, ws)
        return g.cpu().numpy(), R.cpu().numpy().reshape(4, -1)

    g1, R1 = run()
    monkeypatch.setenv("CVW_SENSOR_PATH", "twopass")
    g2, R2 = run()
    monkeypatch.delenv("CVW_SENSOR_PATH")
    g_o, live = _oracle_gamma(sp, U.reshape(4, sp.E, -1)[0], EULER)
    R_o, parts = o_residual(sp, U, EULER, return_parts=True)
    R_o = R_o.reshape(4, -1)
    keep = np.repeat(np.abs(parts["gamma"] - 0.9) >= 1e-4, sp.ref.n_loc)
    for g in (g1, g2):
        assert np.abs(g - g_o)[live].max() < 2e-5
    assert np.abs(g1 - g2)[live].max() < 4e-5
    for R in (R1, R2):
        for v in range(4):
            assert rel_err(R[v][keep], R_o[v][keep]) < 1e-5, v


def test_renumbered_cells_take_the_twopass_path():
    """A periodic grid whose cells are not numbered row by row has no grid
    size; the sensor then runs the two-pass path and still matches the oracle."""
    base = synth.quad_mesh(11, 9)
    perm = np.random.default_rng(3).permutation(base.n_cells)
    mesh = synth.MeshDesc(2, synth.QUAD, base.n_vertices, base.cell_vertices[perm].copy(),
                          base.cell_coords[perm].copy(), base.periodic, base.shape)
    p = 2
    sp = build_space(mesh, p, 1)
    u = f32(rough_scalar(sp, 5))
    gm = cvw.Mesh(mesh, p, cvw.DG)
    assert gm.info["grid_nx"] == 0
    g = _gamma(gm, Params(), u, sp.E)
    g_o, live = _oracle_gamma(sp, u, Params())
    assert np.abs(g - g_o)[live].max() < 2e-5


def test_constant_state_gives_one():
    mesh = synth.quad_mesh(19, 17)
    for p in (1, 2, 3):
        gm = cvw.Mesh(mesh, p, cvw.DG)
        g = _gamma(gm, Params(), np.full(mesh.n_cells * (p + 1) ** 2, 0.37), mesh.n_cells)
        assert (g == 1.0).all()


@pytest.mark.parametrize("p", [2, 3])
def test_stage_with_supplied_gamma_is_the_stage(p):
    """cvw_sensor followed by cvw_rk_stage_gamma equals cvw_rk_stage bit for
    bit (the same two kernels)."""
    mesh = synth.quad_mesh(16, 13)
    sp = build_space(mesh, p, 1, 4)
    U = _dev(f32(euler_state(sp, k=6.0)))
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(EULER)
    ws = cvw.alloc_workspace(gm, cp, 0)
    g = torch.empty(sp.E, dtype=torch.float32, device="cuda")
    a, b = torch.empty_like(U), torch.empty_like(U)
    cvw.sensor(gm, cp, U, g, None, ws)
    cvw.rk_stage_gamma(gm, cp, U, g, U, a, 1e-4, 0.75, 0.25, ws)
    cvw.rk_stage(gm, cp, U, None, U, b, 1e-4, 0.75, 0.25, ws)
    assert torch.equal(a, b)
    with pytest.raises(cvw.CvwError) as ei:
        cvw.rk_stage_gamma(gm, cp, U, g, U, U, 1e-4, 0.75, 0.25, ws)
    assert ei.value.status == cvw.EINVAL


def test_full_size_gamma_sampled_cells():
    """1024^2 DG Q3 Euler state: gamma of sampled cells (many along the
    quadrant interfaces) against the oracle on the sub-mesh of their vertex rings."""
    n = 1024
    mesh = synth.quad_mesh(n, n)
    gm = cvw.Mesh(mesh, 3, cvw.DG)
    ref_nodes = build_space(synth.quad_mesh(1, 1, periodic=(False, False)), 3, 1).ref.nodes
    h = 1.0 / n
    ii, jj = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")
    xc, yc = (ii.ravel() + 0.5) * h, (jj.ravel() + 0.5) * h
    U = np.asarray(synth.euler_state_config4(xc[:, None] + 0.5 * h * ref_nodes[None, :, 0],
                                             yc[:, None] + 0.5 * h * ref_nodes[None, :, 1], smooth_k=400.0),
                   np.float32)
    g = _gamma(gm, EULER, U.reshape(-1), n * n)
    rng = np.random.default_rng(1)
    edge = np.nonzero((np.abs(xc - 0.5) < 3 * h) | (np.abs(yc - 0.5) < 3 * h))[0]
    cells = np.unique(np.concatenate([rng.choice(n * n, 24, replace=False), rng.choice(edge, 40, replace=False),
                                      [0, 15, 16, n - 1, n * n - 1, 17 * n + 16]]))
    # gamma of a cell needs the full patches of its vertices: its vertex ring
    sub, ids, pos = subset_ring(mesh, cells)
    sp = build_space(sub, 3, 1)
    g_o, live = _oracle_gamma(sp, U[0, ids, :].astype(np.float64), EULER)
    assert (g_o[pos] < 0.9).sum() >= 5
    assert np.abs(g[cells] - g_o[pos])[live[pos]].max() < 2e-5
