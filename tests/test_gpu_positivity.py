"""GPU parity: the Zhang-Shu positivity limiter (cvw_positivity, Euler on DG
quadrilaterals) against the oracle's positivity_limit on the same
float32-rounded inputs.

Tolerance 1e-5 of max |U| per variable: both sides scale in float64 (the
device takes its quadratic's root in closed form, the oracle bisects); the
device rounds the result to float32.  Admissible cells must be copied bit for
bit.  Positivity is checked on the stored float32 result up to its rounding.
"""
import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space, positivity_limit
from oracle.method import _face_trace_matrix, _pressure
from tests.parity_helpers import f32, euler_state
from tests.test_oracle_positivity import inadmissible_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import cvw  # noqa: E402

EULER = Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0))


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32).reshape(-1)).cuda()


def _points(sp, V):
    return np.concatenate([V, V @ _face_trace_matrix(sp).T], axis=-1)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_positivity_parity(p):
    sp, U, _ = inadmissible_state(p, seed=p)
    U = f32(U)
    gm = cvw.Mesh(sp.mesh, p, cvw.DG)
    cp = cvw.make_params(EULER)
    Ud = _dev(U)
    out = torch.empty_like(Ud)
    cvw.positivity(gm, cp, Ud, out, 1e-13, cvw.alloc_workspace(gm, cp, cvw.OP_POS))
    got = out.cpu().numpy().reshape(U.shape)
    ref = positivity_limit(sp, U, EULER)
    changed = np.any(ref != U, axis=(0, 2))
    assert changed.sum() >= 20
    for v in range(4):
        assert np.abs(got[v] - ref[v]).max() <= 1e-5 * np.abs(U[v]).max(), v
    assert np.array_equal(got[:, ~changed], U.astype(np.float32)[:, ~changed])
    # cell averages and positivity at the points of the stored result
    w1 = np.polynomial.legendre.leggauss(p + 1)[1]
    w = np.outer(w1, w1).ravel() / 4.0
    g64 = got.astype(np.float64)
    assert np.abs(g64 @ w - U @ w).max() <= 1e-6 * np.abs(U).max()
    Q = np.stack([_points(sp, g64[v]) for v in range(4)])
    scale = np.abs(U).max()
    assert Q[0].min() >= -1e-6 * scale and _pressure(Q, 1.4).min() >= -1e-6 * scale


def test_positivity_in_place_and_admissible_copy():
    sp, U, _ = inadmissible_state(3, seed=7)
    U = f32(U)
    gm = cvw.Mesh(sp.mesh, 3, cvw.DG)
    cp = cvw.make_params(EULER)
    ws = cvw.alloc_workspace(gm, cp, cvw.OP_POS)
    a = torch.empty(U.size, dtype=torch.float32, device="cuda")
    cvw.positivity(gm, cp, _dev(U), a, 1e-13, ws)
    b = _dev(U)
    cvw.positivity(gm, cp, b, b, 1e-13, ws)
    assert torch.equal(a, b)
    sp2 = build_space(synth.quad_mesh(10, 9), 3, 1, 4)
    V = f32(sp2.to_cells(euler_state(sp2, k=10.0)))
    c = _dev(V)
    d = torch.empty_like(c)
    cvw.positivity(gm, cp, c, d, 1e-13, ws)
    assert torch.equal(c, d)


def test_positivity_errors():
    mesh = synth.quad_mesh(8, 8)
    gm = cvw.Mesh(mesh, 2, cvw.DG)
    u = torch.ones(4 * 64 * 9, device="cuda")
    ws = cvw.alloc_workspace(gm, cvw.make_params(EULER), cvw.OP_POS)
    assert ws.numel() == 256 + 256      # count, then 64 cell indices rounded up to 256 bytes
    with pytest.raises(cvw.CvwError) as ei:
        cvw.positivity(gm, cvw.make_params(Params()), u[: 64 * 9], u[: 64 * 9], 1e-13, ws)
    assert ei.value.status == cvw.EUNSUPPORTED
    cp = cvw.make_params(EULER)
    for eps0 in (0.0, -1.0, float("nan")):
        with pytest.raises(cvw.CvwError) as ei:
            cvw.positivity(gm, cp, u, u, eps0, ws)
        assert ei.value.status == cvw.EINVAL
    with pytest.raises(cvw.CvwError) as ei:
        cvw.positivity(gm, cp, u, u, 1e-13, ws[:300])
    assert ei.value.status == cvw.EINVAL
    gc = cvw.Mesh(mesh, 2, cvw.CG)
    with pytest.raises(cvw.CvwError) as ei:
        cvw.positivity(gc, cp, torch.ones(4 * gc.info["n_dof"], device="cuda"),
                       torch.ones(4 * gc.info["n_dof"], device="cuda"), 1e-13, ws)
    assert ei.value.status == cvw.EUNSUPPORTED


def test_full_size_state_admissible_unchanged():
    """1024^2 benchmark state: admissible everywhere, so copied unchanged."""
    import bench
    n = 1024
    mesh = synth.quad_mesh(n, n)
    gm = cvw.Mesh(mesh, 3, cvw.DG)
    U = torch.from_numpy(bench.euler_config4_state(n, bench.gauss_nodes_2d(3), bench.SMOOTH_K).reshape(-1)).cuda()
    out = torch.empty_like(U)
    cp = cvw.make_params(EULER)
    cvw.positivity(gm, cp, U, out, 1e-13, cvw.alloc_workspace(gm, cp, cvw.OP_POS))
    assert torch.equal(U, out)


def test_full_size_one_percent_negative_sampled():
    """1024^2 benchmark state with negative density at one node of 1 % of the
    cells (the benchmark's planted cells): exactly those cells change; 64 of
    them, sampled, match the oracle (the limiter is cell-local, so the sampled
    cells are placed on an 8 x 8 mesh for it)."""
    import bench
    n, p = 1024, 3
    gm = cvw.Mesh(synth.quad_mesh(n, n), p, cvw.DG)
    cp = cvw.make_params(EULER)
    U = torch.from_numpy(bench.euler_config4_state(n, bench.gauss_nodes_2d(p), bench.SMOOTH_K).reshape(-1)).cuda()
    E, nloc = n * n, (p + 1) ** 2
    g = torch.Generator(device="cpu").manual_seed(2024)
    cells = torch.randperm(E, generator=g)[: E // 100]
    V = U.clone()
    V[cells.cuda() * nloc] = -0.1
    out = torch.empty_like(V)
    cvw.positivity(gm, cp, V, out, 1e-13, cvw.alloc_workspace(gm, cp, cvw.OP_POS))
    Vh = V.cpu().numpy().reshape(4, E, nloc)
    Oh = out.cpu().numpy().reshape(4, E, nloc)
    diff = np.any(Oh != Vh, axis=(0, 2))
    assert np.array_equal(np.flatnonzero(diff), np.sort(cells.numpy()))
    pick = np.sort(cells.numpy()[:: len(cells) // 64][:64])
    sp = build_space(synth.quad_mesh(8, 8), p, 1, 4)
    ref = positivity_limit(sp, Vh[:, pick].astype(np.float64), EULER)
    for v in range(4):
        assert np.abs(Oh[v, pick] - ref[v]).max() <= 1e-5 * np.abs(Vh[v, pick]).max(), v


@pytest.mark.parametrize("p", [1, 2, 3])
def test_positivity_parity_triangles(p):
    """DG triangles (jittered, Euler): the points are the volume rule's and the
    edge Gauss points; limited cells match the oracle, admissible ones are
    copied bit for bit, in place equals out of place, cell averages and
    positivity hold on the stored result."""
    from tests.test_oracle_positivity import _points as o_points, _means as o_means
    sp, U, _ = inadmissible_state(p, seed=p, cell=synth.TRI)
    U = f32(U)
    gm = cvw.Mesh(sp.mesh, p, cvw.DG)
    cp = cvw.make_params(EULER)
    ws = cvw.alloc_workspace(gm, cp, cvw.OP_POS)
    Ud = _dev(U)
    out = torch.empty_like(Ud)
    cvw.positivity(gm, cp, Ud, out, 1e-13, ws)
    inplace = Ud.clone()
    cvw.positivity(gm, cp, inplace, inplace, 1e-13, ws)
    assert torch.equal(out, inplace)
    got = out.cpu().numpy().reshape(U.shape)
    ref = positivity_limit(sp, U, EULER)
    changed = np.any(ref != U, axis=(0, 2))
    assert changed.sum() >= 15
    for v in range(4):
        assert np.abs(got[v] - ref[v]).max() <= 1e-5 * np.abs(U[v]).max(), v
    assert np.array_equal(got[:, ~changed], U.astype(np.float32)[:, ~changed])
    g64 = got.astype(np.float64)
    assert np.abs(o_means(sp, g64) - o_means(sp, U)).max() <= 1e-6 * np.abs(U).max()
    Q = np.stack([o_points(sp, g64[v]) for v in range(4)])
    scale = np.abs(U).max()
    assert Q[0].min() >= -1e-6 * scale and _pressure(Q, 1.4).min() >= -1e-6 * scale
