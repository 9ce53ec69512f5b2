"""GPU: batched, graph-captured SSP-RK3 steps over an ensemble of DG
quadrilateral problems (mixed degree 1..3, advection / Burgers), through the
C ABI.

Every work item runs the block body of the single-mesh kernels (the fused
sensor pass over 16 x 16 tiles and the cell pass with that gamma; or, with
CVW_SENSOR_PATH=twopass when the batch is built, the vertex pass and the
cell pass with its candidates), so a batch step must equal cvw_step of each
instance alone on the same path bit for bit, with or without the graph, for
any grid size.  Graph replays are checked one by one against eager
launches, with eager work and synchronisations between them.  One instance is
also checked stage by stage against the float64 oracle.
"""
import numpy as np
import pytest

import synth
from oracle import build_space
from oracle.method import time_derivative
from tests.parity_helpers import f32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import cvw  # noqa: E402

SIZES = (12, 17, 9, 20, 14, 11, 16, 13)


def _ensemble(count=8):
    insts = synth.config5_instances(count=count)
    cases = []
    for k, inst in enumerate(insts):
        mesh, p, prm, U, dt = synth.instance_case(inst, n=SIZES[k % len(SIZES)])
        cases.append((mesh, p, prm, np.asarray(U, np.float32), dt))
    return cases


def _single_steps(cases, n_steps):
    outs = []
    for mesh, p, prm, U, dt in cases:
        gm = cvw.Mesh(mesh, p, cvw.DG)
        cp = cvw.make_params(prm)
        ws = cvw.alloc_workspace(gm, cp, 1)
        u = torch.from_numpy(U.copy()).cuda()
        cvw.step(gm, cp, u, dt, n_steps, ws)
        outs.append(u)
    return outs


def _batch(cases):
    states, items = [], []
    for mesh, p, prm, U, dt in cases:
        gm = cvw.Mesh(mesh, p, cvw.DG)
        u = torch.from_numpy(U.copy()).cuda()
        states.append(u)
        items.append((gm, cvw.make_params(prm), u, dt))
    return cvw.Batch(items), states


def test_ensemble_mix():
    cases = _ensemble()
    assert {c[1] for c in cases} == {1, 2, 3}
    assert {c[2].flux for c in cases} == {synth.ADVECT_CONST, synth.BURGERS}


@pytest.mark.parametrize("path", ["fused", "twopass"])
@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_step_equals_single_instances(use_graph, path, monkeypatch):
    cases = _ensemble()
    if path == "twopass":
        monkeypatch.setenv("CVW_SENSOR_PATH", "twopass")
    ref = _single_steps(cases, 2)
    b, states = _batch(cases)
    monkeypatch.delenv("CVW_SENSOR_PATH", raising=False)
    ws = b.alloc_workspace()
    b.step(2, ws, use_graph=use_graph)
    for k, (u, r) in enumerate(zip(states, ref)):
        assert torch.equal(u, r), k
    assert b.poll_status(ws) == 0


def test_grid_size_does_not_change_results():
    cases = _ensemble()
    b1, s1 = _batch(cases)
    b2, s2 = _batch(cases)
    w1, w2 = b1.alloc_workspace(), b2.alloc_workspace()
    b2.set_grid(7)
    b1.step(1, w1)
    b2.step(1, w2)
    for x, y in zip(s1, s2):
        assert torch.equal(x, y)


def test_graph_replays_match_eager():
    """Replay the captured step several times, with eager work and host
    synchronisation between the replays; each replay equals the eager step
    from the same state."""
    cases = _ensemble()
    bg, sg = _batch(cases)
    be, se = _batch(cases)
    wg, we = bg.alloc_workspace(), be.alloc_workspace()
    for rep in range(4):
        bg.step(1, wg, use_graph=True)
        be.step(1, we, use_graph=False)
        junk = torch.randn(1 << 16, device="cuda").sum()     # unrelated eager work
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        for k, (x, y) in enumerate(zip(sg, se)):
            assert torch.isfinite(x).all(), (rep, k)
            assert torch.equal(x, y), (rep, k)
    assert bg.poll_status(wg) == 0
    assert be.poll_status(we) == 0


def test_one_instance_stage_against_oracle():
    """The first stage u_1 = u + dt L(u) of an ensemble instance, through the
    single-mesh path that the batch equals bitwise, against the oracle on the
    same float32 input."""
    inst = synth.config5_instances(count=3)[2]
    mesh, p, prm, U, dt = synth.instance_case(inst, n=10)
    U = f32(U)
    sp = build_space(mesh, p, 1)
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(prm)
    ws = cvw.alloc_workspace(gm, cp, 0)
    u = torch.from_numpy(U.astype(np.float32)).cuda()
    cand = torch.empty((mesh.n_vertices, len(sp.ks)), dtype=torch.float32, device="cuda")
    cvw.vertex_candidates(gm, cp, u, cand, ws)
    out = torch.empty_like(u)
    cvw.rk_stage(gm, cp, u, cand, None, out, dt, 0.0, 1.0, ws)
    inc = dt * time_derivative(sp, U, prm)
    from oracle.method import cell_sensor, vertex_candidates
    uc = U.reshape(sp.E, -1)
    g = cell_sensor(sp, uc, vertex_candidates(sp, uc, prm), prm)
    near = np.repeat(np.abs(g - 0.9) < 1e-4, sp.ref.n_loc)
    err = np.abs(out.cpu().numpy().astype(np.float64) - (U + inc))[~near].max()
    assert err <= 8 * np.finfo(np.float32).eps * np.abs(U).max() + 1e-5 * np.abs(inc).max()


def test_batch_error_paths():
    mesh = synth.tri_mesh(4, 4)
    gm = cvw.Mesh(mesh, 2, cvw.DG)
    prm = synth.Params()
    u = torch.zeros(mesh.n_cells * 6, device="cuda")
    with pytest.raises(cvw.CvwError) as ei:
        cvw.Batch([(gm, cvw.make_params(prm), u, 1e-3)])
    assert ei.value.status == cvw.EUNSUPPORTED
    qm = synth.quad_mesh(4, 4)
    gq = cvw.Mesh(qm, 1, cvw.DG)
    uq = torch.zeros(16 * 4 * 4, device="cuda")
    with pytest.raises(cvw.CvwError) as ei:
        cvw.Batch([(gq, cvw.make_params(synth.Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0))), uq, 1e-3)])
    assert ei.value.status == cvw.EUNSUPPORTED
    b = cvw.Batch([(gq, cvw.make_params(prm), uq[:64], 1e-3)])
    with pytest.raises(cvw.CvwError) as ei:
        b.step(1, torch.zeros(256, dtype=torch.uint8, device="cuda"))
    assert ei.value.status == cvw.EINVAL


def test_batch_in_caller_buffer():
    """cvw_batch_build_in: the batch's device arrays in a buffer the caller
    owns (sized by cvw_batch_plan) step bitwise like the allocating build; a
    buffer one byte short is refused."""
    cases = _ensemble()
    b1, s1 = _batch(cases)
    states, items = [], []
    for mesh, p, prm, U, dt in cases:
        gm = cvw.Mesh(mesh, p, cvw.DG)
        u = torch.from_numpy(U.copy()).cuda()
        states.append(u)
        items.append((gm, cvw.make_params(prm), u, dt))
    need = cvw.batch_plan(items)
    assert need > 0 and need % 256 == 0
    with pytest.raises(cvw.CvwError):
        cvw.Batch(items, device_buffer=torch.zeros(need - 1, dtype=torch.uint8, device="cuda"))
    buf = torch.zeros(need, dtype=torch.uint8, device="cuda")
    b2 = cvw.Batch(items, device_buffer=buf)
    w1, w2 = b1.alloc_workspace(), b2.alloc_workspace()
    b1.step(2, w1)
    b2.step(2, w2)
    for x, y in zip(s1, states):
        assert torch.equal(x, y)
    assert b2.poll_status(w2) == 0
