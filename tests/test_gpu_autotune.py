"""GPU: the autotuner times candidate launch shapes through the C ABI, keeps
results bitwise equal across them, applies and caches the fastest."""
import numpy as np
import pytest

import synth
from oracle import build_space
from tests.parity_helpers import f32, euler_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import autotune, cvw  # noqa: E402


def test_tune_mesh(tmp_path):
    path = str(tmp_path / "tune.json")
    mesh = synth.quad_mesh(40, 36)
    sp = build_space(mesh, 3, 1, 4)
    U = torch.from_numpy(np.ascontiguousarray(f32(euler_state(sp, k=6.0)), np.float32)).cuda().reshape(-1)
    gm = cvw.Mesh(mesh, 3, cvw.DG)
    cp = cvw.make_params(synth.Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0)))
    ws = cvw.alloc_workspace(gm, cp, 0)
    cand = torch.empty((mesh.n_vertices, 9), dtype=torch.float32, device="cuda")
    cvw.vertex_candidates(gm, cp, U, cand, ws)
    best = autotune.tune_mesh(gm, cp, U, cand, ws, candidates=(8, 24, 0), reps=3, path=path)
    assert best in (8, 24, 0)
    gm.set_grid(0)
    assert autotune.apply_cached(gm, cp, path=path) == best
    entry = autotune.load_cache(path)[autotune.mesh_key(gm, cp)]
    assert set(entry["timings_ms"]) == {"8", "24", "0"}
    # another flux on the same mesh has its own entry
    cp_adv = cvw.make_params(synth.Params(flux=synth.ADVECT_CONST, flux_param=(1.0, 0.5, 0, 0)))
    assert autotune.mesh_key(gm, cp_adv) != autotune.mesh_key(gm, cp)
    assert autotune.apply_cached(gm, cp_adv, path=path) is None


def test_tune_batch_restores_states(tmp_path):
    path = str(tmp_path / "tune.json")
    items = []
    for inst in synth.config5_instances(seed=77, count=6):
        mesh, p, prm, U, dt = synth.instance_case(inst, n=32)
        gm = cvw.Mesh(mesh, p, cvw.DG)
        items.append((gm, cvw.make_params(prm), torch.from_numpy(np.asarray(U, np.float32)).cuda(), dt))
    b = cvw.Batch(items)
    ws = b.alloc_workspace()
    before = [u.clone() for u in b.states]
    best = autotune.tune_batch(b, ws, candidates=(1, 7, 0), reps=2, path=path)
    assert best in (1, 7, 0)
    assert all(torch.equal(u, v) for u, v in zip(b.states, before))
    assert autotune.batch_key(b) in autotune.load_cache(path)
