"""GPU: the allocation-free residual (cvw_residual_noalloc, the library's
per-device scratch array as workspace) against cvw_residual with a caller
workspace, through the C ABI: two calls in a row, the second on a smaller
problem, bit for bit (the same kernels); sizes beyond the array refused."""
import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space
from tests.parity_helpers import f32, euler_state, rough_scalar

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import cvw  # noqa: E402


def _both(mesh, p, prm, U):
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(prm)
    u = torch.from_numpy(np.ascontiguousarray(U, np.float32)).cuda()
    ws = cvw.alloc_workspace(gm, cp, 0)
    R1, R2 = torch.empty_like(u), torch.full_like(u, np.nan)
    g1 = torch.empty(mesh.n_cells, dtype=torch.float32, device="cuda")
    g2 = torch.full_like(g1, np.nan)
    cvw.residual(gm, cp, u, R1, g1, ws)
    cvw.residual_noalloc(gm, cp, u, R2, g2)
    torch.cuda.synchronize()
    return R1, R2, g1, g2


def test_noalloc_residual_matches_twice():
    # first call: DG Q3 Euler on 40 x 36 cells
    mesh = synth.quad_mesh(40, 36)
    sp = build_space(mesh, 3, 1, 4)
    R1, R2, g1, g2 = _both(mesh, 3, Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0)),
                           f32(euler_state(sp, k=60.0)))
    assert torch.equal(R1, R2) and torch.equal(g1, g2)
    assert (g1 < 0.9).sum().item() >= 3           # the shock-capturing weights are active
    # second call, smaller: DG Q2 Burgers on 13 x 11 cells
    mesh = synth.quad_mesh(13, 11)
    sp = build_space(mesh, 2, 1)
    R1, R2, g1, g2 = _both(mesh, 2, Params(flux=synth.BURGERS, flux_param=(1.0, 1.0, 0, 0)),
                           f32(rough_scalar(sp, 3)))
    assert torch.equal(R1, R2) and torch.equal(g1, g2)


def test_noalloc_residual_refuses_large_meshes():
    n = 2048                                   # 4 * n^2 bytes of gamma alone fill the 16 MiB array
    gm = cvw.Mesh(synth.quad_mesh(n, n), 1, cvw.DG)
    cp = cvw.make_params(Params())
    assert cvw.workspace_bytes(gm, cp, 0) > 16 << 20
    u = torch.zeros(n * n * 4, dtype=torch.float32, device="cuda")
    R = torch.empty_like(u)
    with pytest.raises(cvw.CvwError) as ei:
        cvw.residual_noalloc(gm, cp, u, R)
    assert ei.value.status == cvw.EINVAL
    assert "16 MiB" in str(ei.value)
