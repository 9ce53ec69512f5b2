"""GPU: the plain sensor as fallback and judge of the learned sensor.

* a cell whose features leave the network's validity box, or whose network
  output is not finite, takes the plain sensor's gamma_e (eq. gamma) instead:
  with every cell handed over, the learned sensor equals the plain one bit for
  bit (the same fused pass computes both), and the hand-over is counted;
* the audit compares the learned gamma with the plain one on every cell; its
  mean deviation is checked against the two sensors' outputs taken separately;
  a mean above the tolerance switches the run to the plain sensor (the latch
  stays in the workspace), also inside cvw_step with audit_every.
"""
import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space
from tests.parity_helpers import f32, euler_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import cvw, learned  # noqa: E402

EULER = Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0))
LEARNED = Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0), sensor=cvw.LEARNED)


def _case(n=32, p=3):
    mesh = synth.quad_mesh(n, n)
    sp = build_space(mesh, p, 1, 4)
    U = torch.from_numpy(np.ascontiguousarray(f32(euler_state(sp, k=6.0)), np.float32)).cuda()
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(EULER)
    return gm, U, cp, learned.sigma_reference(gm, cp, U)


def _sensor(gm, cp, U, ws=None):
    ws = cvw.alloc_workspace(gm, cp, 0) if ws is None else ws
    g = torch.empty(gm.info["n_cells"], dtype=torch.float32, device="cuda")
    cvw.sensor(gm, cp, U, g, None, ws)
    return g


def test_cells_outside_the_box_take_the_plain_sensor():
    gm, U, cp, sref = _case()
    net = cvw.Mlp(learned.init_params(4))
    cl = cvw.make_params(LEARNED, mlp=net, sigma_ref=sref)
    ws = cvw.alloc_workspace(gm, cl, 0)
    g_free = _sensor(gm, cl, U, ws)                       # unbounded box: the network decides everywhere
    assert cvw.poll_status(gm, ws) == 0
    g_plain = _sensor(gm, cp, U)
    assert not torch.equal(g_free, g_plain)
    # a box that no cell fits: every cell is handed over
    net.set_range(np.full(48, 5.0), np.full(48, 6.0))
    g = _sensor(gm, cl, U, ws)
    assert torch.equal(g, g_plain)
    assert cvw.poll_status(gm, ws) & 8
    # a box around one feature's observed range minus its top: some cells only
    f = learned.features_of(gm, cp, U)
    v = ((f.to(torch.int32) & 0xFFFF) << 16).view(torch.float32)[:, 0]
    lo = np.full(48, -np.inf, np.float32)
    hi = np.full(48, np.inf, np.float32)
    hi[0] = float(torch.quantile(v, 0.9).item())
    net.set_range(lo, hi)
    g = _sensor(gm, cl, U, ws)
    out = (v > hi[0])
    assert 0 < int(out.sum().item()) < gm.info["n_cells"]
    assert torch.equal(g[out], g_plain[out])
    assert torch.equal(g[~out], g_free[~out])
    aud = cvw.learned_audit(gm, cl, U, ws)
    assert aud["handed_over"] >= 2 * int(out.sum().item())   # this call and the audit's own evaluation
    with pytest.raises(cvw.CvwError):
        net.set_range(np.full(48, 1.0), np.full(48, 0.0))


def test_non_finite_output_takes_the_plain_sensor():
    """Huge (finite) weights overflow the hidden activations: where the raw
    network output is not finite the plain sensor decides, elsewhere the
    network's value is kept."""
    gm, U, cp, sref = _case()
    P = cvw.unpack_params(learned.init_params(5))
    P["W1"] = P["W1"] * 1e36
    P["W2"] = P["W2"] * 1e36
    net = cvw.Mlp(cvw.pack_params(P))
    cl = cvw.make_params(LEARNED, mlp=net, sigma_ref=sref)
    ws = cvw.alloc_workspace(gm, cl, 0)
    g = _sensor(gm, cl, U, ws)
    g_plain = _sensor(gm, cp, U)
    raw = learned.predict(net, learned.features_of(gm, cl, U))      # unguarded inference
    bad = ~torch.isfinite(raw)
    assert int(bad.sum().item()) > 0
    assert torch.isfinite(g).all()
    assert torch.equal(g[bad], g_plain[bad])
    assert torch.equal(g[~bad], raw[~bad])
    assert cvw.poll_status(gm, ws) & 8


def test_audit_measures_and_switches():
    gm, U, cp, sref = _case()
    net = cvw.Mlp(learned.init_params(4))                 # untrained: far from the plain sensor
    cl = cvw.make_params(LEARNED, mlp=net, sigma_ref=sref, audit_tol=1.0)
    ws = cvw.alloc_workspace(gm, cl, 0)
    g_l = _sensor(gm, cl, U, ws).double()
    g_p = _sensor(gm, cp, U).double()
    aud = cvw.learned_audit(gm, cl, U, ws)
    d = (g_l - g_p).abs()
    assert abs(aud["mean_abs_dev"] - d.mean().item()) <= 1e-9 + 1e-6 * d.mean().item()
    assert aud["max_abs_dev"] == pytest.approx(d.max().item(), rel=1e-6, abs=1e-9)
    assert not aud["switched_off"]
    assert cvw.poll_status(gm, ws) & 16 == 0
    # a tolerance below the measured mean switches the run to the plain sensor
    cs = cvw.make_params(LEARNED, mlp=net, sigma_ref=sref, audit_tol=0.5 * aud["mean_abs_dev"])
    assert cvw.learned_audit(gm, cs, U, ws)["switched_off"]
    assert cvw.poll_status(gm, ws) & 16
    assert torch.equal(_sensor(gm, cl, U, ws), g_p.float())
    assert cvw.poll_status(gm, ws) & 16 == 0               # reported once; the latch stays
    assert torch.equal(_sensor(gm, cl, U, ws), g_p.float())


def test_step_audit_switches_to_plain():
    """cvw_step with audit_every = 1 and a zero tolerance: the audit at the
    start of the step switches an untrained network off, so the step equals
    the plain step bit for bit."""
    gm, U, cp, sref = _case(24, 3)
    net = cvw.Mlp(learned.init_params(6))
    cl = cvw.make_params(LEARNED, mlp=net, sigma_ref=sref, audit_every=1, audit_tol=0.0)
    wl = cvw.alloc_workspace(gm, cl, 1)
    wp = cvw.alloc_workspace(gm, cp, 1)
    a, b = U.clone(), U.clone()
    cvw.step(gm, cl, a, 2e-4, 2, wl)
    cvw.step(gm, cp, b, 2e-4, 2, wp)
    assert torch.equal(a, b)
    assert cvw.poll_status(gm, wl) & 16
