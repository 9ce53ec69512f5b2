"""GPU parity of the learned sensor against the float64 reference
(oracle/learned.py), through the C ABI.

* features: the device computes them in float64 and stores bfloat16; the
  reference gets the device's (float32) vertex candidates, so both evaluate
  the same function of the same inputs: every feature within half a bfloat16
  spacing (2^-8 relative) plus 1e-6 of the largest feature;
* inference: bfloat16 inputs, weights and hidden activations, float32
  accumulation; the reference rounds at the same points in float64, so a
  hidden unit whose value sits at a bfloat16 rounding boundary may round the
  other way: |gamma - gamma_ref| <= 2e-3 everywhere and <= 1e-4 for 99 % of
  the cells;
* gradient: float32 activations and errors (as two bfloat16 terms on the
  matrix cores) through bfloat16 weights and inputs vs the float64 gradient of
  the same network: 2e-4 of the largest entry per parameter tensor;
* Adam: one step moves every parameter by lr g / (|g| + eps);
* the residual with the learned gamma equals the residual of the reference
  with the same gamma (1e-5 of max |R|).
"""
import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space, residual as o_residual
from oracle.learned import (features as o_features, mlp_init, mlp_forward, mlp_loss_grad, bf16_weights,
                            bf16_round, N_FEAT)
from tests.parity_helpers import rel_err, f32, rough_scalar, euler_state

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import cvw  # noqa: E402


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


def _bits_to_float(t):
    b = t.cpu().numpy().view(np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def _float_to_bits(x):
    x = bf16_round(x).astype(np.float32)
    return torch.from_numpy((x.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)).cuda()


def _random_net(seed):
    P = mlp_init(seed)
    rng = np.random.default_rng(seed + 100)
    P["b1"] = rng.normal(size=64) * 0.2
    P["b2"] = rng.normal(size=64) * 0.2
    P["b3"] = np.array([0.3])
    return cvw.unpack_params(cvw.pack_params(P))      # float32 master values


@pytest.mark.parametrize("p", [1, 2, 3])
def test_features(p):
    mesh = synth.quad_mesh(13, 11)
    sp = build_space(mesh, p, 1)
    u = f32(rough_scalar(sp, 1))
    prm = Params()
    gm = cvw.Mesh(mesh, p, cvw.DG)
    sigma_ref = 0.37
    cp = cvw.make_params(prm, sigma_ref=sigma_ref)
    ws = cvw.alloc_workspace(gm, cp, 0)
    ud = _dev(u)
    cand = torch.empty((mesh.n_vertices, len(sp.ks)), dtype=torch.float32, device="cuda")
    cvw.vertex_candidates(gm, cp, ud, cand, ws)
    feat = torch.empty((sp.E, 48), dtype=torch.int16, device="cuda")
    cvw.mlp_features(gm, cp, ud, cand, feat)
    got = _bits_to_float(feat)
    want = o_features(sp, u, cand.cpu().numpy().astype(np.float64), sigma_ref)
    tol = 2.0 ** -8 * np.abs(want) + 1e-6 * np.abs(want).max()
    assert np.all(np.abs(got - want) <= tol), np.abs(got - want).max()
    if p < 3:
        pad = [t for t, k in enumerate([(1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3)])
               if sum(k) > p]
        cols = [9 * l + t for l in range(4) for t in pad] + [36 + t for t in pad]
        assert np.all(got[:, cols] == 0.0)


@pytest.mark.parametrize("n", [0, 5, 32, 1000, 4133])
def test_inference(n):
    P = _random_net(3)
    net = cvw.Mlp(cvw.pack_params(P))
    X = bf16_round(np.random.default_rng(n).normal(size=(max(n, 1), N_FEAT)) * 1.5)[:n]
    g = torch.full((max(n, 1),), -1.0, device="cuda")
    feat = _float_to_bits(X.reshape(-1)).reshape(-1) if n else torch.zeros(48, dtype=torch.int16, device="cuda")
    net.infer(feat[:n * 48] if n else feat[:0], g)
    if n == 0:
        assert g.item() == -1.0
        return
    got = g.cpu().numpy().astype(np.float64)
    want = mlp_forward(P, X, bf16=True)
    d = np.abs(got - want)
    assert d.max() <= 2e-3, d.max()
    assert np.quantile(d, 0.99) <= 1e-4


def test_network_in_caller_buffer():
    """cvw_mlp_create_in: the network's device memory in a buffer the caller
    owns gives bitwise the inference of the allocating handle; a misaligned
    or short buffer is refused."""
    packed = cvw.pack_params(_random_net(7))
    need = cvw.mlp_device_bytes()
    assert need > 0 and need % 256 == 0
    buf = torch.zeros(need + 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(cvw.CvwError):
        cvw.Mlp(packed, device_buffer=buf[:need - 1])
    with pytest.raises(cvw.CvwError):
        cvw.Mlp(packed, device_buffer=buf[8:])
    a, b = cvw.Mlp(packed), cvw.Mlp(packed, device_buffer=buf)
    X = bf16_round(np.random.default_rng(2).normal(size=(777, N_FEAT)))
    feat = _float_to_bits(X.reshape(-1)).reshape(-1)
    ga = torch.empty(777, device="cuda")
    gb = torch.empty(777, device="cuda")
    a.infer(feat, ga)
    b.infer(feat, gb)
    assert torch.equal(ga, gb)
    assert np.array_equal(a.get_params(), b.get_params())


def test_gradient_against_reference():
    P = _random_net(5)
    net = cvw.Mlp(cvw.pack_params(P))
    rng = np.random.default_rng(9)
    N = 300
    X = bf16_round(rng.normal(size=(N, N_FEAT)))
    t = rng.uniform(size=N).astype(np.float32).astype(np.float64)
    idx = rng.integers(0, N, size=100)                 # ragged batch with repeats
    feat = _float_to_bits(X.reshape(-1))
    grad = torch.zeros(cvw.MLP_NPARAM, device="cuda")
    ws = cvw.Mlp.train_workspace(len(idx))
    net.train_step(feat, _dev(t), torch.from_numpy(idx.astype(np.int32)).cuda(), 0.0, ws, grad_out=grad)
    G = cvw.unpack_params(grad.cpu().numpy())
    _, Go = mlp_loss_grad(bf16_weights(P), X[idx], t[idx])
    for k in Go:
        scale = np.abs(Go[k]).max()
        assert np.abs(G[k] - Go[k]).max() <= 2e-4 * scale, (k, np.abs(G[k] - Go[k]).max(), scale)
    # lr = 0 leaves the parameters unchanged
    assert np.array_equal(net.get_params(), cvw.pack_params(P))


def test_adam_step():
    P = _random_net(6)
    net = cvw.Mlp(cvw.pack_params(P))
    rng = np.random.default_rng(2)
    N = 64
    X = bf16_round(rng.normal(size=(N, N_FEAT)))
    t = rng.uniform(size=N).astype(np.float32).astype(np.float64)
    idx = np.arange(N)
    ws = cvw.Mlp.train_workspace(N)
    grad = torch.zeros(cvw.MLP_NPARAM, device="cuda")
    lr = 1e-3
    net.train_step(_float_to_bits(X.reshape(-1)), _dev(t), torch.from_numpy(idx.astype(np.int32)).cuda(), lr, ws,
                   grad_out=grad)
    g = grad.cpu().numpy().astype(np.float64)
    before = cvw.pack_params(P).astype(np.float64)
    after = net.get_params().astype(np.float64)
    want = before - lr * g / (np.abs(g) + 1e-8)
    assert np.all(np.abs(after - want) <= 1e-6 * lr + 3e-7 * np.abs(before) + 1e-9)


@pytest.mark.parametrize("p", [2, 3])
def test_learned_residual_equals_reference_with_same_gamma(p):
    mesh = synth.quad_mesh(16, 12)
    sp = build_space(mesh, p, 1, 4)
    U = f32(euler_state(sp, k=6.0))
    prm = Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0))
    net = cvw.Mlp(cvw.pack_params(_random_net(7)))
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0), sensor=cvw.LEARNED), mlp=net,
                         sigma_ref=0.5)
    ws = cvw.alloc_workspace(gm, cp, 0)
    Ud = _dev(U)
    R = torch.empty_like(Ud)
    gam = torch.empty(sp.E, dtype=torch.float32, device="cuda")
    cvw.residual(gm, cp, Ud, R, gam, ws)
    g = gam.cpu().numpy().astype(np.float64)
    assert g.min() >= 0.0 and g.max() <= 1.0 and g.std() > 0
    R_o = o_residual(sp, U, prm, gamma=g).reshape(4, -1)
    keep = np.repeat(np.abs(g - 0.9) >= 1e-4, sp.ref.n_loc)
    R = R.cpu().numpy().reshape(4, -1)
    for v in range(4):
        assert rel_err(R[v][keep], R_o[v][keep]) < 1e-5, v
    # gamma of cvw_sensor equals the network on the device's own features
    cand = torch.empty((mesh.n_vertices, len(sp.ks)), dtype=torch.float32, device="cuda")
    cvw.vertex_candidates(gm, cp, Ud, cand, ws)
    feat = torch.empty((sp.E, 48), dtype=torch.int16, device="cuda")
    cvw.mlp_features(gm, cp, Ud, cand, feat)
    g2 = torch.empty(sp.E, dtype=torch.float32, device="cuda")
    net.infer(feat, g2)
    assert torch.equal(g2, gam)
