"""Training and use of the learned smoothness sensor, through the C ABI only.

The network replaces the cell-vertex WENO sensor gamma_e (Sec. 3.2, eq. gamma)
by a prediction from normalised cell and vertex Hermite data; it is trained on
gamma_e of the method itself (the plain sensor) at snapshots of runs of the
method.  Every step runs in the library's kernels: the time steps, the plain
sensor, the features, and the network's forward and backward passes.

    snapshots: collect(mesh, prm, u, ...) -> (features [n, 48] bfloat16 bits, gamma [n])
    training:  train(net, feats, targets, epochs, batch, lr, seed)
    scale:     sigma_reference(mesh, prm, u) = max_e ||s^e||_e of a state
"""
from __future__ import annotations

import numpy as np

from . import cvw

N_FEAT = cvw.MLP_IN


def _torch():
    import torch
    return torch


def init_params(seed: int) -> np.ndarray:
    """Packed float32 parameters: weights N(0, 1/fan_in), zero biases."""
    rng = np.random.default_rng(seed)
    P = {"W1": rng.normal(size=(cvw.MLP_IN, cvw.MLP_HID)) / np.sqrt(cvw.MLP_IN), "b1": np.zeros(cvw.MLP_HID),
         "W2": rng.normal(size=(cvw.MLP_HID, cvw.MLP_HID)) / np.sqrt(cvw.MLP_HID), "b2": np.zeros(cvw.MLP_HID),
         "w3": rng.normal(size=cvw.MLP_HID) / np.sqrt(cvw.MLP_HID), "b3": np.zeros(1)}
    return cvw.pack_params(P)


def features_of(mesh, cp, u, ws=None):
    """Features of every cell of state u (int16 device tensor [E, 48] of bfloat16 bits)."""
    torch = _torch()
    E, nk = mesh.info["n_cells"], mesh.info["n_k"]
    if ws is None:
        ws = cvw.alloc_workspace(mesh, cp, 0)
    cand = torch.empty((mesh.info["n_vertices"], nk), dtype=torch.float32, device=u.device)
    cvw.vertex_candidates(mesh, cp, u, cand, ws)
    feat = torch.empty((E, N_FEAT), dtype=torch.int16, device=u.device)
    cvw.mlp_features(mesh, cp, u, cand, feat)
    return feat


def sigma_reference(mesh, cp, u) -> float:
    """max_e sigma_e of the state (sigma_e from the features computed with a
    unit reference scale: feature 45 is log10(sigma_e / 1))."""
    torch = _torch()
    params = cvw.ParamsC.from_buffer_copy(cp)
    params.sigma_ref = 1.0
    f = features_of(mesh, params, u)
    col = f[:, 45].to(torch.int32) & 0xFFFF
    vals = (col << 16).view(torch.float32)
    return float(10.0 ** vals.max().item())


def plain_gamma(mesh, cp_plain, u, ws=None):
    torch = _torch()
    if ws is None:
        ws = cvw.alloc_workspace(mesh, cp_plain, 0)
    g = torch.empty(mesh.info["n_cells"], dtype=torch.float32, device=u.device)
    cvw.sensor(mesh, cp_plain, u, g, None, ws)
    return g


def collect(mesh, prm, u, dt: float, n_snap: int, every: int, sigma_ref: float):
    """Snapshots of a plain-sensor run from state u (modified in place): at
    steps 0, every, 2 every, ... the features (scale sigma_ref) and gamma_e."""
    torch = _torch()
    cp = cvw.make_params(prm, sigma_ref=sigma_ref)
    ws = cvw.alloc_workspace(mesh, cp, 1)
    feats, gams = [], []
    for k in range(n_snap):
        if k:
            cvw.step(mesh, cp, u, dt, every, ws)
        feats.append(features_of(mesh, cp, u, ws))
        gams.append(plain_gamma(mesh, cp, u, ws))
    torch.cuda.synchronize()
    return torch.cat(feats), torch.cat(gams)


def balanced_batches(targets: np.ndarray, batch: int, n_batches: int, seed: int, frac: float = 0.5,
                     cut: float = 0.99) -> np.ndarray:
    """Row indices [n_batches, batch]: a fraction `frac` drawn from the cells
    with gamma < cut (the sensor is active there), the rest from all others."""
    rng = np.random.default_rng(seed)
    hot = np.nonzero(targets < cut)[0]
    cold = np.nonzero(targets >= cut)[0]
    nh = int(round(frac * batch)) if len(hot) and len(cold) else (batch if len(hot) else 0)
    out = np.empty((n_batches, batch), np.int32)
    for b in range(n_batches):
        a = rng.choice(hot, nh) if nh else np.empty(0, np.int64)
        c = rng.choice(cold, batch - nh) if batch - nh else np.empty(0, np.int64)
        out[b] = rng.permutation(np.concatenate([a, c]))
    return out


def feature_box(feats, margin: float = 0.25):
    """Per-feature range of a feature set (int16 device tensor of bfloat16
    bits), widened by `margin` times its span on either side: the network's
    validity box (outside it the plain sensor decides)."""
    torch = _torch()
    v = ((feats.to(torch.int32) & 0xFFFF) << 16).view(torch.float32)
    lo = v.min(0).values.cpu().numpy().astype(np.float64)
    hi = v.max(0).values.cpu().numpy().astype(np.float64)
    span = hi - lo
    return (lo - margin * span).astype(np.float32), (hi + margin * span).astype(np.float32)


def train(net, feats, targets, epochs: int, batch: int = 4096, lr: float = 1e-3, seed: int = 4):
    """Adam on mean squared error against the plain sensor, balanced batches,
    then the network's validity box from the training features; returns the
    step count (the losses are not read back)."""
    torch = _torch()
    n = feats.shape[0]
    per_epoch = max(1, n // batch)
    idx = balanced_batches(targets.cpu().numpy(), batch, epochs * per_epoch, seed)
    idx_d = torch.from_numpy(idx).to(feats.device)
    ws = cvw.Mlp.train_workspace(batch)
    for b in range(idx.shape[0]):
        net.train_step(feats, targets, idx_d[b], lr, ws)
    net.set_range(*feature_box(feats))
    torch.cuda.synchronize()
    return idx.shape[0]


def predict(net, feats):
    torch = _torch()
    g = torch.empty(feats.shape[0], dtype=torch.float32, device=feats.device)
    net.infer(feats, g)
    return g
