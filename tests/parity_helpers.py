"""Shared helpers of the GPU parity tests: run the HIP path through the C ABI
and the oracle on the same float32-rounded inputs."""
from __future__ import annotations

import numpy as np

import synth
from oracle import build_space, nodal_interpolate


def rel_err(a, b, axis=None):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    return np.abs(a - b).max(axis=axis) / max(np.abs(b).max(), 1e-300)


def f32(x):
    """Round to float32 and back (the inputs both sides see)."""
    return np.asarray(x, np.float32).astype(np.float64)


def rough_scalar(sp, seed=0):
    """Smooth field plus a disc-shaped jump: some cells troubled, some smooth."""
    xn = sp.node_coords()
    x, y = xn[..., 0], xn[..., 1]
    g = synth.smooth_field(x, y, seed)
    return g + 1.5 * (((x - 0.45) ** 2 + (y - 0.55) ** 2) < 0.07)


def euler_state(sp, k=60.0):
    return nodal_interpolate(sp, [(lambda c: (lambda x: synth.euler_state_config4(
        x[..., 0], x[..., 1], smooth_k=k)[c]))(c) for c in range(4)])


def subset_ring(mesh, cells):
    """All cells sharing a vertex with one of `cells` (the data the residual of
    those cells depends on) as a non-periodic sub-mesh; returns (submesh,
    original ids of its cells, positions of `cells` in it)."""
    cv = mesh.cell_vertices
    verts = np.unique(cv[cells].ravel())
    mask = np.isin(cv, verts).any(axis=1)
    sub = np.nonzero(mask)[0]
    used = np.unique(cv[sub].ravel())
    remap = -np.ones(mesh.n_vertices, np.int64)
    remap[used] = np.arange(len(used))
    desc = synth.MeshDesc(mesh.dim, mesh.cell, len(used), remap[cv[sub]].astype(np.int32),
                          mesh.cell_coords[sub], (0, 0))
    pos = np.searchsorted(sub, cells)
    return desc, sub, pos


def oracle_space(mesh, p, kind, nv=1):
    return build_space(mesh, p, kind, nv)
