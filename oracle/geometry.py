"""Cell maps and physical derivatives D^k u on a cell (oracle, test infrastructure only).

The paper works on affine meshes (Sec. 2.1); on those every D^k u with
|k| <= p is obtained from reference derivatives of the same order by the chain
rule with the constant inverse Jacobian A = J^{-1}:

    d^n u / dx_{a1}..dx_{an} = sum_{b1..bn} A_{b1 a1} .. A_{bn an} d^n u / dxi_{b1}..dxi_{bn}.

Hexahedra are trilinear maps of [-1, 1]^3 (affine for the boxes of the
structured meshes used here).  Jittered quadrilaterals are bilinear, not affine (a reading of the paper for
that workload): there the second derivatives gain the term of the inverse
map's Hessian,

    d^2 u / dx_a dx_c = sum_{bd} A_ba A_dc u_{,bd} + sum_b u_{,b} d^2 xi_b / dx_a dx_c,
    d^2 xi_b / dx_a dx_c = - sum_{m n s} A_bm (d^2 x_m / dxi_n dxi_s) A_sc A_na,

and orders above two are not supported on non-affine cells.
"""
from __future__ import annotations

import itertools

import numpy as np


def map_jacobian(cell: int, X: np.ndarray, pts: np.ndarray):
    """Jacobian J[E, n, d, d] (J_ab = dx_a / dxi_b) and map Hessian H[E, n, d, d, d]
    (H_mns = d^2 x_m / dxi_n dxi_s) at reference points pts [n, d].

    X: [E, v_e, d] unwrapped vertex coordinates.
    """
    E = X.shape[0]
    n = pts.shape[0]
    if cell == 1:
        J = ((X[:, 1, 0] - X[:, 0, 0]) / 2.0)[:, None, None, None] * np.ones((1, n, 1, 1))
        return J, np.zeros((E, n, 1, 1, 1))
    if cell == 2:
        J1 = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0]], axis=-1)   # [E, d, 2]
        J = np.broadcast_to(J1[:, None], (E, n, 2, 2)).copy()
        return J, np.zeros((E, n, 2, 2, 2))
    if cell == 4:
        return _trilinear_jacobian(X, pts)
    if cell == 5:
        J1 = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=-1)   # [E, 3, 3]
        return np.broadcast_to(J1[:, None], (E, n, 3, 3)).copy(), np.zeros((E, n, 3, 3, 3))
    # bilinear quadrilateral, reference vertices (-1,-1),(1,-1),(1,1),(-1,1)
    s = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], dtype=np.float64)
    xi, eta = pts[:, 0], pts[:, 1]
    dNdxi = 0.25 * s[None, :, 0] * (1 + s[None, :, 1] * eta[:, None])     # [n, 4]
    dNdeta = 0.25 * s[None, :, 1] * (1 + s[None, :, 0] * xi[:, None])
    J = np.empty((E, n, 2, 2))
    J[:, :, :, 0] = np.einsum("nv,evd->end", dNdxi, X)
    J[:, :, :, 1] = np.einsum("nv,evd->end", dNdeta, X)
    cross = 0.25 * np.einsum("v,evd->ed", s[:, 0] * s[:, 1], X)          # d^2 x / dxi deta
    H = np.zeros((E, n, 2, 2, 2))
    H[:, :, :, 0, 1] = cross[:, None, :]
    H[:, :, :, 1, 0] = cross[:, None, :]
    return J, H


_HEX_S = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                   [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)


def _trilinear_shape(pts):
    """Shape functions N_v = prod_a (1 + s_va xi_a) / 8 [n, 8], their first
    derivatives [n, 8, 3] and second derivatives [n, 8, 3, 3] (zero diagonal)."""
    f = 1.0 + _HEX_S[None, :, :] * pts[:, None, :]              # [n, 8, 3]
    N = f.prod(-1) / 8.0
    dN = np.empty(f.shape)
    d2N = np.zeros(f.shape + (3,))
    for a in range(3):
        o = [b for b in range(3) if b != a]
        dN[:, :, a] = _HEX_S[None, :, a] * f[:, :, o[0]] * f[:, :, o[1]] / 8.0
        for b in o:
            c = 3 - a - b
            d2N[:, :, a, b] = _HEX_S[None, :, a] * _HEX_S[None, :, b] * f[:, :, c] / 8.0
    return N, dN, d2N


def _trilinear_jacobian(X, pts):
    _, dN, d2N = _trilinear_shape(np.asarray(pts, np.float64))
    J = np.einsum("nva,evm->enma", dN, X)
    H = np.einsum("nvab,evm->enmab", d2N, X)
    return J, H


def map_points(cell: int, X: np.ndarray, pts: np.ndarray):
    """Physical coordinates [E, n, d] of reference points pts [n, d]."""
    if cell == 4:
        N, _, _ = _trilinear_shape(np.asarray(pts, np.float64))
        return np.einsum("nv,evd->end", N, X)
    if cell == 5:
        J1 = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=-1)
        return X[:, None, 0, :] + np.einsum("edk,nk->end", J1, np.asarray(pts, np.float64))
    if cell == 1:
        return (X[:, 0, 0][:, None] + 0.5 * (pts[None, :, 0] + 1.0) * (X[:, 1, 0] - X[:, 0, 0])[:, None])[..., None]
    if cell == 2:
        return (X[:, 0][:, None, :] + pts[None, :, 0:1] * (X[:, 1] - X[:, 0])[:, None, :]
                + pts[None, :, 1:2] * (X[:, 2] - X[:, 0])[:, None, :])
    s = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], dtype=np.float64)
    N = 0.25 * (1 + s[None, :, 0] * pts[:, 0:1]) * (1 + s[None, :, 1] * pts[:, 1:2])   # [n, 4]
    return np.einsum("nv,evd->end", N, X)


def ref_multi(dim: int, seq):
    """Reference multi-index counting how often each direction occurs in seq."""
    return tuple(sum(1 for b in seq if b == a) for a in range(dim))


def physical_derivatives(ref, cell: int, X: np.ndarray, u: np.ndarray, pts: np.ndarray, ks):
    """D^k u (|k| >= 1) at reference points for every multi-index k in ks.

    u: [E, n_loc] nodal values; returns dict k -> [E, n].
    """
    dim = ref.dim
    J, H = map_jacobian(cell, X, pts)
    A = np.linalg.inv(J)                         # A_ba = dxi_b / dx_a
    # derivatives of order >= 1 annihilate constants: take them of the data
    # relative to its first nodal value, so that constant data gives exactly 0
    u = u - u[:, :1]
    cache = {}

    def refd(m):
        if m not in cache:
            cache[m] = np.einsum("ej,nj->en", u, ref.deriv(pts, m))
        return cache[m]

    nonaffine = np.abs(H).max() > 1e-12 * np.abs(J).max()
    out = {}
    for k in ks:
        order = sum(k)
        aseq = [a for a in range(dim) for _ in range(k[a])]
        val = np.zeros(u.shape[:1] + (len(pts),))
        for bseq in itertools.product(range(dim), repeat=order):
            coef = np.ones_like(val)
            for a, b in zip(aseq, bseq):
                coef = coef * A[:, :, b, a]
            val = val + coef * refd(ref_multi(dim, bseq))
        if order == 2 and nonaffine:
            a, c = aseq
            # + sum_b u_{,b} d^2 xi_b / dx_a dx_c
            for b in range(dim):
                hxi = -np.einsum("enm,enmqs,ens,enq->en",
                                 A[:, :, b, :], H, A[:, :, :, c], A[:, :, :, a])
                val = val + refd(ref_multi(dim, [b])) * hxi
        elif order >= 3 and nonaffine:
            raise NotImplementedError("derivatives of order >= 3 on non-affine cells")
        out[k] = val
    return out


def basis_gradients(ref, cell: int, X: np.ndarray, pts: np.ndarray):
    """Physical gradients of the basis functions [E, n, n_loc, d] and |det J| [E, n]."""
    J, _ = map_jacobian(cell, X, pts)
    A = np.linalg.inv(J)
    dim = ref.dim
    G = np.stack([ref.deriv(pts, tuple(int(i == b) for i in range(dim))) for b in range(dim)], axis=-1)
    grad = np.einsum("njb,enba->enja", G, A)
    return grad, np.abs(np.linalg.det(J))
