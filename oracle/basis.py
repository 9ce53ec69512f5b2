"""Reference elements, nodal Lagrange bases and quadrature rules (oracle).

Readings fixed here (the paper names no basis or rule, Sec. 2.1 and Sec. 4
only require "a nodal basis" and "a quadrature rule"):

* segments / quadrilaterals, DG: Lagrange basis at the p+1 Gauss-Legendre
  points per direction; volume rule = the same (p+1)^d Gauss points
  (collocated, so the element mass matrix is diagonal and exact).
* segments / quadrilaterals, CG: Lagrange basis at the p+1 Gauss-Lobatto
  points per direction (vertices are nodes); volume rule = (p+1)^d Gauss points.
* triangles: Lagrange basis at the equispaced points (i/p, j/p), i+j<=p;
  volume rule = the (p+1)^2-point conical-product (Stroud) rule, exact for
  total degree 2p+1.
* face rules: p+1 Gauss points on [-1, 1].

All routines are plain numpy in float64.
"""
from __future__ import annotations

import math

import numpy as np
from numpy.polynomial import legendre as npleg
from scipy.special import roots_jacobi


def gauss_legendre(n: int):
    """n-point Gauss-Legendre rule on [-1, 1]."""
    x, w = npleg.leggauss(n)
    return x.astype(np.float64), w.astype(np.float64)


def gauss_lobatto(n: int):
    """n-point Gauss-Lobatto-Legendre rule on [-1, 1] (n >= 2)."""
    if n == 2:
        return np.array([-1.0, 1.0]), np.array([1.0, 1.0])
    P = npleg.Legendre.basis(n - 1)
    inner = np.sort(P.deriv().roots().real)
    x = np.concatenate([[-1.0], inner, [1.0]])
    w = 2.0 / (n * (n - 1) * P(x) ** 2)
    return x, w


class Lagrange1D:
    """Lagrange polynomials l_j on the given nodes, with derivatives of any order.

    Each l_j is held as a Legendre series: with V[i, n] = P_n(x_i) the
    Legendre-Vandermonde matrix of the nodes, l_j = sum_n (V^{-1})[n, j] P_n.
    For Gauss and Gauss-Lobatto nodes V is well conditioned at every degree
    (cond(V) ~ 10 at p = 32), whereas monomial coefficients of l_j lose about
    five digits there; derivatives are taken term by term on the series.
    """

    def __init__(self, nodes):
        self.nodes = np.asarray(nodes, dtype=np.float64)
        n = len(self.nodes)
        self.coef = np.linalg.inv(npleg.legvander(self.nodes, n - 1))      # [n (mode), n (j)]

    def __call__(self, x, order: int = 0):
        """Matrix [len(x), n] of d^order l_j / dx^order evaluated at x."""
        x = np.atleast_1d(np.asarray(x, dtype=np.float64))
        c = npleg.legder(self.coef, order, axis=0) if order > 0 else self.coef
        if c.shape[0] == 0:
            return np.zeros((len(x), self.coef.shape[1]))
        return npleg.legval(x, c).T


def stroud_triangle(n: int):
    """n*n-point conical-product rule on the triangle (0,0),(1,0),(0,1).

    Collapsed coordinates xi = a (1 - b), eta = b with a, b in [0, 1]; Gauss-
    Legendre in a and Gauss-Jacobi (weight 1-b) in b.  Exact for total
    degree 2n-1.  Point index = ia + n * ib.
    """
    xa, wa = gauss_legendre(n)
    a = 0.5 * (xa + 1.0)
    wa = 0.5 * wa
    xb, wb = roots_jacobi(n, 1.0, 0.0)
    b = 0.5 * (xb + 1.0)
    wb = wb / 4.0
    pts, wts = [], []
    for ib in range(n):
        for ia in range(n):
            pts.append((a[ia] * (1.0 - b[ib]), b[ib]))
            wts.append(wa[ia] * wb[ib])
    return np.array(pts), np.array(wts)


def stroud_tet(n: int):
    """n^3-point conical-product rule on the tetrahedron (0,0,0), (1,0,0),
    (0,1,0), (0,0,1): collapsed coordinates x = a (1 - b)(1 - c),
    y = b (1 - c), z = c with Gauss-Legendre in a, Gauss-Jacobi with weight
    (1 - b) in b and (1 - c)^2 in c (all on [0, 1]).  Exact for total degree
    2n - 1.  Point index = ia + n (ib + n ic)."""
    xa, wa = gauss_legendre(n)
    a, wa = 0.5 * (xa + 1.0), 0.5 * wa
    xb, wb = roots_jacobi(n, 1.0, 0.0)
    b, wb = 0.5 * (xb + 1.0), wb / 4.0
    xc, wc = roots_jacobi(n, 2.0, 0.0)
    c, wc = 0.5 * (xc + 1.0), wc / 8.0
    pts, wts = [], []
    for ic in range(n):
        for ib in range(n):
            for ia in range(n):
                pts.append((a[ia] * (1.0 - b[ib]) * (1.0 - c[ic]), b[ib] * (1.0 - c[ic]), c[ic]))
                wts.append(wa[ia] * wb[ib] * wc[ic])
    return np.array(pts), np.array(wts)


def radon_triangle():
    """Radon's 7-point rule of degree 5 on the triangle (0,0),(1,0),(0,1),
    symmetric under every permutation of the vertices: the centroid and two
    orbits of three points, barycentric (a, a, 1 - 2a) with
    a = (6 -+ sqrt 15) / 21, weights 9/40 and (155 -+ sqrt 15) / 1200 of the
    area (1/2).  Returns points [7, 2] (the last two barycentric coordinates)
    and weights [7]."""
    r = math.sqrt(15.0)
    bary = [(1 / 3, 1 / 3, 1 / 3)]
    wts = [9 / 40]
    for a, w in (((6 - r) / 21, (155 - r) / 1200), ((6 + r) / 21, (155 + r) / 1200)):
        b = 1.0 - 2.0 * a
        bary += [(a, a, b), (a, b, a), (b, a, a)]
        wts += [w, w, w]
    bary = np.array(bary)
    return bary[:, 1:], 0.5 * np.array(wts)


def multi_indices(dim: int, p: int):
    """Derivative multi-indices k with 1 <= |k| <= p, ordered by |k|, then by
    decreasing first component, then decreasing second: (1,0),(0,1),(2,0),
    (1,1),(0,2),... in 2D; (1,0,0),(0,1,0),(0,0,1),(2,0,0),(1,1,0),(1,0,1),
    (0,2,0),... in 3D."""
    out = []
    for n in range(1, p + 1):
        if dim == 1:
            out.append((n,))
        elif dim == 2:
            for j in range(n + 1):
                out.append((n - j, j))
        else:
            for a in range(n, -1, -1):
                for b in range(n - a, -1, -1):
                    out.append((a, b, n - a - b))
    return out


class RefSeg:
    dim = 1
    n_vert = 2
    n_faces = 2

    def __init__(self, p: int, nodes: str):
        self.p = p
        x, _ = gauss_legendre(p + 1) if nodes == "gauss" else gauss_lobatto(p + 1)
        self.x1d = x
        self.L = Lagrange1D(x)
        self.n_loc = p + 1
        self.nodes = x[:, None]
        self.vertices = np.array([[-1.0], [1.0]])
        qx, qw = gauss_legendre(p + 1)
        self.vol_pts, self.vol_w = qx[:, None], qw
        qx2, qw2 = gauss_legendre(p + 2)
        self.norm_pts, self.norm_w = qx2[:, None], qw2

    def deriv(self, pts, m):
        return self.L(np.asarray(pts)[:, 0], m[0])

    def face_points(self, f):
        """Face f (0 = left vertex, 1 = right vertex): reference points of the face rule, weights."""
        return self.vertices[f][None, :], np.array([1.0])


class RefQuad:
    dim = 2
    n_vert = 4
    n_faces = 4

    def __init__(self, p: int, nodes: str):
        self.p = p
        x, _ = gauss_legendre(p + 1) if nodes == "gauss" else gauss_lobatto(p + 1)
        self.x1d = x
        self.L = Lagrange1D(x)
        self.n_loc = (p + 1) ** 2
        X, Y = np.meshgrid(x, x, indexing="xy")       # index a + (p+1) b
        self.nodes = np.stack([X.ravel(), Y.ravel()], axis=1)
        self.vertices = np.array([[-1.0, -1.0], [1.0, -1.0], [1.0, 1.0], [-1.0, 1.0]])
        qx, qw = gauss_legendre(p + 1)
        QX, QY = np.meshgrid(qx, qx, indexing="xy")
        self.vol_pts = np.stack([QX.ravel(), QY.ravel()], axis=1)
        self.vol_w = np.outer(qw, qw).ravel()
        qx2, qw2 = gauss_legendre(p + 2)
        QX2, QY2 = np.meshgrid(qx2, qx2, indexing="xy")
        self.norm_pts = np.stack([QX2.ravel(), QY2.ravel()], axis=1)
        self.norm_w = np.outer(qw2, qw2).ravel()
        self.face_x, self.face_w = gauss_legendre(p + 1)

    def deriv(self, pts, m):
        pts = np.asarray(pts)
        Lx = self.L(pts[:, 0], m[0])          # [n, p+1]
        Ly = self.L(pts[:, 1], m[1])
        return (Lx[:, None, :] * Ly[:, :, None]).reshape(len(pts), -1)

    def face_points(self, f):
        """Face f joins local vertices f and f+1 (mod 4); points ordered from vertex f to f+1."""
        s = self.face_x
        a, b = self.vertices[f], self.vertices[(f + 1) % 4]
        pts = 0.5 * (1 - s)[:, None] * a + 0.5 * (1 + s)[:, None] * b
        return pts, self.face_w


class RefTri:
    dim = 2
    n_vert = 3
    n_faces = 3

    def __init__(self, p: int, nodes: str = "equispaced"):
        self.p = p
        self.n_loc = (p + 1) * (p + 2) // 2
        nd = []
        for j in range(p + 1):
            for i in range(p + 1 - j):
                nd.append((i / p, j / p) if p > 0 else (1 / 3, 1 / 3))
        self.nodes = np.array(nd)
        self.mono = [(a, n - a) for n in range(p + 1) for a in range(n, -1, -1)]
        V = np.stack([self.nodes[:, 0] ** a * self.nodes[:, 1] ** b for a, b in self.mono], axis=1)
        self.Vinv = np.linalg.inv(V)      # column j = monomial coefficients of phi_j
        self.vertices = np.array([[0.0, 0.0], [1.0, 0.0], [0.0, 1.0]])
        self.vol_pts, self.vol_w = stroud_triangle(p + 1)
        self.norm_pts, self.norm_w = self.vol_pts, self.vol_w
        self.face_x, self.face_w = gauss_legendre(p + 1)

    def deriv(self, pts, m):
        pts = np.asarray(pts)
        cols = []
        for a, b in self.mono:
            if a < m[0] or b < m[1]:
                cols.append(np.zeros(len(pts)))
                continue
            ca = np.prod(np.arange(a - m[0] + 1, a + 1)) if m[0] else 1.0
            cb = np.prod(np.arange(b - m[1] + 1, b + 1)) if m[1] else 1.0
            cols.append(ca * cb * pts[:, 0] ** (a - m[0]) * pts[:, 1] ** (b - m[1]))
        M = np.stack(cols, axis=1)
        return M @ self.Vinv

    def face_points(self, f):
        s = self.face_x
        a, b = self.vertices[f], self.vertices[(f + 1) % 3]
        pts = 0.5 * (1 - s)[:, None] * a + 0.5 * (1 + s)[:, None] * b
        # the face rule on [-1,1] is scaled to the reference edge by the physical
        # edge length / 2 in the caller
        return pts, self.face_w


class RefHex:
    """Tensor-product Lagrange element on [-1, 1]^3 (DG: Gauss-Legendre nodes),
    local node a + (p+1) b + (p+1)^2 c (x fastest).  Vertices in the order of
    the mesh: the face z = -1 counter-clockwise from (-1,-1), then z = +1.
    Faces: 2 axis + side (0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z); the points of a
    face are the tensor Gauss rule in its two tangential directions, the
    lower axis fastest, so that opposite faces share one parametrisation."""
    dim = 3
    n_vert = 8
    n_faces = 6

    def __init__(self, p: int, nodes: str):
        self.p = p
        x, _ = gauss_legendre(p + 1) if nodes == "gauss" else gauss_lobatto(p + 1)
        self.x1d = x
        self.L = Lagrange1D(x)
        self.n_loc = (p + 1) ** 3
        self.nodes = self._tensor(x)
        self.vertices = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                                  [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], dtype=np.float64)
        qx, qw = gauss_legendre(p + 1)
        self.vol_pts = self._tensor(qx)
        self.vol_w = np.einsum("c,b,a->cba", qw, qw, qw).ravel()
        qx2, qw2 = gauss_legendre(p + 2)
        self.norm_pts = self._tensor(qx2)
        self.norm_w = np.einsum("c,b,a->cba", qw2, qw2, qw2).ravel()
        self.face_x, self.face_w1 = gauss_legendre(p + 1)

    @staticmethod
    def _tensor(x):
        Z, Y, X = np.meshgrid(x, x, x, indexing="ij")          # x fastest
        return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)

    def deriv(self, pts, m):
        pts = np.asarray(pts)
        Lx = self.L(pts[:, 0], m[0])
        Ly = self.L(pts[:, 1], m[1])
        Lz = self.L(pts[:, 2], m[2])
        return (Lz[:, :, None, None] * Ly[:, None, :, None] * Lx[:, None, None, :]).reshape(len(pts), -1)

    def face_points(self, f):
        axis, side = divmod(f, 2)
        t = [a for a in range(3) if a != axis]
        s = self.face_x
        S1, S0 = np.meshgrid(s, s, indexing="ij")             # t[0] fastest
        pts = np.empty((S0.size, 3))
        pts[:, axis] = 1.0 if side else -1.0
        pts[:, t[0]] = S0.ravel()
        pts[:, t[1]] = S1.ravel()
        return pts, np.outer(self.face_w1, self.face_w1).ravel()


class RefTet:
    """Lagrange P_p on the tetrahedron (0,0,0), (1,0,0), (0,1,0), (0,0,1) at
    the equispaced lattice points (i, j, k) / p, i + j + k <= p, ordered with
    i fastest, then j, then k.  Face f is opposite vertex f; its points are
    Radon's degree-5 rule on its three vertices (weights summing to 1/2, the
    area of the parameter triangle).  The rule is symmetric under the
    permutations of a triangle's vertices, so the two cells of a face
    integrate over one and the same set of points (conservation), whatever
    the order in which each holds the face's vertices."""
    dim = 3
    n_vert = 4
    n_faces = 4
    FACE_VERTICES = [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]

    def __init__(self, p: int, nodes: str = "equispaced"):
        self.p = p
        nd = []
        for k in range(p + 1):
            for j in range(p + 1 - k):
                for i in range(p + 1 - j - k):
                    nd.append((i / p, j / p, k / p))
        self.nodes = np.array(nd)
        self.n_loc = len(nd)
        self.mono = [(a, b, n - a - b) for n in range(p + 1) for a in range(n, -1, -1) for b in range(n - a, -1, -1)]
        V = np.stack([self.nodes[:, 0] ** a * self.nodes[:, 1] ** b * self.nodes[:, 2] ** c for a, b, c in self.mono], axis=1)
        self.Vinv = np.linalg.inv(V)      # column j = monomial coefficients of phi_j
        self.vertices = np.array([[0.0, 0.0, 0.0], [1.0, 0.0, 0.0], [0.0, 1.0, 0.0], [0.0, 0.0, 1.0]])
        self.vol_pts, self.vol_w = stroud_tet(p + 1)
        self.norm_pts, self.norm_w = self.vol_pts, self.vol_w
        self.face_st, self.face_w = radon_triangle()

    def deriv(self, pts, m):
        pts = np.asarray(pts)
        cols = []
        for a, b, c in self.mono:
            if a < m[0] or b < m[1] or c < m[2]:
                cols.append(np.zeros(len(pts)))
                continue
            f = math.perm(a, m[0]) * math.perm(b, m[1]) * math.perm(c, m[2])
            cols.append(f * pts[:, 0] ** (a - m[0]) * pts[:, 1] ** (b - m[1]) * pts[:, 2] ** (c - m[2]))
        return np.stack(cols, axis=1) @ self.Vinv

    def face_points(self, f):
        va, vb, vc = (self.vertices[i] for i in self.FACE_VERTICES[f])
        s, t = self.face_st[:, 0:1], self.face_st[:, 1:2]
        return va + s * (vb - va) + t * (vc - va), self.face_w


def make_ref(cell: int, p: int, space: int):
    """cell: 1 segment, 2 triangle, 3 quadrilateral, 4 hexahedron, 5 tetrahedron; space: 0 CG, 1 DG."""
    if cell == 5:
        if space != 1:
            raise NotImplementedError("tetrahedra: DG only")
        return RefTet(p)
    if cell == 4:
        if space != 1:
            raise NotImplementedError("hexahedra: DG only")
        return RefHex(p, "gauss")
    if cell == 1:
        return RefSeg(p, "lobatto" if space == 0 else "gauss")
    if cell == 3:
        return RefQuad(p, "lobatto" if space == 0 else "gauss")
    if cell == 2:
        return RefTri(p)
    raise ValueError(cell)
