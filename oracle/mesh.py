"""Mesh connectivity for the oracle (test infrastructure only).

* vertex patches C(x_i) = {cells containing vertex x_i} (Sec. 3.2), stored as
  a CSR list of (cell, local vertex) pairs per vertex in ascending
  (cell, local vertex) order;
* face neighbours for DG interface terms (eq. convop);
* the canonical CG numbering: vertex DOFs by vertex id, then edge DOFs by edge
  (edges sorted by (min id, max id), oriented min -> max), then cell-interior
  DOFs by cell id.  The paper fixes no numbering; this one is a reading.
"""
from __future__ import annotations

import numpy as np


def vertex_patches(cell_vertices: np.ndarray, n_vertices: int):
    """CSR (ptr [N_v+1], cell [nnz], local_vertex [nnz]) sorted by (vertex, cell, lv)."""
    E, nv = cell_vertices.shape
    vid = cell_vertices.ravel().astype(np.int64)
    cells = np.repeat(np.arange(E), nv)
    lvs = np.tile(np.arange(nv), E)
    order = np.lexsort((lvs, cells, vid))
    counts = np.bincount(vid, minlength=n_vertices)
    ptr = np.zeros(n_vertices + 1, np.int64)
    ptr[1:] = np.cumsum(counts)
    return ptr, cells[order], lvs[order]


def face_vertex_pairs(cell: int, cell_vertices: np.ndarray):
    """[E, n_faces, 2] vertex ids of each face, ordered along the cell boundary."""
    E, nv = cell_vertices.shape
    if cell == 1:
        return cell_vertices[:, :, None]          # faces are the two vertices
    a = cell_vertices
    b = np.roll(cell_vertices, -1, axis=1)
    return np.stack([a, b], axis=2)


# local vertices of the six faces of a hexahedron, face 2 axis + side
# (0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z), vertex order of synth.hex_mesh
HEX_FACE_VERTICES = np.array([[0, 3, 7, 4], [1, 2, 6, 5], [0, 1, 5, 4], [3, 2, 6, 7],
                              [0, 1, 2, 3], [4, 5, 6, 7]])


# local vertices of the four faces of a tetrahedron, face f opposite vertex f
TET_FACE_VERTICES = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])


def hex_face_neighbours(cell_vertices: np.ndarray, table=HEX_FACE_VERTICES):
    """(nbr [E, F], nbr_face [E, F]) of 3D cells whose faces are the vertex
    sets of `table` (hexahedra by default): two faces match when they hold the
    same vertices; -1 on boundary faces."""
    E = cell_vertices.shape[0]
    F = len(table)
    fv = np.sort(cell_vertices[:, table], axis=2).astype(np.int64)   # [E, F, nv]
    keys = {}
    for e in range(E):
        for f in range(F):
            keys.setdefault(tuple(fv[e, f]), []).append((e, f))
    nbr = -np.ones((E, F), np.int64)
    nbr_face = -np.ones((E, F), np.int64)
    for ents in keys.values():
        if len(ents) > 2:
            raise ValueError("non-conforming mesh: face shared by more than two cells")
        if len(ents) == 2:
            (e0, f0), (e1, f1) = ents
            nbr[e0, f0], nbr_face[e0, f0] = e1, f1
            nbr[e1, f1], nbr_face[e1, f1] = e0, f0
    return nbr, nbr_face


def face_neighbours(cell: int, cell_vertices: np.ndarray):
    """(nbr [E, F], nbr_face [E, F]); -1 on boundary faces.

    Two faces match when they join the same vertex pair; in a conforming,
    consistently oriented mesh the neighbour traverses the shared face in the
    opposite direction, which is checked here.
    """
    if cell == 4:
        return hex_face_neighbours(cell_vertices)
    if cell == 5:
        return hex_face_neighbours(cell_vertices, TET_FACE_VERTICES)
    E = cell_vertices.shape[0]
    fv = face_vertex_pairs(cell, cell_vertices)
    F = fv.shape[1]
    if cell == 1:
        key = fv[:, :, 0].astype(np.int64)
    else:
        lo = np.minimum(fv[:, :, 0], fv[:, :, 1]).astype(np.int64)
        hi = np.maximum(fv[:, :, 0], fv[:, :, 1]).astype(np.int64)
        key = lo * (int(cell_vertices.max()) + 1) + hi
    flat = key.ravel()
    order = np.argsort(flat, kind="stable")
    sk = flat[order]
    same = sk[1:] == sk[:-1]
    if np.any(same[1:] & same[:-1]):
        raise ValueError("non-conforming mesh: face shared by more than two cells")
    i = np.nonzero(same)[0]
    a, b = order[i], order[i + 1]
    e0, f0 = np.divmod(a, F)
    e1, f1 = np.divmod(b, F)
    if cell != 1:
        ok = (fv[e0, f0, 0] == fv[e1, f1, 1]) & (fv[e0, f0, 1] == fv[e1, f1, 0])
        if not ok.all():
            raise ValueError("inconsistently oriented shared face")
    nbr = -np.ones((E, F), np.int64)
    nbr_face = -np.ones((E, F), np.int64)
    nbr[e0, f0], nbr_face[e0, f0] = e1, f1
    nbr[e1, f1], nbr_face[e1, f1] = e0, f0
    return nbr, nbr_face


def cg_numbering(cell: int, p: int, cell_vertices: np.ndarray, n_vertices: int):
    """(cell_dof [E, n_loc], n_dof) for Gauss-Lobatto CG spaces on segments and quads."""
    E = cell_vertices.shape[0]
    if cell == 1:
        n_loc = p + 1
        cd = np.empty((E, n_loc), np.int64)
        cd[:, 0] = cell_vertices[:, 0]
        cd[:, p] = cell_vertices[:, 1]
        for t in range(1, p):
            cd[:, t] = n_vertices + np.arange(E) * (p - 1) + (t - 1)
        return cd, n_vertices + E * (p - 1)
    if cell != 3:
        raise NotImplementedError("CG numbering implemented for segments and quadrilaterals")
    n1 = p + 1
    cd = -np.ones((E, n1 * n1), np.int64)

    def loc(a, b):
        return a + n1 * b

    corners = [(0, 0), (p, 0), (p, p), (0, p)]
    for lv, (a, b) in enumerate(corners):
        cd[:, loc(a, b)] = cell_vertices[:, lv]
    # edges
    fv = face_vertex_pairs(3, cell_vertices)
    lo = np.minimum(fv[:, :, 0], fv[:, :, 1]).astype(np.int64)
    hi = np.maximum(fv[:, :, 0], fv[:, :, 1]).astype(np.int64)
    keys = np.stack([lo.ravel(), hi.ravel()], axis=1)
    uniq, inv = np.unique(keys, axis=0, return_inverse=True)
    edge_id = inv.reshape(E, 4)
    n_edges = len(uniq)

    def edge_node(f, t):   # t = 1..p-1, counted from vertex f towards vertex f+1
        return [(t, 0), (p, t), (p - t, p), (0, p - t)][f]

    for f in range(4):
        same = fv[:, f, 0] < fv[:, f, 1]
        for t in range(1, p):
            g = np.where(same, t - 1, p - 1 - t)
            a, b = edge_node(f, t)
            cd[:, loc(a, b)] = n_vertices + edge_id[:, f] * (p - 1) + g
    base = n_vertices + n_edges * (p - 1)
    ni = (p - 1) * (p - 1)
    for b in range(1, p):
        for a in range(1, p):
            cd[:, loc(a, b)] = base + np.arange(E) * ni + (a - 1) + (p - 1) * (b - 1)
    assert (cd >= 0).all()
    return cd, base + E * ni
