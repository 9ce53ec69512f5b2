"""A finite element space on a mesh description (oracle, test infrastructure only).

Holds the reference element, the connectivity (vertex patches, DG face
neighbours, CG numbering) and per-cell geometry: h_e = diam(K_e), the largest
distance between two vertices of the (convex) cell (Sec. 2.1).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .basis import make_ref, multi_indices
from .mesh import vertex_patches, face_neighbours, cg_numbering
from .geometry import map_points


@dataclass
class Space:
    mesh: object
    p: int
    kind: int            # 0 CG, 1 DG
    n_var: int
    ref: object
    ks: list
    patch_ptr: np.ndarray
    patch_cell: np.ndarray
    patch_lv: np.ndarray
    h: np.ndarray
    nbr: np.ndarray | None = None
    nbr_face: np.ndarray | None = None
    cell_dof: np.ndarray | None = None
    n_dof: int = 0

    @property
    def E(self):
        return self.mesh.n_cells

    @property
    def X(self):
        return self.mesh.cell_coords

    @property
    def cell(self):
        return self.mesh.cell

    def node_coords(self):
        """Physical coordinates of the local nodes [E, n_loc, dim]."""
        return map_points(self.cell, self.X, self.ref.nodes)

    def to_cells(self, U):
        """Global state -> per-cell nodal values [n_var, E, n_loc]."""
        U = np.asarray(U, dtype=np.float64).reshape(self.n_var, -1)
        if self.kind == 1:
            return U.reshape(self.n_var, self.E, self.ref.n_loc)
        return U[:, self.cell_dof]

    def state_size(self):
        return self.n_var * (self.E * self.ref.n_loc if self.kind == 1 else self.n_dof)


def build_space(mesh, p: int, kind: int, n_var: int = 1) -> Space:
    ref = make_ref(mesh.cell, p, kind)
    ptr, pc, plv = vertex_patches(mesh.cell_vertices, mesh.n_vertices)
    X = mesh.cell_coords
    diffs = X[:, :, None, :] - X[:, None, :, :]
    h = np.sqrt((diffs ** 2).sum(-1)).max(axis=(1, 2))
    sp = Space(mesh, p, kind, n_var, ref, multi_indices(ref.dim, p), ptr, pc, plv, h)
    if kind == 1:
        sp.nbr, sp.nbr_face = face_neighbours(mesh.cell, mesh.cell_vertices)
    else:
        sp.cell_dof, sp.n_dof = cg_numbering(mesh.cell, p, mesh.cell_vertices, mesh.n_vertices)
    return sp
