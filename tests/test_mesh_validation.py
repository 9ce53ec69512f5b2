"""Mesh validation on the host (cvw_mesh_plan runs the whole build without a
device): meshes the method is not defined on are refused before any device
memory is touched."""
import numpy as np
import pytest

import synth
from paper_2601_16911_amd import cvw


@pytest.mark.parametrize("shape", [(2, 2), (2, 5), (5, 2)])
def test_periodic_width_two_rejected(shape):
    """Two cells that meet across both of their faces in a periodic direction
    of width 2: a face is then not determined by its vertices, which the
    face-neighbour tables (and the oracle) require."""
    with pytest.raises(cvw.CvwError) as ei:
        cvw.mesh_plan(synth.quad_mesh(*shape), 2, cvw.DG)
    assert ei.value.status == cvw.EINVAL
    assert "non-conforming" in str(ei.value)


@pytest.mark.parametrize("shape", [(1, 1), (1, 3), (3, 1)])
def test_periodic_width_one_rejected(shape):
    """One cell across a periodic direction: two corners of the cell are the
    same mesh vertex, so the cell would enter that vertex's patch twice, at two
    different corners."""
    with pytest.raises(cvw.CvwError) as ei:
        cvw.mesh_plan(synth.quad_mesh(*shape), 2, cvw.DG)
    assert ei.value.status == cvw.EINVAL
    assert "repeated vertex" in str(ei.value)


def test_empty_mesh_rejected():
    desc = synth.MeshDesc(2, synth.QUAD, 0, np.zeros((0, 4), np.int32), np.zeros((0, 4, 2)), (0, 0))
    with pytest.raises(cvw.CvwError) as ei:
        cvw.mesh_plan(desc, 2, cvw.DG)
    assert ei.value.status == cvw.EINVAL
    assert "empty" in str(ei.value)


@pytest.mark.parametrize("shape", [(1, 1), (1, 3), (3, 1), (3, 3)])
def test_small_meshes_accepted(shape):
    """Small meshes whose cells have four distinct vertices are valid: without
    periodicity down to one cell, periodic from width 3."""
    assert cvw.mesh_plan(synth.quad_mesh(*shape, periodic=(False, False)), 2, cvw.DG) > 0
    if min(shape) >= 3:
        assert cvw.mesh_plan(synth.quad_mesh(*shape), 2, cvw.DG) > 0
