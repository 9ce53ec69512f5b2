"""Pins of the oracle's Zhang-Shu positivity limiter (the limiter the paper
adds for its double Mach reflection run, Sec. 5): properties that fix the
scaling without restating its formulas.

* admissible states are returned bit for bit;
* cell averages are preserved;
* afterwards density and pressure are >= eps at every point of the set
  (Gauss nodes and face Gauss points), with equality at the worst point of a
  limited cell: theta is the largest admissible scaling (optimality);
* one factor per cell and step scales every variable and node (the limited
  state is a point of the segment between the cell average and the input).
"""
import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space, positivity_limit
from oracle.method import _face_trace_matrix, _pressure
from tests.parity_helpers import euler_state

EULER = Params(flux=synth.EULER, flux_param=(1.4, 0, 0, 0))


def inadmissible_state(p, seed=0, cell=synth.QUAD):
    """The four-quadrant Euler data with negative density at one node of some
    cells and negative pressure at one node of others (cell averages stay
    admissible); quadrilaterals or jittered triangles."""
    if cell == synth.TRI:
        mesh = synth.tri_mesh(8, 7, jitter=0.1, seed=4)
    else:
        mesh = synth.quad_mesh(10, 9)
    sp = build_space(mesh, p, 1, 4)
    U = sp.to_cells(euler_state(sp, k=200.0)).copy()
    rng = np.random.default_rng(seed)
    n = sp.ref.n_loc
    cells = rng.choice(sp.E, 24, replace=False)
    for c in cells[:12]:
        j = rng.integers(n)
        U[0, c, j] = -0.3 * U[0, c].mean()
    for c in cells[12:]:
        j = rng.integers(n)
        kin = 0.5 * (U[1, c, j] ** 2 + U[2, c, j] ** 2) / U[0, c, j]
        U[3, c, j] = kin - 0.5 * U[3, c].mean()
    return sp, U, cells


def _points(sp, V):
    if sp.cell == synth.TRI:
        ref = sp.ref
        B = np.concatenate([ref.deriv(ref.vol_pts, (0, 0))] + [ref.deriv(ref.face_points(f)[0], (0, 0))
                                                                 for f in range(3)])
        return V @ B.T
    return np.concatenate([V, V @ _face_trace_matrix(sp).T], axis=-1)


def _means(sp, U):
    if sp.cell == synth.TRI:
        # exact cell average of the element polynomial: a degree-2p Gauss rule
        # on the collapsed square, independent of the volume rule
        ref = sp.ref
        g, w = np.polynomial.legendre.leggauss(sp.p + 2)
        a, b = np.meshgrid((g + 1) / 2, (g + 1) / 2, indexing="xy")
        pts = np.stack([(a * (1 - b)).ravel(), b.ravel()], axis=1)
        wt = (np.outer(w, w) / 4 * (1 - b)).ravel() * 2.0        # weights of the unit-area triangle average
        return np.einsum("ven,n->ve", U, wt @ ref.deriv(pts, (0, 0)))
    w1 = np.polynomial.legendre.leggauss(sp.p + 1)[1]
    return np.einsum("ven,n->ve", U, np.outer(w1, w1).ravel() / 4.0)


CELLS = [synth.QUAD, synth.TRI]


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("p", [1, 2, 3])
def test_admissible_states_unchanged(p, cell):
    mesh = synth.tri_mesh(8, 7, jitter=0.1, seed=4) if cell == synth.TRI else synth.quad_mesh(10, 9)
    sp = build_space(mesh, p, 1, 4)
    U = sp.to_cells(euler_state(sp, k=10.0))
    Q = np.stack([_points(sp, U[v]) for v in range(4)])
    assert Q[0].min() > 0 and _pressure(Q, 1.4).min() > 0
    assert np.array_equal(positivity_limit(sp, U, EULER), U)


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("p", [1, 2, 3])
def test_positivity_restored_optimally(p, cell):
    sp, U, cells = inadmissible_state(p, cell=cell)
    gam = 1.4
    m0 = _means(sp, U)
    eps = np.minimum(1e-13, np.minimum(m0[0], _pressure(m0, gam)))
    Q0 = np.stack([_points(sp, U[v]) for v in range(4)])
    bad = (Q0[0].min(1) < eps) | (_pressure(Q0, gam).min(1) < eps)
    assert bad.sum() >= 20 and m0[0].min() > 0 and _pressure(m0, gam).min() > 0
    out = positivity_limit(sp, U, EULER)
    # conservation
    assert np.abs(_means(sp, out) - m0).max() < 1e-13 * np.abs(m0).max()
    Q = np.stack([_points(sp, out[v]) for v in range(4)])
    rho, pr = Q[0], _pressure(Q, gam)
    scale = np.abs(m0).max()
    assert (rho.min(1) >= eps - 1e-12 * scale).all()
    assert (pr.min(1) >= eps - 1e-12 * scale).all()
    # optimal: the worst point of a limited cell sits on the bound
    worst = np.minimum(rho.min(1) - eps, pr.min(1) - eps)
    assert np.abs(worst[bad]).max() < 1e-10 * scale
    # untouched elsewhere
    assert np.array_equal(out[:, ~bad], U[:, ~bad])


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("p", [2, 3])
def test_single_factor_per_cell(p, cell):
    """Cells whose density is admissible and pressure is not: the result is
    mean + theta (U - mean) with one theta for every variable and node."""
    sp, U, cells = inadmissible_state(p, seed=3, cell=cell)
    m0 = _means(sp, U)
    out = positivity_limit(sp, U, EULER)
    for c in cells[12:]:
        d_in = U[:, c, :] - m0[:, c, None]
        d_out = out[:, c, :] - m0[:, c, None]
        big = np.abs(d_in) > 1e-6 * np.abs(U[:, c, :]).max()
        th = d_out[big] / d_in[big]
        assert th.max() - th.min() < 1e-9
        assert 0.0 <= th.min() < 1.0
