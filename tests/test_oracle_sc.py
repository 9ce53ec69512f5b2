"""Pins of the oracle's shock-capturing quadrature weights alpha_q (Sec. 4)."""
import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space
from oracle.method import sensor_gamma, sc_weights, projected_gradient, residual
from oracle.basis import RefSeg


def _rough_state(sp, seed):
    """Smooth data plus a jump, so that some cells have gamma_e < 0.9."""
    xn = sp.node_coords()
    x = xn[..., 0]
    y = xn[..., 1] if sp.ref.dim == 2 else 0.51 + 0.0 * x
    return np.sin(2 * np.pi * x) * np.cos(2 * np.pi * y) + 2.0 * ((x - 0.43) ** 2 + (y - 0.51) ** 2 < 0.06)


@pytest.mark.parametrize("cell,p,kind,jit", [
    (synth.QUAD, 3, 1, 0.0), (synth.QUAD, 2, 0, 0.1), (synth.TRI, 3, 1, 0.1), (synth.SEG, 4, 1, 0.0)])
def test_dissipation_rate_preserved(cell, p, kind, jit):
    """sum_q w_q alpha_q f_q = sum_q w_q f_q on every cell (eq. dissratescaled = eq. dissrateorig)."""
    if cell == synth.SEG:
        mesh = synth.segment_mesh(24)
    else:
        mk = synth.tri_mesh if cell == synth.TRI else synth.quad_mesh
        mesh = mk(10, 10, jitter=jit, seed=5)
    sp = build_space(mesh, p, kind)
    if kind == 1:
        u = _rough_state(sp, 1)
    else:
        ug = synth.random_nodal(sp.n_dof, 1, 0.05)
        u = sp.to_cells(ug)[0] + _rough_state(sp, 1)
        # make the CG data continuous: re-gather from a global vector
        g = np.zeros(sp.n_dof)
        g[sp.cell_dof.ravel()] = u.ravel()
        u = sp.to_cells(g)[0]
    prm = Params()
    gamma = sensor_gamma(sp, u, prm)
    pg = None
    if kind == 0:
        from oracle.method import map_points  # noqa: F401
        PGn = projected_gradient(sp, u[None])
        phi = sp.ref.deriv(sp.ref.vol_pts, (0,) * sp.ref.dim)
        pg = np.einsum("qj,ejd->eqd", phi, PGn[0][sp.cell_dof])
    alpha, parts = sc_weights(sp, u, gamma, prm, pg, return_parts=True)
    act = parts["active"]
    assert act.sum() >= 2
    W, f = parts["W"], parts["f"]
    lhs = (W * alpha * f).sum(1)
    rhs = (W * f).sum(1)
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()
    assert (alpha[~act] == 1.0).all()
    assert (alpha >= 0).all()
    assert not np.allclose(alpha[act], 1.0)     # it does redistribute


@pytest.mark.parametrize("cell", [synth.SEG, synth.TRI])
def test_p1_weights_are_one(cell):
    """p = 1 with constant gradients (segments, triangles): alpha_q = 1 (Sec. 4 remark)."""
    mesh = synth.segment_mesh(20) if cell == synth.SEG else synth.tri_mesh(8, 8, jitter=0.1, seed=2)
    sp = build_space(mesh, 1, 1)
    u = _rough_state(sp, 2)
    prm = Params()
    gamma = sensor_gamma(sp, u, prm)
    alpha, parts = sc_weights(sp, u, gamma, prm, return_parts=True)
    assert parts["active"].sum() >= 2
    assert np.abs(alpha - 1.0).max() < 1e-12


def test_quadweights_figure_shape():
    """Fig. quadweights setting: a 1D p=5 element with a jump at its centre.  The
    weights are symmetric, not uniform, proportional to the pointwise sensor
    ||u_h||_{x_q} (Sec. 4 remark), and the uniform rule is recovered with SC off."""
    mesh = synth.segment_mesh(3, -1.5, 1.5)
    sp = build_space(mesh, 5, 1)
    xn = sp.node_coords()[..., 0]
    u = (xn > 0).astype(float)
    prm = Params()
    gamma = sensor_gamma(sp, u, prm)
    assert gamma[1] < 0.9
    alpha, parts = sc_weights(sp, u, gamma, prm, return_parts=True)
    a = alpha[1]
    assert np.allclose(a, a[::-1], rtol=1e-12)
    assert a.max() / a.min() > 1.05
    ratio = a / parts["atil"][1]
    assert np.allclose(ratio, ratio[0], rtol=1e-12)
    assert (sc_weights(sp, u, gamma, Params(sc_on=0)) == 1.0).all()


def test_sc_inactive_when_smooth():
    """All gamma_e >= 0.9: SC on and SC off give identical residuals (Sec. 5.2)."""
    mesh = synth.segment_mesh(32)
    sp = build_space(mesh, 3, 0)
    from oracle import nodal_interpolate
    U = nodal_interpolate(sp, [lambda x: np.sin(2 * np.pi * x[..., 0])])
    p_on = Params(flux=synth.BURGERS, flux_param=(1.0, 0, 0, 0), sc_on=1)
    p_off = Params(flux=synth.BURGERS, flux_param=(1.0, 0, 0, 0), sc_on=0)
    R1, parts = residual(sp, U, p_on, return_parts=True)
    assert parts["gamma"].min() >= 0.9
    R0 = residual(sp, U, p_off)
    assert np.array_equal(R1, R0)
