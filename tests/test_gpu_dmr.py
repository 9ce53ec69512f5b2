"""GPU: the double Mach reflection setting of Sec. 5.4 at reduced size, stage
by stage through the public entry points, against the float64 oracle.

DG Q2 on (0, 4) x (0, 1) with 32 x 8 cells; a Mach 10 shock at 60 degrees to
the bottom wall; inflow of the post-shock state at the left side and on the
bottom for x < 1/6, a reflecting wall on the rest of the bottom, outflow on
the right, and on the top the post-shock state left of the moving shock and
the pre-shock state right of it, rewritten before every stage for the
stage's time (SSP-RK3 stage times t, t + dt, t + dt / 2); the Zhang-Shu
positivity limiter after every stage, as in the paper's run.

The initial state (the nodal interpolant of the jump) is limited once before
the first stage: its polynomials overshoot to negative pressure at face
points, which no later limiting can repair once a cell mean has gone
negative.  The limiter's floor is eps0 = 1e-4 rather than Zhang and Shu's
1e-13: the float32 state resolves the pressure of these cells to about
1e-7 (E - |m|^2 / 2 rho with E near 2.5), so a pressure limited to 1e-13
comes back with either sign and the next stage flags it.

Ten steps: the state within 1e-3 (L1, per variable) of the oracle's run (the
oracle itself moves by 1.3e-6 under a 1e-7 relative perturbation of its
initial data; the limiter acts on 8 cells at the start and on about 150
cell-stages after), positive density and pressure at the nodes, no status
flags.
"""
import numpy as np
import pytest

import synth
from synth import Params
from oracle import build_space, nodal_interpolate, positivity_limit
from oracle import residual as o_residual
from oracle.method import boundary_faces, face_geometry, time_derivative, wave_speed
from tests.parity_helpers import f32

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_2601_16911_amd import cvw  # noqa: E402

G = 1.4
EPS0 = 1e-4          # the limiter's floor (see above)


def _setup(ny=8, p=2):
    mesh = synth.quad_mesh(4 * ny, ny, x1=4.0, periodic=(False, False))
    sp = build_space(mesh, p, 1, 4)
    U0 = f32(nodal_interpolate(sp, [(lambda c: (lambda x: synth.u0_dmr(x[..., 0], x[..., 1])[c]))(c)
                                    for c in range(4)]))
    cells, faces = boundary_faces(sp)
    mid = np.empty((len(cells), 2))
    nrm = np.empty((len(cells), 2))
    for b, (e, f) in enumerate(zip(cells, faces)):
        X = sp.X[e]
        mid[b] = 0.5 * (X[f] + X[(f + 1) % 4])
        nrm[b] = face_geometry(sp, f)[0][e]

    def prm_at(t):
        k, s = synth.dmr_boundary(mid, nrm, t)
        return Params(flux=synth.EULER, flux_param=(G, 0, 0, 0), bc_face_kind=k, bc_face_state=f32(s))

    lam = wave_speed(prm_at(0.0), sp.to_cells(U0), sp.node_coords()).max()
    dt = 0.1 * (1.0 / ny) / ((2 * p + 1) * lam)
    return mesh, sp, U0, prm_at, dt


def _oracle_run(sp, U, prm_at, dt, steps):
    def pos(V, prm):
        return positivity_limit(sp, V.reshape(4, sp.E, -1), prm, eps0=EPS0).reshape(-1)
    U = pos(U, prm_at(0.0))
    t = 0.0
    for _ in range(steps):
        U1 = pos(U + dt * time_derivative(sp, U, prm_at(t)), prm_at(t))
        U2 = pos(0.75 * U + 0.25 * (U1 + dt * time_derivative(sp, U1, prm_at(t + dt))), prm_at(t))
        U = pos(U / 3.0 + 2.0 / 3.0 * (U2 + dt * time_derivative(sp, U2, prm_at(t + 0.5 * dt))), prm_at(t))
        t += dt
    return U


def test_double_mach_setting_stage_by_stage():
    p, steps = 2, 10
    mesh, sp, U0, prm_at, dt = _setup(p=p)
    gm = cvw.Mesh(mesh, p, cvw.DG)
    assert gm.info["n_bfaces"] == len(prm_at(0.0).bc_face_kind)
    cp = cvw.make_params(prm_at(0.0))
    ws = cvw.alloc_workspace(gm, cp, cvw.OP_STEP)
    wp = cvw.alloc_workspace(gm, cp, cvw.OP_POS)
    cand = torch.zeros(gm.info["n_vertices"] * gm.info["n_k"], dtype=torch.float32, device="cuda")
    V = torch.from_numpy(np.ascontiguousarray(U0, np.float32)).cuda()
    V1, V2 = torch.empty_like(V), torch.empty_like(V)
    cvw.positivity(gm, cp, V, V, EPS0, wp)
    t = 0.0
    for _ in range(steps):
        for (us, un, uo, a0, b0, ts) in ((V, None, V1, 0.0, 1.0, t), (V1, V, V2, 0.75, 0.25, t + dt),
                                         (V2, V, V, 1.0 / 3.0, 2.0 / 3.0, t + 0.5 * dt)):
            cvw.set_boundary_data(cp, states=prm_at(ts).bc_face_state)
            cvw.vertex_candidates(gm, cp, us, cand, ws)
            cvw.rk_stage(gm, cp, us, cand, un, uo, dt, a0, b0, ws)
            cvw.positivity(gm, cp, uo, uo, EPS0, wp)
        t += dt
    assert cvw.poll_status(gm, ws) == 0
    got = V.cpu().numpy().astype(np.float64)
    ref = _oracle_run(sp, U0.copy(), prm_at, dt, steps)
    d = np.abs(got - ref).reshape(4, -1).sum(1) / np.abs(ref).reshape(4, -1).sum(1)
    assert (d <= 1e-3).all(), d
    c = got.reshape(4, -1)
    pr = (G - 1.0) * (c[3] - 0.5 * (c[1] ** 2 + c[2] ** 2) / c[0])
    assert c[0].min() > 0 and pr.min() > 0
    # the run moved the state, and the moving top data mattered
    assert (np.abs(got - U0).reshape(4, -1).sum(1) > 1e-3 * np.abs(U0).reshape(4, -1).sum(1)).all()


def test_boundary_rewrite_is_seen_by_the_next_call():
    """set_boundary_data between two residual calls: the second residual is
    the oracle's for the new data (stream order, no stale copy)."""
    p = 2
    mesh, sp, U0, prm_at, dt = _setup(ny=4, p=p)
    gm = cvw.Mesh(mesh, p, cvw.DG)
    cp = cvw.make_params(prm_at(0.0))
    ws = cvw.alloc_workspace(gm, cp, 0)
    u = torch.from_numpy(np.ascontiguousarray(U0, np.float32)).cuda()
    R = torch.empty_like(u)
    for t in (0.0, 0.05):
        cvw.set_boundary_data(cp, states=prm_at(t).bc_face_state)
        cvw.residual(gm, cp, u, R, None, ws)
        R_o, parts = o_residual(sp, U0, prm_at(t), return_parts=True)
        keep = np.repeat(np.abs(parts["gamma"] - 0.9) >= 1e-4, sp.ref.n_loc)
        Rg, Ro = R.cpu().numpy().astype(np.float64).reshape(4, -1), R_o.reshape(4, -1)
        for v in range(4):
            assert np.abs(Rg[v][keep] - Ro[v][keep]).max() <= 1e-5 * np.abs(Ro[v]).max(), (t, v)
    assert cvw.poll_status(gm, ws) == 0
