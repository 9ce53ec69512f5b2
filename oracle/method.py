"""The cell-vertex WENO stabilised scheme, step by step, in float64 (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every function follows
the paper's definitions in its order and notation:

* Hermite data D^k u_h^{e'}(x_i), 1 <= |k| <= p, of each cell at each of its
  vertices: the Taylor expansion eq. (taylorsol), Sec. 3.2;
* vertex smoothness indicators beta_{e'}^i = ||u_h^{e'}||_{x_i}^q with the
  pointwise semi-norm eq. (pointsnorm), Jiang-Shu weights with equal linear
  weights, eps = 1e-6, r = 2, and the vertex candidate eq. (taylorcand);
* cell candidates u_{h,l}^e (the vertex Taylor polynomials), their element
  semi-norms eq. (snorm), the nonlinear weights with linear weights 1e-3 for
  the vertex candidates and 1 - v_e 1e-3 for the cell candidate, the
  reconstruction eq. (finalweno) and the sensor eq. (gamma), Sec. 2.2 / 3.2;
* low-order viscosity nu_e = lambda_e h_e / (2p), eq. (lostab);
* the shock-capturing quadrature weights alpha_q, eqs. (dissrateorig) to
  (alpha_prelim), used only where gamma_e < C_gamma (Sec. 5);
* the stabilised residual of eq. (stabform) / (sdstab) with the DG form
  (P_h = identity on gradients, so s^H = 0) or the simplified CG form
  nu_e (grad v, grad u - gamma_e P_h grad u), and LLF / HLL interface fluxes;
* the mass matrix solve and the three-stage SSP Runge-Kutta method;
* the reconstruction used as an HWENO limiter (Sec. 3): on cells with gamma_e
  below a threshold, u_h^e is overwritten by u_h^{e,*} built from vertex
  candidates with corrected cell averages (Sec. 3.2), componentwise.

Readings of points the paper leaves open:
q = 1 for every exponent, lambda_e = max of the wave speed over the volume
quadrature points, h_e = diam(K_e) of the cell whose polynomial is measured,
gamma_e = 1 when ||u_h^e||_e = 0, alpha_q = 1 when either sum in eq. (alphaq)
is not positive, P_h for CG = nodal averaging of the broken gradient, exact
element mass for DG and the consistent global mass for CG.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sps
import scipy.sparse.linalg as spla

from synth import Params, ADVECT_CONST, ADVECT_ROT, BURGERS, KPP, EULER, BC_NONE, BC_OUTFLOW, BC_WALL, BC_INFLOW
from .geometry import physical_derivatives, map_jacobian, map_points, basis_gradients
from .mesh import face_neighbours


# ---------------------------------------------------------------------------
# semi-norms
# ---------------------------------------------------------------------------
def _orders(sp):
    return np.array([sum(k) for k in sp.ks], dtype=np.float64)


def pointwise_seminorm(sp, D, h):
    """eq. (pointsnorm): (sum_k h^{2|k|} |D^k v(x)|^2)^{1/2}; D [..., n_k], h broadcastable."""
    w = h[..., None] ** (2.0 * _orders(sp))
    return np.sqrt((w * D * D).sum(-1))


def element_seminorm_sq(sp, D, W):
    """eq. (snorm) squared: sum_k h_e^{2|k|-d} int_K |D^k v|^2, with D [E, nq, n_k]
    sampled at the cell's semi-norm rule and W [E, nq] its physical weights."""
    d = sp.ref.dim
    w = sp.h[:, None] ** (2.0 * _orders(sp) - d)          # [E, n_k]
    return np.einsum("eq,eqk,ek->e", W, D * D, w)


# ---------------------------------------------------------------------------
# vertex stage (Sec. 3.2)
# ---------------------------------------------------------------------------
def hermite_at_vertices(sp, s):
    """H[E, v_e, n_k] = D^k s^e(x_i) at each local vertex (eq. taylorsol)."""
    D = physical_derivatives(sp.ref, sp.cell, sp.X, s, sp.ref.vertices, sp.ks)
    return np.stack([D[k] for k in sp.ks], axis=-1)


def vertex_candidates(sp, s, prm: Params, return_weights: bool = False):
    """Vertex HWENO candidate data c_i[k] = sum_{e in C(x_i)} omega_e^i D^k s^e(x_i) (eq. taylorcand)."""
    H = hermite_at_vertices(sp, s)
    beta = pointwise_seminorm(sp, H, sp.h[:, None]) ** prm.q_beta       # [E, v_e]
    wt = (prm.eps_vertex + beta) ** (-prm.r)
    pc, plv, ptr = sp.patch_cell, sp.patch_lv, sp.patch_ptr
    w_ent = wt[pc, plv]
    row = np.repeat(np.arange(len(ptr) - 1), np.diff(ptr))
    tot = np.zeros(len(ptr) - 1)
    np.add.at(tot, row, w_ent)
    omega = w_ent / tot[row]
    c = np.zeros((len(ptr) - 1, len(sp.ks)))
    np.add.at(c, row, omega[:, None] * H[pc, plv])
    if return_weights:
        return c, omega, H, beta
    return c


# ---------------------------------------------------------------------------
# cell stage (Sec. 3.2, eq. finalweno, eq. gamma)
# ---------------------------------------------------------------------------
def taylor_derivatives(sp, coef, x, x0):
    """D^m of s(x) = sum_{k in ks} coef[k] (x - x0)^k / k! at points x, for every m in ks.

    coef [E, n_k], x [E, nq, d], x0 [E, d]; returns [E, nq, n_k].
    """
    dx = x - x0[:, None, :]
    out = np.zeros(x.shape[:2] + (len(sp.ks),))
    for im, m in enumerate(sp.ks):
        for ik, k in enumerate(sp.ks):
            if any(kk < mm for kk, mm in zip(k, m)):
                continue
            term = coef[:, ik][:, None] * np.ones(x.shape[:2])
            for a in range(len(k)):
                e = k[a] - m[a]
                term = term * dx[:, :, a] ** e / math.factorial(e)
            out[:, :, im] += term
    return out


def cell_sensor(sp, s, c, prm: Params, return_parts: bool = False):
    """gamma_e of eq. (gamma) from the cell-vertex WENO reconstruction u_h^{e,*}."""
    ref = sp.ref
    pts = ref.norm_pts
    J, _ = map_jacobian(sp.cell, sp.X, pts)
    W = ref.norm_w[None, :] * np.abs(np.linalg.det(J))
    xq = map_points(sp.cell, sp.X, pts)
    Du = physical_derivatives(ref, sp.cell, sp.X, s, pts, sp.ks)
    U = np.stack([Du[k] for k in sp.ks], axis=-1)              # [E, nq, n_k]
    ve = sp.mesh.cell_vertices.shape[1]
    S = []
    for l in range(ve):
        ci = c[sp.mesh.cell_vertices[:, l]]
        S.append(taylor_derivatives(sp, ci, xq, sp.X[:, l]))
    n0 = np.sqrt(element_seminorm_sq(sp, U, W))
    betas = [n0 ** prm.q_beta] + [np.sqrt(element_seminorm_sq(sp, Sl, W)) ** prm.q_beta for Sl in S]
    lin = [1.0 - ve * prm.lin_w_vertex] + [prm.lin_w_vertex] * ve
    wt = np.stack([g / (prm.eps_cell + b) ** prm.r for g, b in zip(lin, betas)], axis=1)
    omega = wt / wt.sum(axis=1, keepdims=True)                 # [E, v_e + 1]
    diff = np.zeros_like(U)
    for l in range(ve):
        diff += omega[:, l + 1][:, None, None] * (U - S[l])
    d = np.sqrt(element_seminorm_sq(sp, diff, W))
    with np.errstate(divide="ignore", invalid="ignore"):
        ratio = np.where(n0 > 0, d / np.where(n0 > 0, n0, 1.0), 0.0)
    gamma = np.where(n0 > 0, 1.0 - np.minimum(1.0, ratio) ** prm.q_sensor, 1.0)
    if return_parts:
        return gamma, dict(n=n0, d=d, omega=omega, betas=np.stack(betas, 1))
    return gamma


# ---------------------------------------------------------------------------
# shock-capturing quadrature (Sec. 4)
# ---------------------------------------------------------------------------
def sc_weights(sp, s, gamma, prm: Params, pg=None, return_parts: bool = False):
    """alpha_q of eq. (alphaq) at the volume quadrature points; [E, nq].

    pg: CG only, (P_h grad s)(x_q) [E, nq, d].
    """
    ref = sp.ref
    pts = ref.vol_pts
    J, _ = map_jacobian(sp.cell, sp.X, pts)
    W = ref.vol_w[None, :] * np.abs(np.linalg.det(J))
    Du = physical_derivatives(ref, sp.cell, sp.X, s, pts, sp.ks)
    D = np.stack([Du[k] for k in sp.ks], axis=-1)
    atil = pointwise_seminorm(sp, D, sp.h[:, None])            # eq. (alpha_prelim), R8
    d = ref.dim
    grad = D[:, :, :d]                                          # first-order multi-indices come first
    g2 = (grad * grad).sum(-1)
    if sp.kind == 1:
        f = (1.0 - gamma)[:, None] * g2
    else:
        f = g2 - gamma[:, None] * (grad * pg).sum(-1)
    S = (W * f).sum(1)
    T = (W * atil * f).sum(1)
    active = (prm.sc_on != 0) & (gamma < prm.c_gamma) & (S > 0) & (T > 0)
    with np.errstate(divide="ignore", invalid="ignore"):
        alpha = np.where(active[:, None], atil * (S / np.where(T > 0, T, 1.0))[:, None], 1.0)
    if return_parts:
        return alpha, dict(f=f, W=W, atil=atil, active=active)
    return alpha


# ---------------------------------------------------------------------------
# fluxes
# ---------------------------------------------------------------------------
def flux(prm: Params, U, x):
    """Physical flux f(U) [n_var, ..., d] at points x [..., d]."""
    d = x.shape[-1]
    if prm.flux in (KPP, ADVECT_ROT) and d != 2:
        raise ValueError("the KPP and rotating-advection fluxes are two-dimensional")
    if prm.flux == ADVECT_CONST:
        v = np.array(prm.flux_param[:d])
        return U[..., None] * v
    if prm.flux == ADVECT_ROT:
        cx, cy, om = prm.flux_param[0], prm.flux_param[1], prm.flux_param[2]
        v = np.stack([om * (cy - x[..., 1]), om * (x[..., 0] - cx)], axis=-1)
        return U[..., None] * v[None]
    if prm.flux == BURGERS:
        b = np.array(prm.flux_param[:d])
        return 0.5 * U[..., None] ** 2 * b
    if prm.flux == KPP:
        return np.stack([np.sin(U), np.cos(U)], axis=-1)
    if prm.flux == EULER:
        g = prm.flux_param[0]
        if d == 3:                                  # (rho, m_x, m_y, m_z, E)
            rho, mx, my, mz, En = U
            vx, vy, vz = mx / rho, my / rho, mz / rho
            p = (g - 1.0) * (En - 0.5 * rho * (vx * vx + vy * vy + vz * vz))
            F = [np.stack([m, mx * v, my * v, mz * v, (En + p) * v]) for m, v in ((mx, vx), (my, vy), (mz, vz))]
            F[0][1] += p
            F[1][2] += p
            F[2][3] += p
            return np.stack(F, axis=-1)
        if d == 1:                                  # (rho, m, E) on a line
            rho, mx, En = U
            vx = mx / rho
            p = (g - 1.0) * (En - 0.5 * rho * vx * vx)
            return np.stack([mx, mx * vx + p, (En + p) * vx])[..., None]
        rho, mx, my, En = U
        vx, vy = mx / rho, my / rho
        p = (g - 1.0) * (En - 0.5 * rho * (vx * vx + vy * vy))
        Fx = np.stack([mx, mx * vx + p, my * vx, (En + p) * vx])
        Fy = np.stack([my, mx * vy, my * vy + p, (En + p) * vy])
        return np.stack([Fx, Fy], axis=-1)
    raise ValueError(prm.flux)


def wave_speed(prm: Params, U, x):
    """Local maximum wave speed |f'(u)| (systems: |v| + c) at points; shape of U[0]."""
    d = x.shape[-1]
    if prm.flux == ADVECT_CONST:
        return np.full(U.shape[1:], float(np.linalg.norm(prm.flux_param[:d])))
    if prm.flux == ADVECT_ROT:
        cx, cy, om = prm.flux_param[0], prm.flux_param[1], prm.flux_param[2]
        return abs(om) * np.hypot(cy - x[..., 1], x[..., 0] - cx)
    if prm.flux == BURGERS:
        return np.abs(U[0]) * float(np.linalg.norm(prm.flux_param[:d]))
    if prm.flux == KPP:
        return np.ones(U.shape[1:])
    if prm.flux == EULER:
        g = prm.flux_param[0]
        vz = 0.0
        if d == 1:
            rho, mx, En = U
            vx, vy = mx / rho, 0.0
        elif d == 2:
            rho, mx, my, En = U
            vx, vy = mx / rho, my / rho
        else:
            rho, mx, my, mz, En = U
            vx, vy, vz = mx / rho, my / rho, mz / rho
        p = (g - 1.0) * (En - 0.5 * rho * (vx * vx + vy * vy + vz * vz))
        c = np.sqrt(np.maximum(g * p / rho, 0.0))
        return np.sqrt(vx * vx + vy * vy + vz * vz) + c
    raise ValueError(prm.flux)


def numerical_flux(prm: Params, Um, Up, n, x):
    """Interface flux f*(U-, U+, n) [n_var, ...]: local Lax-Friedrichs (scalar)
    or HLL with Davis wave-speed estimates (Euler)."""
    Fm = (flux(prm, Um, x) * n).sum(-1)
    Fp = (flux(prm, Up, x) * n).sum(-1)
    if prm.flux == EULER:
        g = prm.flux_param[0]

        def vn_c(U):
            vz, nz = 0.0, 0.0
            if n.shape[-1] == 1:
                rho, mx, En = U
                vx, vy, ny = mx / rho, 0.0, 0.0
            elif n.shape[-1] == 2:
                rho, mx, my, En = U
                vx, vy, ny = mx / rho, my / rho, n[..., 1]
            else:
                rho, mx, my, mz, En = U
                vx, vy, vz, ny, nz = mx / rho, my / rho, mz / rho, n[..., 1], n[..., 2]
            p = (g - 1.0) * (En - 0.5 * rho * (vx * vx + vy * vy + vz * vz))
            return vx * n[..., 0] + vy * ny + vz * nz, np.sqrt(np.maximum(g * p / rho, 0.0))

        vm, cm = vn_c(Um)
        vp, cp = vn_c(Up)
        SL = np.minimum(vm - cm, vp - cp)
        SR = np.maximum(vm + cm, vp + cp)
        with np.errstate(divide="ignore", invalid="ignore"):
            mid = (SR * Fm - SL * Fp + SL * SR * (Up - Um)) / (SR - SL)
        return np.where(SL >= 0, Fm, np.where(SR <= 0, Fp, mid))
    if prm.lambda_global > 0:
        lam = prm.lambda_global
    else:
        d = x.shape[-1]
        if prm.flux == ADVECT_CONST:
            lam = np.abs((np.array(prm.flux_param[:d]) * n).sum(-1))
        elif prm.flux == ADVECT_ROT:
            cx, cy, om = prm.flux_param[0], prm.flux_param[1], prm.flux_param[2]
            v = np.stack([om * (cy - x[..., 1]), om * (x[..., 0] - cx)], axis=-1)
            lam = np.abs((v * n).sum(-1))
        elif prm.flux == BURGERS:
            bn = np.abs((np.array(prm.flux_param[:d]) * n).sum(-1))
            lam = np.maximum(np.abs(Um[0]), np.abs(Up[0])) * bn
        elif prm.flux == KPP:
            def fpn(u):
                return np.abs(np.cos(u) * n[..., 0] - np.sin(u) * n[..., 1])
            lam = np.maximum(fpn(Um[0]), fpn(Up[0]))
        else:
            raise ValueError(prm.flux)
    return 0.5 * (Fm + Fp) - 0.5 * lam * (Up - Um)


# ---------------------------------------------------------------------------
# residual (eq. stabform / sdstab)
# ---------------------------------------------------------------------------
def projected_gradient(sp, Uc):
    """CG: nodal values of P_h grad U (average over the cells sharing each node) [n_var, n_dof, d]."""
    ref = sp.ref
    gphi, _ = basis_gradients(ref, sp.cell, sp.X, ref.nodes)    # [E, nloc(pts), nloc, d]
    g = np.einsum("vei,ejid->vejd", Uc, gphi)
    nv, d = Uc.shape[0], ref.dim
    acc = np.zeros((nv, sp.n_dof, d))
    cnt = np.bincount(sp.cell_dof.ravel(), minlength=sp.n_dof).astype(np.float64)
    for v in range(nv):
        for a in range(d):
            np.add.at(acc[v, :, a], sp.cell_dof.ravel(), g[v, :, :, a].ravel())
    return acc / cnt[None, :, None]


# ---------------------------------------------------------------------------
# HWENO limiter (Sec. 3: the cell-vertex reconstruction may overwrite u_h^e
# by u_h^{e,*}; Sec. 3.2: candidates with corrected cell averages)
# ---------------------------------------------------------------------------
def taylor_value(sp, c0, coef, x, x0):
    """s(x) = c0 + sum_{k in ks} coef[k] (x - x0)^k / k! (eq. taylorcand with its
    k = 0 term); c0 [E], coef [E, n_k], x [E, n, d], x0 [E, d]; returns [E, n]."""
    dx = x - x0[:, None, :]
    out = np.repeat(c0[:, None], x.shape[1], axis=1).astype(np.float64)
    for ik, k in enumerate(sp.ks):
        term = coef[:, ik][:, None] * np.ones(x.shape[:2])
        for a in range(len(k)):
            term = term * dx[:, :, a] ** k[a] / math.factorial(k[a])
        out += term
    return out


def hweno_limit(sp, U, prm: Params, threshold: float, gamma=None):
    """CV-WENO used as an HWENO limiter for DG: on every cell whose sensor value
    gamma_e (eq. gamma, of the sensor field U[0]) is below `threshold`, the
    nodal values of u_h^e are replaced by those of u_h^{e,*} = sum_l omega_l^e
    ubar_{h,l}^e (eq. finalweno) with the cell candidate ubar_0 = u_h^e and the
    vertex candidates with corrected cell averages,
        ubar_{h,i}^*(x) = u_{h,i}^*(x) + mean_{K_e}(u_h^e - u_{h,i}^*),
    where u_{h,i}^* is the Taylor polynomial of eq. (taylorcand) including its
    k = 0 term sum_e' omega_e'^i u_h^{e'}(x_i).  Each variable is reconstructed
    with its own candidates and weights (componentwise).

    U: [E, n_loc] (scalar) or [n_var, E, n_loc]; returns the same shape.
    threshold > 1 limits every cell, threshold <= 0 none.
    """
    scalar = np.ndim(U) == 2
    Us = np.asarray(U, np.float64)[None] if scalar else np.asarray(U, np.float64)
    if gamma is None:
        gamma = sensor_gamma(sp, Us[0], prm)
    troubled = gamma < threshold
    ref = sp.ref
    xn = sp.node_coords()                                          # [E, n_loc, d]
    pts = ref.norm_pts                                             # exact for Q_p products
    J, _ = map_jacobian(sp.cell, sp.X, pts)
    W = ref.norm_w[None, :] * np.abs(np.linalg.det(J))             # [E, nq]
    xq = map_points(sp.cell, sp.X, pts)
    Bq = ref.deriv(pts, (0,) * ref.dim)                            # values at the rule's points
    Bv = ref.deriv(ref.vertices, (0,) * ref.dim)                   # values at the vertices
    cv = sp.mesh.cell_vertices
    ve = cv.shape[1]
    pc, plv, ptr = sp.patch_cell, sp.patch_lv, sp.patch_ptr
    row = np.repeat(np.arange(len(ptr) - 1), np.diff(ptr))
    out = Us.copy()
    for v in range(Us.shape[0]):
        s = Us[v]
        c, omega_ent, _, _ = vertex_candidates(sp, s, prm, return_weights=True)
        vals = s @ Bv.T                                            # u_h^{e'}(x_i) [E, v_e]
        c0 = np.zeros(len(ptr) - 1)
        np.add.at(c0, row, omega_ent * vals[pc, plv])
        _, parts = cell_sensor(sp, s, c, prm, return_parts=True)
        om = parts["omega"]                                        # [E, v_e + 1]
        mean_u = (W * (s @ Bq.T)).sum(1) / W.sum(1)
        rec = om[:, :1] * s
        for l in range(ve):
            i = cv[:, l]
            at_nodes = taylor_value(sp, c0[i], c[i], xn, sp.X[:, l])
            at_pts = taylor_value(sp, c0[i], c[i], xq, sp.X[:, l])
            corr = mean_u - (W * at_pts).sum(1) / W.sum(1)
            rec = rec + om[:, l + 1][:, None] * (at_nodes + corr[:, None])
        out[v] = np.where(troubled[:, None], rec, s)
    return out[0] if scalar else out


# ---------------------------------------------------------------------------
# positivity limiter for the Euler equations on DG quadrilaterals (the
# Zhang-Shu limiter the paper adds in its double Mach reflection run, Sec. 5;
# restated from Zhang and Shu's published construction)
# ---------------------------------------------------------------------------
def _face_trace_matrix(sp):
    """Values at the Gauss points of the four faces (W, E, S, N; p + 1 points
    each, ordered along the face) from the nodal values: [4 (p+1), n_loc]."""
    ref = sp.ref
    n1 = sp.p + 1
    x = ref.x1d
    pts = []
    for side in ((-1.0, None), (1.0, None), (None, -1.0), (None, 1.0)):
        for t in x:
            pts.append((side[0], t) if side[0] is not None else (t, side[1]))
    return ref.deriv(np.array(pts), (0, 0))                  # [4 n1, n_loc]


def _pressure(U, gam):
    rho, mx, my, En = U
    return (gam - 1.0) * (En - 0.5 * (mx * mx + my * my) / rho)


def positivity_limit(sp, U, prm: Params, eps0: float = 1e-13, iters: int = 200):
    """Zhang-Shu scaling limiter: per cell, with the cell averages
    Ubar and the points Q (the Gauss nodes and the Gauss points of the faces),
    eps = min(eps0, rhobar, p(Ubar));
    (1) rho <- rhobar + th1 (rho - rhobar), th1 = min(1, (rhobar - eps) / (rhobar - min_Q rho));
    (2) U <- Ubar + th2 (U - Ubar), th2 = min over Q of the t in [0, 1] where
        p(Ubar + t (U_q - Ubar)) = eps (t = 1 where p(U_q) >= eps), found by
        bisection (p is concave along the segment, positive at t = 0).
    Cells with th = 1 keep their values bit for bit.
    U: [4, E, n_loc] nodal values (Euler); returns the limited values.

    Quadrilaterals: Q = the Gauss nodes (the volume rule) and the face Gauss
    points.  Triangles: Q = the points of the volume rule (where the DG scheme
    evaluates the state) and the Gauss points of the three edges; the cell
    average is the volume rule's (exact for the element's polynomials)."""
    gam = prm.flux_param[0]
    U = np.asarray(U, np.float64).copy()
    if sp.cell == 2:                                          # triangles
        ref = sp.ref
        Bv = ref.deriv(ref.vol_pts, (0, 0))                   # [nq, n_loc]
        Bq = np.concatenate([Bv] + [ref.deriv(ref.face_points(f)[0], (0, 0)) for f in range(3)])
        wn = (ref.vol_w / ref.vol_w.sum()) @ Bv               # the cell average from the nodal values
        at_pts = lambda V: V @ Bq.T
        mean = np.einsum("ven,n->ve", U, wn)
    else:
        w1 = np.polynomial.legendre.leggauss(sp.p + 1)[1]
        w = np.outer(w1, w1).ravel() / 4.0                    # collocated Gauss rule of the nodes
        F = _face_trace_matrix(sp)
        at_pts = lambda V: np.concatenate([V, V @ F.T], axis=-1)                     # nodes, then faces
        mean = np.einsum("ven,n->ve", U, w)                                         # [4, E]
    eps = np.minimum(eps0, np.minimum(mean[0], _pressure(mean, gam)))
    # (1) density
    rq = at_pts(U[0])
    rmin = rq.min(1)
    low = rmin < eps
    th1 = np.ones_like(rmin)
    th1[low] = (mean[0][low] - eps[low]) / (mean[0][low] - rmin[low])
    th1 = np.minimum(1.0, th1)
    U[0] = np.where((th1 < 1.0)[:, None], mean[0][:, None] + th1[:, None] * (U[0] - mean[0][:, None]), U[0])
    # (2) pressure
    Q = np.stack([at_pts(U[v]) for v in range(4)])                                  # [4, E, nq]
    D = Q - mean[:, :, None]
    pq = _pressure(Q, gam)
    lo = np.zeros(pq.shape)
    hi = np.ones(pq.shape)
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        ok = _pressure(mean[:, :, None] + mid[None] * D, gam) >= eps[:, None]
        lo = np.where(ok, mid, lo)
        hi = np.where(ok, hi, mid)
    t = np.where(pq >= eps[:, None], 1.0, lo)
    th2 = t.min(1)
    return np.where((th2 < 1.0)[None, :, None], mean[:, :, None] + th2[None, :, None] * (U - mean[:, :, None]), U)


def sensor_gamma(sp, s, prm: Params):
    if prm.sensor == 2:
        return np.full(sp.E, prm.fixed_gamma)
    c = vertex_candidates(sp, s, prm)
    return cell_sensor(sp, s, c, prm)


def residual(sp, U, prm: Params, gamma=None, return_parts: bool = False, allow_boundary: bool = False):
    """R with M dU/dt = -R (eq. sdstab): volume Galerkin term, stabilisation with
    the shock-capturing weights, DG interface terms, CG assembly.

    Returns R in the state layout ([n_var, E, n_loc] flattened for DG,
    [n_var, n_dof] for CG).
    """
    ref = sp.ref
    Uc = sp.to_cells(U)                           # [nv, E, nloc]
    nv = Uc.shape[0]
    s = Uc[0]
    if gamma is None:
        gamma = sensor_gamma(sp, s, prm)
    pts = ref.vol_pts
    gphi, detJ = basis_gradients(ref, sp.cell, sp.X, pts)    # [E, nq, nloc, d]
    W = ref.vol_w[None, :] * detJ
    phi = ref.deriv(pts, (0,) * ref.dim)                        # [nq, nloc]
    Uq = np.einsum("vej,qj->veq", Uc, phi)
    gU = np.einsum("vej,eqjd->veqd", Uc, gphi)
    xq = map_points(sp.cell, sp.X, pts)
    F = flux(prm, Uq, xq)                                       # [nv, E, nq, d]
    if prm.lambda_global > 0:
        lam = np.full(sp.E, prm.lambda_global)
    else:
        lam = wave_speed(prm, Uq, xq).max(axis=1)
    nu = lam * sp.h / (2.0 * sp.p)
    pg = None
    if sp.kind == 0:
        PGn = projected_gradient(sp, Uc)                        # [nv, ndof, d]
        PGq = np.einsum("qj,vejd->veqd", phi, PGn[:, sp.cell_dof])
        pg = PGq[0]
        G = gU - gamma[None, :, None, None] * PGq
    else:
        G = (1.0 - gamma)[None, :, None, None] * gU
    alpha = sc_weights(sp, s, gamma, prm, pg)
    r = (-np.einsum("eq,eqjd,veqd->vej", W, gphi, F)
         + np.einsum("e,eq,eq,eqjd,veqd->vej", nu, W, alpha, gphi, G))
    ends = any(b != BC_NONE for b in prm.bc) or prm.bc_face_kind is not None
    if sp.kind == 1:
        r = r + face_terms(sp, Uc, prm, allow_boundary or ends)
    if ends:
        r = r + boundary_terms(sp, Uc, prm)
    if sp.kind == 1:
        R = r.reshape(nv, -1)
    else:
        R = np.zeros((nv, sp.n_dof))
        for v in range(nv):
            np.add.at(R[v], sp.cell_dof.ravel(), r[v].ravel())
    if return_parts:
        return R.ravel(), dict(gamma=gamma, alpha=alpha, nu=nu, lam=lam, r_cell=r)
    return R.ravel()


def face_geometry(sp, f):
    """Outward unit normal [E, d] and face Jacobian [E] of face f (the length / 2
    of an edge; the area / 4 of a flat hexahedron face, whose reference face
    [-1, 1]^2 has area 4; twice the area of a tetrahedron face, whose
    parameter triangle has area 1/2)."""
    X = sp.X
    if sp.cell == 1:
        n = np.full((sp.E, 1), -1.0 if f == 0 else 1.0)
        return n, np.ones(sp.E)
    if sp.cell == 5:
        from .mesh import TET_FACE_VERTICES
        c = TET_FACE_VERTICES[f]
        cr = np.cross(X[:, c[1]] - X[:, c[0]], X[:, c[2]] - X[:, c[0]])
        jac = np.linalg.norm(cr, axis=1)                         # twice the area: the parameter triangle has area 1/2
        n = cr / jac[:, None]
        out = X[:, c].mean(1) - X.mean(1)
        n = np.where(((n * out).sum(1) < 0)[:, None], -n, n)
        return n, jac
    if sp.cell == 4:
        from .mesh import HEX_FACE_VERTICES
        c = HEX_FACE_VERTICES[f]
        t1 = 0.5 * (X[:, c[1]] - X[:, c[0]])
        t2 = 0.5 * (X[:, c[3]] - X[:, c[0]])
        cr = np.cross(t1, t2)
        area4 = np.linalg.norm(cr, axis=1)
        n = cr / area4[:, None]
        out = (X[:, c].mean(1) - X.mean(1))                      # from the cell centre to the face centre
        n = np.where(((n * out).sum(1) < 0)[:, None], -n, n)
        return n, area4
    nvx = X.shape[1]
    t = X[:, (f + 1) % nvx] - X[:, f]
    L = np.hypot(t[:, 0], t[:, 1])
    n = np.stack([t[:, 1], -t[:, 0]], axis=1) / L[:, None]
    return n, 0.5 * L


def face_terms(sp, Uc, prm: Params, allow_boundary: bool = False):
    """DG interface terms.  allow_boundary=True drops boundary faces; it exists
    only to evaluate the residual of interior cells of a sub-mesh cut out of a
    larger periodic mesh (those cells never touch a boundary face)."""
    ref = sp.ref
    nv, E, nloc = Uc.shape
    out = np.zeros_like(Uc)
    if (sp.nbr < 0).any() and not allow_boundary:
        raise NotImplementedError("DG residual requires a mesh without boundary faces")
    for f in range(ref.n_faces):
        pts, wf = ref.face_points(f)
        phif = ref.deriv(pts, (0,) * ref.dim)                    # [ng, nloc]
        Um = np.einsum("vej,gj->veg", Uc, phif)
        en, fn = sp.nbr[:, f], sp.nbr_face[:, f]
        Up = Um.copy()                                             # boundary faces: zero jump, dropped below
        if sp.cell == 4:
            Up[:, en >= 0] = _neighbour_traces_by_position(sp, Uc, f, en, fn)[:, en >= 0]
        elif sp.cell == 5:
            Up[:, en >= 0] = _tet_neighbour_traces(sp, Uc, f, en, fn)[:, en >= 0]
        for f2 in range(ref.n_faces if sp.cell not in (4, 5) else 0):
            sel = fn == f2
            if not sel.any():
                continue
            p2, _ = ref.face_points(f2)
            phi2 = ref.deriv(p2[::-1], (0,) * ref.dim)            # reversed traversal
            Up[:, sel] = np.einsum("vej,gj->veg", Uc[:, en[sel]], phi2)
        n, Jf = face_geometry(sp, f)
        xf = map_points(sp.cell, sp.X, pts)
        ng = len(wf)
        nb = np.broadcast_to(n[:, None, :], (E, ng, n.shape[1]))
        Fs = numerical_flux(prm, Um, Up, nb, xf)                   # [nv, E, ng]
        Fs = np.where((en >= 0)[None, :, None], Fs, 0.0)
        out += np.einsum("g,e,gj,veg->vej", wf, Jf, phif, Fs)
    return out


def _neighbour_traces_by_position(sp, Uc, f, en, fn):
    """The neighbour's trace at the points of face f of every cell [nv, E, ng].
    The points are paired by position: the neighbour's face points, moved by
    the offset between the two face centres (zero, or a period of the domain
    when the neighbour lies across a periodic boundary), must coincide with
    the cell's own."""
    ref = sp.ref
    pts, _ = ref.face_points(f)
    xf = map_points(sp.cell, sp.X, pts)                            # [E, ng, 3]
    out = np.zeros((Uc.shape[0], sp.E, len(pts)))
    for e in range(sp.E):
        if en[e] < 0:
            continue
        p2, _ = ref.face_points(int(fn[e]))
        x2 = map_points(sp.cell, sp.X[en[e]:en[e] + 1], p2)[0]
        x2 = x2 - x2.mean(0) + xf[e].mean(0)
        dist = np.linalg.norm(xf[e][:, None, :] - x2[None, :, :], axis=2)
        perm = dist.argmin(1)
        if dist[np.arange(len(pts)), perm].max() > 1e-9 * sp.h[e] or len(set(perm)) != len(pts):
            raise ValueError("face points of neighbouring cells do not coincide")
        phi2 = ref.deriv(p2[perm], (0,) * ref.dim)
        out[:, e] = np.einsum("vj,gj->vg", Uc[:, en[e]], phi2)
    return out


def _tet_neighbour_traces(sp, Uc, f, en, fn):
    """The neighbour's trace at the cell's own points of face f [nv, E, ng]:
    each point, moved by the offset between the two face centres (zero, or a
    period of the domain), is mapped into the neighbour's reference
    coordinates by the inverse of its affine map and must lie on the
    neighbour's face fn (the face rule is not symmetric under a permutation of
    the face's vertices, so the two cells' point sets differ)."""
    from .mesh import TET_FACE_VERTICES
    ref = sp.ref
    pts, _ = ref.face_points(f)
    X = sp.X
    xf = map_points(sp.cell, X, pts)                               # [E, ng, 3]
    out = np.zeros((Uc.shape[0], sp.E, len(pts)))
    for e in range(sp.E):
        if en[e] < 0:
            continue
        e2, f2 = int(en[e]), int(fn[e])
        shift = X[e2, TET_FACE_VERTICES[f2]].mean(0) - X[e, TET_FACE_VERTICES[f]].mean(0)
        J2 = np.stack([X[e2, 1] - X[e2, 0], X[e2, 2] - X[e2, 0], X[e2, 3] - X[e2, 0]], axis=-1)
        xi = np.linalg.solve(J2, (xf[e] + shift - X[e2, 0]).T).T   # [ng, 3]
        bary = np.concatenate([1.0 - xi.sum(1, keepdims=True), xi], axis=1)
        if np.abs(bary[:, f2]).max() > 1e-10 or bary.min() < -1e-10:
            raise ValueError("face points of neighbouring cells do not coincide")
        out[:, e] = np.einsum("vj,gj->vg", Uc[:, e2], ref.deriv(xi, (0, 0, 0)))
    return out


# ---------------------------------------------------------------------------
# boundary data at the ends of a 1D domain (the paper's shock-tube and blast-
# wave runs, Sec. 5.4: an inflow end and reflecting walls)
# ---------------------------------------------------------------------------
def ghost_state(prm: Params, kind: int, state, Ub, n):
    """Exterior state at boundary points of one kind: outflow copies the
    interior trace, inflow imposes the given state, a reflecting wall mirrors
    the normal momentum (Euler only).  Ub [n_var, ...], n [..., d]."""
    if kind == BC_OUTFLOW:
        return Ub.copy()
    if kind == BC_INFLOW:
        st = np.asarray(state[:Ub.shape[0]], np.float64)
        return np.broadcast_to(st.reshape((-1,) + (1,) * (Ub.ndim - 1)), Ub.shape).copy()
    if kind == BC_WALL:
        if prm.flux != EULER:
            raise ValueError("a reflecting wall needs the Euler equations")
        d = n.shape[-1]
        out = Ub.copy()
        mn = sum(Ub[1 + a] * n[..., a] for a in range(d))
        for a in range(d):
            out[1 + a] = Ub[1 + a] - 2.0 * mn * n[..., a]
        return out
    raise ValueError("boundary point without boundary data")


def boundary_state(prm: Params, Ub, n, end: int):
    """Exterior state at an end of a line (the end's kind and state)."""
    return ghost_state(prm, prm.bc[end], prm.bc_state[end], Ub, n)


def boundary_faces(sp):
    """Boundary faces (cell [nb], local face [nb]) in ascending (cell, face) order."""
    nbr = sp.nbr if sp.nbr is not None else face_neighbours(sp.cell, sp.mesh.cell_vertices)[0]
    return np.nonzero(nbr < 0)


def boundary_terms(sp, Uc, prm: Params):
    """Weak boundary terms phi_j(x_b) f*(u_h(x_b), u_ext; n) at the two ends of a
    1D domain, for DG and CG alike: face 0 of a cell without a left neighbour
    is the left end (n = -1), face 1 without a right neighbour the right end."""
    ref = sp.ref
    if ref.dim != 1:
        return boundary_terms_2d(sp, Uc, prm)
    nbr = sp.nbr if sp.nbr is not None else face_neighbours(sp.cell, sp.mesh.cell_vertices)[0]
    out = np.zeros_like(Uc)
    for f in range(2):
        sel = nbr[:, f] < 0
        if not sel.any():
            continue
        pts, _ = ref.face_points(f)
        phif = ref.deriv(pts, (0,))[0]                              # [nloc]
        Ub = np.einsum("vej,j->ve", Uc[:, sel], phif)[..., None]     # [nv, nb, 1]
        n = np.full(Ub.shape[1:] + (1,), -1.0 if f == 0 else 1.0)
        xf = map_points(sp.cell, sp.X[sel], pts)
        Fs = numerical_flux(prm, Ub, boundary_state(prm, Ub, n, f), n, xf)   # [nv, nb, 1]
        out[:, sel] += Fs[..., 0][..., None] * phif
    return out


def boundary_terms_2d(sp, Uc, prm: Params):
    """Weak boundary terms int_f phi_j f*(u_h, u_ext; n) over the boundary faces
    of a 2D mesh, each face with its own kind and state (prm.bc_face_kind,
    prm.bc_face_state in the order of boundary_faces)."""
    ref = sp.ref
    cells, faces = boundary_faces(sp)
    if prm.bc_face_kind is None:
        raise ValueError("boundary faces without boundary data")
    kinds = np.asarray(prm.bc_face_kind)
    states = np.asarray(prm.bc_face_state, np.float64) if prm.bc_face_state is not None else \
        np.zeros((len(cells), Uc.shape[0]))
    if len(kinds) != len(cells):
        raise ValueError("one boundary kind per boundary face")
    out = np.zeros_like(Uc)
    for f in range(ref.n_faces):
        on_f = np.nonzero(faces == f)[0]
        if len(on_f) == 0:
            continue
        pts, wf = ref.face_points(f)
        phif = ref.deriv(pts, (0,) * ref.dim)                       # [ng, nloc]
        n_all, Jf_all = face_geometry(sp, f)
        for b in on_f:
            e = cells[b]
            Ub = np.einsum("vj,gj->vg", Uc[:, e], phif)              # [nv, ng]
            nb = np.broadcast_to(n_all[e], (len(wf), n_all.shape[1]))
            Ug = ghost_state(prm, int(kinds[b]), states[b], Ub, nb)
            xf = map_points(sp.cell, sp.X[e:e + 1], pts)[0]
            Fs = numerical_flux(prm, Ub, Ug, nb, xf)                 # [nv, ng]
            out[:, e] += np.einsum("g,gj,vg->vj", wf * Jf_all[e], phif, Fs)
    return out


# ---------------------------------------------------------------------------
# mass matrix and time stepping
# ---------------------------------------------------------------------------
def _cell_mass(sp):
    ref = sp.ref
    pts = ref.vol_pts
    J, _ = map_jacobian(sp.cell, sp.X, pts)
    W = ref.vol_w[None, :] * np.abs(np.linalg.det(J))
    phi = ref.deriv(pts, (0,) * ref.dim)
    return np.einsum("eq,qi,qj->eij", W, phi, phi)


def apply_mass_inverse(sp, R):
    """Solve M L = R (DG: exact element mass per cell; CG: consistent global mass)."""
    Me = _cell_mass(sp)
    nv = sp.n_var
    if sp.kind == 1:
        r = R.reshape(nv, sp.E, -1)
        out = np.stack([np.linalg.solve(Me, r[v][..., None])[..., 0] for v in range(nv)])
        return out.ravel()
    cd = sp.cell_dof
    rows = np.repeat(cd, cd.shape[1], axis=1).ravel()
    cols = np.tile(cd, (1, cd.shape[1])).ravel()
    M = sps.csr_matrix((Me.ravel(), (rows, cols)), shape=(sp.n_dof, sp.n_dof))
    r = R.reshape(nv, sp.n_dof)
    solve = spla.factorized(M.tocsc())
    return np.concatenate([solve(r[v]) for v in range(nv)])


def time_derivative(sp, U, prm: Params):
    return -apply_mass_inverse(sp, residual(sp, U, prm))


def rk3_step(sp, U, dt: float, prm: Params):
    """Three-stage SSP Runge-Kutta step (Shu-Osher form)."""
    U1 = U + dt * time_derivative(sp, U, prm)
    U2 = 0.75 * U + 0.25 * (U1 + dt * time_derivative(sp, U1, prm))
    return U / 3.0 + 2.0 / 3.0 * (U2 + dt * time_derivative(sp, U2, prm))


def nodal_interpolate(sp, funcs):
    """State vector from the initial data sampled at the nodes (DG) or DOF
    positions (CG; first occurrence in (cell, local) order).  funcs: one
    callable per variable taking physical coordinates [..., d]."""
    xn = sp.node_coords()                       # [E, nloc, d]
    vals = np.stack([f(xn) for f in funcs])     # [nv, E, nloc]
    if sp.kind == 1:
        return vals.reshape(len(funcs), -1).ravel()
    flat = sp.cell_dof.ravel()
    _, first = np.unique(flat, return_index=True)
    out = np.empty((len(funcs), sp.n_dof))
    out[:, flat[first]] = vals.reshape(len(funcs), -1)[:, first]
    return out.ravel()
