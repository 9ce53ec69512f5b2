// Host side of libcvw: argument validation, mesh connectivity (vertex patches,
// face neighbours, canonical CG numbering), reference tables and dispatch of
// the gfx950 kernels.  Everything here runs once per mesh (cvw_mesh_build) or
// once per call; no host work depends on the state.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "cvw_internal.h"
#include "cvw_cells3d.h"
#include "cvw_limit.h"

namespace cvw {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int n_var(const cvw_mesh* m, int flux) { return flux == CVW_EULER ? m->dim + 2 : 1; }

MethodScalars make_scalars(const cvw_params* p) {
  MethodScalars s{};
  s.eps_v = static_cast<float>(p->eps_vertex);
  s.eps_c = static_cast<float>(p->eps_cell);
  s.r = static_cast<float>(p->r);
  s.q_sensor = static_cast<float>(p->q_sensor);
  s.q_beta = static_cast<float>(p->q_beta);
  s.lin_w = static_cast<float>(p->lin_w_vertex);
  s.c_gamma = static_cast<float>(p->c_gamma);
  s.lam_g = static_cast<float>(p->lambda_global);
  for (int i = 0; i < 4; ++i) s.fp[i] = static_cast<float>(p->flux_param[i]);
  s.sc_on = p->sc_on;
  s.fast_exp = (p->r == 2 && p->q_sensor == 1.0 && p->q_beta == 1.0) ? 1 : 0;
  s.sensor_kind = p->sensor;
  s.fixed_gamma = static_cast<float>(p->fixed_gamma);
  s.eps_vd = p->eps_vertex;
  s.eps_cd = p->eps_cell;
  s.lin_wd = p->lin_w_vertex;
  s.c_gammad = p->c_gamma;
  s.lam_gd = p->lambda_global;
  s.fixed_gammad = p->fixed_gamma;
  for (int i = 0; i < 4; ++i) s.fpd[i] = p->flux_param[i];
  s.bck = p->bc_face_kind;
  s.bcs = p->bc_face_state;
  return s;
}

// The 1D kernels of any degree serve degrees above 3, the Euler equations and
// lines with ends; scalar laws of degree <= 3 on closed lines keep the
// one-thread-per-cell kernels.
bool seg_hp(const cvw_mesh* m, const cvw_params* prm) {
  return m->cell == CVW_SEG && (m->degree > MAXP || prm->flux == CVW_EULER || m->open_ends > 0);
}

SegHPArgs seghp_args(const cvw_mesh* m, const cvw_params* prm) {
  SegHPArgs A{};
  A.tab = m->d_hp;
  A.cell_dof = m->d_cell_dof;
  A.cell_vtx = m->d_cell_vtx;
  A.nbr = m->d_nbr;
  A.hcell = m->d_hcell;
  A.vptr = m->d_vtx_ptr;
  A.vent = m->d_vtx_ent;
  A.dptr = m->d_dof_ptr;
  A.dent = m->d_dof_ent;
  A.E = m->E;
  A.Nv = m->Nv;
  A.ndof = m->ndof;
  A.p = m->degree;
  A.nv = n_var(m, prm->flux);
  A.flux = prm->flux;
  A.cg = m->space == CVW_CG ? 1 : 0;
  for (int e = 0; e < 2; ++e) {
    A.bc[e] = prm->bc[e];
    for (int v = 0; v < 4; ++v) A.bcs[e][v] = prm->bc_state[e][v];
  }
  A.ms = make_scalars(prm);
  return A;
}

// ---------------------------------------------------------------------------
// 1D rules and Lagrange polynomials (double precision, computed here from
// their definitions: Newton iteration on the Legendre polynomial and its
// derivative)
// ---------------------------------------------------------------------------
static void legendre(int n, double x, double& p, double& dp) {
  double p0 = 1.0, p1 = x;
  if (n == 0) { p = 1.0; dp = 0.0; return; }
  for (int k = 2; k <= n; ++k) {
    const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  p = p1;
  dp = n * (x * p1 - p0) / (x * x - 1.0);
}

void gauss_rule(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = -std::cos(M_PI * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre(n, z, p, dp);
      const double dz = p / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p, dp;
    legendre(n, z, p, dp);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

void lobatto_nodes(int n, std::vector<double>& x) {
  // endpoints and the roots of P'_{n-1}
  x.assign(n, 0.0);
  x[0] = -1.0;
  x[n - 1] = 1.0;
  const int m = n - 1;
  for (int i = 1; i < n - 1; ++i) {
    double z = -std::cos(M_PI * i / m);
    for (int it = 0; it < 100; ++it) {
      // f = P'_m(z), f' = P''_m(z) from the Legendre ODE: (1-z^2) P'' = 2 z P' - m(m+1) P
      double p, dp;
      legendre(m, z, p, dp);
      const double d2p = (2.0 * z * dp - m * (m + 1.0) * p) / (1.0 - z * z);
      const double dz = dp / d2p;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
  }
}

// value of the m-th derivative of the Lagrange polynomial l_i (nodes xs) at t
static double lagrange_deriv(const std::vector<double>& xs, int i, int m, double t) {
  const int n = static_cast<int>(xs.size());
  // monomial coefficients of l_i
  std::vector<double> c(1, 1.0);
  double den = 1.0;
  for (int j = 0; j < n; ++j) {
    if (j == i) continue;
    std::vector<double> nc(c.size() + 1, 0.0);
    for (size_t k = 0; k < c.size(); ++k) {
      nc[k + 1] += c[k];
      nc[k] -= xs[j] * c[k];
    }
    c.swap(nc);
    den *= xs[i] - xs[j];
  }
  for (auto& v : c) v /= den;
  for (int d = 0; d < m; ++d) {
    if (c.size() <= 1) return 0.0;
    std::vector<double> nc(c.size() - 1);
    for (size_t k = 1; k < c.size(); ++k) nc[k - 1] = c[k] * static_cast<double>(k);
    c.swap(nc);
  }
  double v = 0.0;
  for (size_t k = c.size(); k-- > 0;) v = v * t + c[k];
  return v;
}

static void fill_tensor_tables(TensorTables& T, int p, bool lobatto) {
  std::memset(&T, 0, sizeof(T));
  std::vector<double> x, w, xn;
  gauss_rule(p + 1, x, w);
  if (lobatto) lobatto_nodes(p + 1, xn); else xn = x;
  for (int a = 0; a <= p; ++a) {
    T.xi[a] = static_cast<float>(xn[a]);
    T.w[a] = static_cast<float>(w[a]);
    T.wd[a] = w[a];
  }
  // D[m][a][i] = l_i^{(m)} at the volume quadrature point a (= node a for Gauss nodes)
  for (int m = 0; m <= p; ++m)
    for (int a = 0; a <= p; ++a)
      for (int i = 0; i <= p; ++i) {
        T.Dd[m][a][i] = lagrange_deriv(xn, i, m, x[a]);
        T.D[m][a][i] = static_cast<float>(T.Dd[m][a][i]);
      }
  for (int i = 0; i <= p; ++i) {
    T.B[0][i] = static_cast<float>(lagrange_deriv(xn, i, 0, -1.0));
    T.B[1][i] = static_cast<float>(lagrange_deriv(xn, i, 0, 1.0));
    for (int m = 0; m <= p; ++m) {
      T.Ld[m][i] = lagrange_deriv(xn, i, m, -1.0);
      T.L[m][i] = static_cast<float>(T.Ld[m][i]);
      T.Cd[m][i] = lagrange_deriv(xn, i, m, 0.0);
    }
  }
}

static void fill_lane_tables1(LaneRec* R, const TensorTables& T) {
  std::memset(R, 0, 16 * sizeof(LaneRec));
  LaneRec1 r[4];
  std::memset(r, 0, sizeof(r));
  for (int l = 0; l < 4; ++l) {
    const int a = l & 1, b = l >> 1;
    LaneRec1& L = r[l];
    for (int i = 0; i < 2; ++i) {
      L.CX1[i] = static_cast<float>(T.Dd[1][a][i]);
      L.CY1[i] = static_cast<float>(T.Dd[1][b][i]);
      L.TX[i] = static_cast<float>(T.Dd[1][i][a]);
      L.TY[i] = static_cast<float>(T.Dd[1][i][b]);
      L.OX[i] = T.B[a][i];
      L.OY[i] = T.B[b][i];
      L.FX[i] = T.B[1 - a][i];
      L.FY[i] = T.B[1 - b][i];
      L.DX[i] = T.Dd[1][a][i];
      L.DY[i] = T.Dd[1][b][i];
    }
    L.lift[0] = T.B[0][a];
    L.lift[1] = T.B[1][a];
    L.lift[2] = T.B[0][b];
    L.lift[3] = T.B[1][b];
    L.wa = T.w[a];
    L.wb = T.w[b];
    L.xq = T.xi[a];
    L.yq = T.xi[b];
    L.nx = a == 0 ? -1.0f : 1.0f;
    L.ny = b == 0 ? -1.0f : 1.0f;
    L.slotx = a == 0 ? 3 : 1;
    L.sloty = b == 0 ? 0 : 2;
  }
  std::memcpy(static_cast<void*>(R), r, sizeof(r));
}

static void fill_lane_tables(LaneRec* R, const TensorTables& T, int p) {
  if (p == 1) {
    fill_lane_tables1(R, T);
    return;
  }
  std::memset(R, 0, 16 * sizeof(LaneRec));
  for (int q = 0; q < 16; ++q) {
    const int a = q & 3, b = q >> 2;
    if (a > p || b > p) continue;
    LaneRec& L = R[q];
    for (int s = 0; s < 4; ++s) {
      const int src = (b - s) & 3;         // row brought by a rotation of 4 s lanes
      L.CX1[s] = static_cast<float>(T.Dd[1][a][s]);
      L.CY1[s] = static_cast<float>(T.Dd[1][b][src]);
      L.TX[s] = static_cast<float>(T.Dd[1][s][a]);
      L.TY[s] = static_cast<float>(T.Dd[1][src][b]);
      L.BY0[s] = T.B[0][src];
      L.BY1[s] = T.B[1][src];
      for (int m = 1; m <= 3; ++m) {
        L.DX[m - 1][s] = T.Dd[m][a][s];
        L.DY[m - 1][s] = T.Dd[m][b][src];
      }
    }
    L.misc[0] = T.B[0][a];
    L.misc[1] = T.B[1][a];
    L.misc[2] = T.B[0][b];
    L.misc[3] = T.B[1][b];
    L.misc[4] = T.w[a];
    L.misc[5] = T.w[b];
    L.misc[6] = T.xi[a];
    L.misc[7] = T.xi[b];
    for (int i = 0; i < 4; ++i) {
      L.BX0[i] = T.B[0][i];
      L.BX1[i] = T.B[1][i];
    }
    if (p == 3) {
      const bool xf = (a == 0 || a == 3);
      const bool inner = !xf && (b == 1 || b == 2);
      const bool south = inner ? (b == 1) : (b == 0);
      const int col = inner ? (a == 1 ? 0 : 3) : a;
      L.slot = xf ? (a == 0 ? 3 : 1) : (south ? 0 : 2);
      const bool far_plus = (L.slot == 3 || L.slot == 0);      // W / S neighbour: its +1 side
      for (int i = 0; i < 4; ++i) {
        L.OX[i] = (a == 0) ? T.B[0][i] : T.B[1][i];
        const int src = (b - i) & 3;
        L.OY[i] = (b <= 1) ? T.B[0][src] : T.B[1][src];
        L.FB[i] = far_plus ? T.B[1][i] : T.B[0][i];
      }
      L.noff = xf ? 4 * b : col;
      L.nstep = xf ? 1 : 4;
      L.nx = xf ? (a == 0 ? -1.0f : 1.0f) : 0.0f;
      L.ny = xf ? 0.0f : (south ? -1.0f : 1.0f);
      L.fwx = xf ? 0.5f * T.w[b] : 0.0f;
      L.fwy = xf ? 0.0f : 0.5f * T.w[col];
      const bool ccol = (a == 0 || a == 3);
      const int ia = (a == 0) ? 1 : 2;
      L.srcS = ccol ? ia + 4 : a;
      L.srcN = ccol ? ia + 8 : a + 12;
    }
  }
}

static void fill_cg_tables(CGTables& T, int p) {
  std::memset(&T, 0, sizeof(T));
  std::vector<double> xn, xv, wv, xs, ws;
  lobatto_nodes(p + 1, xn);
  gauss_rule(p + 1, xv, wv);
  gauss_rule(p + 2, xs, ws);
  for (int a = 0; a <= p; ++a) {
    T.xn[a] = static_cast<float>(xn[a]);
    T.xv[a] = static_cast<float>(xv[a]);
    T.wv[a] = static_cast<float>(wv[a]);
  }
  for (int a = 0; a <= p + 1; ++a) {
    T.xs[a] = static_cast<float>(xs[a]);
    T.ws[a] = static_cast<float>(ws[a]);
  }
  for (int m = 0; m < 3; ++m)
    for (int i = 0; i <= p; ++i) {
      for (int q = 0; q <= p; ++q) {
        T.Dvd[m][q][i] = lagrange_deriv(xn, i, m, xv[q]);
        T.Dv[m][q][i] = static_cast<float>(T.Dvd[m][q][i]);
      }
      for (int q = 0; q <= p + 1; ++q) {
        T.Dsd[m][q][i] = lagrange_deriv(xn, i, m, xs[q]);
        T.Ds[m][q][i] = static_cast<float>(T.Dsd[m][q][i]);
      }
      T.Lmd[m][i] = lagrange_deriv(xn, i, m, -1.0);
      T.Lpd[m][i] = lagrange_deriv(xn, i, m, 1.0);
      T.Lm[m][i] = static_cast<float>(T.Lmd[m][i]);
      T.Lp[m][i] = static_cast<float>(T.Lpd[m][i]);
    }
  for (int a = 0; a <= p; ++a)
    for (int i = 0; i <= p; ++i) T.Dn[a][i] = static_cast<float>(lagrange_deriv(xn, i, 1, xn[a]));
}

// ---------------------------------------------------------------------------
// Triangle tables
// ---------------------------------------------------------------------------
// Gauss rule for the weight (1 - x) on [-1, 1]: nodes are the roots of the
// Jacobi polynomial P_n^{(1,0)} (three-term recurrence, bracketed by a sign
// scan and bisected to full precision); weights from the moment equations.
static double jacobi10(int n, double x) {
  const double a = 1.0, b = 0.0;
  double p0 = 1.0, p1 = (a + 1.0) + (a + b + 2.0) * (x - 1.0) / 2.0;
  if (n == 0) return p0;
  for (int k = 2; k <= n; ++k) {
    const double c = 2.0 * k + a + b;
    const double p2 = ((c - 1.0) * (c * (c - 2.0) * x + a * a - b * b) * p1 - 2.0 * (k + a - 1.0) * (k + b - 1.0) * c * p0) /
                      (2.0 * k * (k + a + b) * (c - 2.0));
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

static bool solve_dense(std::vector<double> M, std::vector<double>& rhs, int n) {
  // Gauss-Jordan elimination with partial pivoting on M [n][n]; rhs [n][k] row-major is overwritten
  // by M^{-1} rhs
  const int k = static_cast<int>(rhs.size()) / n;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(M[r * n + c]) > std::fabs(M[piv * n + c])) piv = r;
    if (!(std::fabs(M[piv * n + c]) > 0)) return false;
    if (piv != c) {
      for (int j = 0; j < n; ++j) std::swap(M[c * n + j], M[piv * n + j]);
      for (int j = 0; j < k; ++j) std::swap(rhs[c * k + j], rhs[piv * k + j]);
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = M[r * n + c] / M[c * n + c];
      if (f == 0.0) continue;
      for (int j = c; j < n; ++j) M[r * n + j] -= f * M[c * n + j];
      for (int j = 0; j < k; ++j) rhs[r * k + j] -= f * rhs[c * k + j];
    }
  }
  for (int r = 0; r < n; ++r)
    for (int j = 0; j < k; ++j) rhs[r * k + j] /= M[r * n + r];
  return true;
}

static void gauss_jacobi10(int n, std::vector<double>& x, std::vector<double>& w) {
  x.clear();
  const int scan = 4000;
  double xa = -1.0, fa = jacobi10(n, xa);
  for (int i = 1; i <= scan && static_cast<int>(x.size()) < n; ++i) {
    const double xb = -1.0 + 2.0 * i / scan, fb = jacobi10(n, xb);
    if (fa == 0.0) { x.push_back(xa); }
    else if (fa * fb < 0.0) {
      double lo = xa, hi = xb, flo = fa;
      for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        const double fm = jacobi10(n, mid);
        if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else { hi = mid; }
      }
      x.push_back(0.5 * (lo + hi));
    }
    xa = xb;
    fa = fb;
  }
  // moments int_{-1}^{1} x^k (1 - x) dx
  std::vector<double> V(n * n), m(n);
  for (int k = 0; k < n; ++k) {
    m[k] = ((k % 2 == 0) ? 2.0 / (k + 1) : 0.0) - ((k % 2 == 1) ? 2.0 / (k + 2) : 0.0);
    for (int i = 0; i < n; ++i) V[k * n + i] = std::pow(x[i], k);
  }
  solve_dense(V, m, n);
  w = m;
}

// Lagrange basis on the equispaced nodes of the reference triangle: monomial
// coefficients C[i][j] (monomial i = xi^a eta^b in the order (a, b) of total
// degree then decreasing a; column j = basis function j)
struct TriBasis {
  int p = 0, n = 0;
  std::vector<std::pair<int, int>> mono;
  std::vector<double> C;        // [n][n]
  double deriv(int j, int mx, int my, double xi, double eta) const {
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
      const int a = mono[i].first, b = mono[i].second;
      if (a < mx || b < my) continue;
      double ca = 1.0, cb = 1.0;
      for (int t = 0; t < mx; ++t) ca *= (a - t);
      for (int t = 0; t < my; ++t) cb *= (b - t);
      s += C[i * n + j] * ca * cb * std::pow(xi, a - mx) * std::pow(eta, b - my);
    }
    return s;
  }
};

static TriBasis tri_basis(int p) {
  TriBasis B;
  B.p = p;
  B.n = (p + 1) * (p + 2) / 2;
  for (int t = 0; t <= p; ++t)
    for (int a = t; a >= 0; --a) B.mono.push_back({a, t - a});
  std::vector<std::pair<double, double>> nodes;
  for (int j = 0; j <= p; ++j)
    for (int i = 0; i <= p - j; ++i) nodes.push_back({double(i) / p, double(j) / p});
  const int n = B.n;
  // V[r][i] = monomial i at node r;  C = V^{-1}
  std::vector<double> V(n * n), I(n * n, 0.0);
  for (int r = 0; r < n; ++r) {
    for (int i = 0; i < n; ++i)
      V[r * n + i] = std::pow(nodes[r].first, B.mono[i].first) * std::pow(nodes[r].second, B.mono[i].second);
    I[r * n + r] = 1.0;
  }
  solve_dense(V, I, n);
  B.C = I;
  return B;
}

static void fill_tri_tables(TriTables& T, int p) {
  std::memset(&T, 0, sizeof(T));
  const TriBasis B = tri_basis(p);
  const int n = B.n, nq1 = p + 1;
  std::vector<double> xa, wa, xb, wb;
  gauss_rule(nq1, xa, wa);
  gauss_jacobi10(nq1, xb, wb);
  std::vector<double> qx, qy, qw;
  for (int ib = 0; ib < nq1; ++ib)
    for (int ia = 0; ia < nq1; ++ia) {
      const double a = 0.5 * (xa[ia] + 1.0), b = 0.5 * (xb[ib] + 1.0);
      qx.push_back(a * (1.0 - b));
      qy.push_back(b);
      qw.push_back(0.5 * wa[ia] * wb[ib] / 4.0);
    }
  const int nq = nq1 * nq1;
  for (int q = 0; q < nq; ++q) {
    T.xq[q] = static_cast<float>(qx[q]);
    T.yq[q] = static_cast<float>(qy[q]);
    T.wq[q] = static_cast<float>(qw[q]);
    T.xqd[q] = qx[q];
    T.yqd[q] = qy[q];
    T.wqd[q] = qw[q];
    for (int j = 0; j < n; ++j) {
      T.Bd[q][j] = B.deriv(j, 0, 0, qx[q], qy[q]);
      T.B[q][j] = static_cast<float>(B.deriv(j, 0, 0, qx[q], qy[q]));
      T.Gx[q][j] = static_cast<float>(B.deriv(j, 1, 0, qx[q], qy[q]));
      T.Gy[q][j] = static_cast<float>(B.deriv(j, 0, 1, qx[q], qy[q]));
    }
  }
  const double vx[3] = {0.0, 1.0, 0.0}, vy[3] = {0.0, 0.0, 1.0};
  std::vector<double> gx, gw;
  gauss_rule(p + 1, gx, gw);
  for (int g = 0; g <= p; ++g) T.wf[g] = static_cast<float>(gw[g]);
  for (int f = 0; f < 3; ++f)
    for (int g = 0; g <= p; ++g) {
      const int f1 = (f + 1) % 3;
      const double xi = 0.5 * (1.0 - gx[g]) * vx[f] + 0.5 * (1.0 + gx[g]) * vx[f1];
      const double eta = 0.5 * (1.0 - gx[g]) * vy[f] + 0.5 * (1.0 + gx[g]) * vy[f1];
      T.xf[f][g] = static_cast<float>(xi);
      T.yf[f][g] = static_cast<float>(eta);
      for (int j = 0; j < n; ++j) {
        T.Bfd[f][g][j] = B.deriv(j, 0, 0, xi, eta);
        T.Bf[f][g][j] = static_cast<float>(T.Bfd[f][g][j]);
      }
    }
  {
    double ws = 0.0;
    for (int q = 0; q < nq; ++q) ws += qw[q];
    for (int j = 0; j < n; ++j) {
      double a = 0.0;
      for (int q = 0; q < nq; ++q) a += qw[q] * T.Bd[q][j];
      T.mwd[j] = a / ws;
    }
  }
  for (int l = 0; l < 3; ++l) {
    int t = 0;
    for (int ord = 1; ord <= p; ++ord)
      for (int b = 0; b <= ord; ++b, ++t)
        for (int j = 0; j < n; ++j) T.TV[l][t][j] = B.deriv(j, ord - b, b, vx[l], vy[l]);
  }
  // reference mass (the Stroud rule integrates degree 2p exactly) and its inverse
  std::vector<double> M(n * n, 0.0), Mi(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double mv = 0.0;
    for (int q = 0; q < nq; ++q) {
      const double pi = B.deriv(i, 0, 0, qx[q], qy[q]);
      mv += qw[q] * pi;
      for (int j = 0; j < n; ++j) M[i * n + j] += qw[q] * pi * B.deriv(j, 0, 0, qx[q], qy[q]);
    }
    T.mvec[i] = static_cast<float>(mv);
    Mi[i * n + i] = 1.0;
  }
  solve_dense(M, Mi, n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) T.Minv[i][j] = static_cast<float>(Mi[i * n + j]);
}

static void fill_seg_tables(SegTables& T, int p, bool lobatto) {
  std::memset(&T, 0, sizeof(T));
  std::vector<double> xq, wq, xn;
  gauss_rule(p + 1, xq, wq);
  if (lobatto) lobatto_nodes(p + 1, xn); else xn = xq;
  for (int a = 0; a <= p; ++a) {
    T.xn[a] = xn[a];
    T.xq[a] = xq[a];
    T.wq[a] = wq[a];
  }
  for (int m = 0; m <= p; ++m)
    for (int i = 0; i <= p; ++i) {
      for (int q = 0; q <= p; ++q) T.D[m][q][i] = lagrange_deriv(xn, i, m, xq[q]);
      T.Lv[0][m][i] = lagrange_deriv(xn, i, m, -1.0);
      T.Lv[1][m][i] = lagrange_deriv(xn, i, m, 1.0);
    }
  for (int a = 0; a <= p; ++a)
    for (int i = 0; i <= p; ++i) T.Dn[a][i] = lagrange_deriv(xn, i, 1, xn[a]);
}

// ---------------------------------------------------------------------------
// Reference operators of the 1D Lagrange basis at any degree (hp_off layout),
// in extended precision: the nodes by Newton's method on the Legendre
// polynomials, each l_j as a Legendre series (the inverse of the Legendre-
// Vandermonde matrix of the nodes), and the derivatives of every order of the
// P_n from the three-term recurrence differentiated m times:
//   n P_n^(m)(x) = (2n - 1) (x P_{n-1}^(m)(x) + m P_{n-1}^(m-1)(x)) - (n - 1) P_{n-2}^(m)(x).
// ---------------------------------------------------------------------------
using ld = long double;

// P_n^(m)(x) for n = 0..N, m = 0..M into T[m * (N + 1) + n]
static void legendre_all(int N, int M, ld x, std::vector<ld>& T) {
  T.assign(static_cast<size_t>(M + 1) * (N + 1), 0.0L);
  for (int m = 0; m <= M; ++m)
    for (int n = 0; n <= N; ++n) {
      ld v;
      if (n == 0) {
        v = m == 0 ? 1.0L : 0.0L;
      } else {
        const ld a = T[m * (N + 1) + n - 1];
        const ld b = m > 0 ? T[(m - 1) * (N + 1) + n - 1] : 0.0L;
        const ld c = n >= 2 ? T[m * (N + 1) + n - 2] : 0.0L;
        v = ((2 * n - 1) * (x * a + m * b) - (n - 1) * c) / n;
      }
      T[m * (N + 1) + n] = v;
    }
}

// n-point Gauss rule (nodes ascending) or n-point Gauss-Lobatto nodes
static void rule_ld(int n, bool lobatto, std::vector<ld>& x, std::vector<ld>& w) {
  x.assign(n, 0.0L);
  w.assign(n, 0.0L);
  std::vector<ld> T;
  if (!lobatto) {
    for (int i = 0; i < n; ++i) {
      ld z = -std::cos(static_cast<ld>(M_PI) * (i + 0.75L) / (n + 0.5L));
      for (int it = 0; it < 100; ++it) {
        legendre_all(n, 1, z, T);
        const ld dz = T[n] / T[(n + 1) + n];
        z -= dz;
        if (std::fabs(dz) < 1e-19L) break;
      }
      legendre_all(n, 1, z, T);
      x[i] = z;
      w[i] = 2.0L / ((1.0L - z * z) * T[(n + 1) + n] * T[(n + 1) + n]);
    }
    return;
  }
  const int m = n - 1;               // interior nodes: roots of P_m'
  x[0] = -1.0L;
  x[n - 1] = 1.0L;
  for (int i = 1; i < n - 1; ++i) {
    ld z = -std::cos(static_cast<ld>(M_PI) * i / m);
    for (int it = 0; it < 100; ++it) {
      legendre_all(m, 2, z, T);
      const ld dz = T[(m + 1) + m] / T[2 * (m + 1) + m];
      z -= dz;
      if (std::fabs(dz) < 1e-19L) break;
    }
    x[i] = z;
  }
}

// ---------------------------------------------------------------------------
// hexahedra (DG Q_p on boxes hx x hy x hz), in extended precision: the
// Lagrange basis of the Gauss nodes through the inverse of its Vandermonde
// matrix in the monomials xi^a, its derivatives at the nodes and at the
// corners, the semi-norm Gram matrix of the monomials of a cell (Sec. 3.2,
// eq. snorm with h_e^{2|k|-d}, d = 3), and the re-expansion of a vertex
// candidate (Taylor data about the vertex, eq. taylorcand) about the centre.
// ---------------------------------------------------------------------------
static bool fill_hex_tables(HexTables& T, int p, double hx, double hy, double hz) {
  T = HexTables{};
  const int n1 = p + 1;
  T.p = p; T.n1 = n1; T.nl = n1 * n1 * n1;
  std::vector<ld> x, w;
  rule_ld(n1, false, x, w);
  // V[j][a] = x_j^a; C = V^{-1}: l_j(xi) = sum_a C[a][j] xi^a
  std::vector<ld> V(n1 * n1), C(n1 * n1, 0.0L);
  for (int j = 0; j < n1; ++j)
    for (int a = 0; a < n1; ++a) V[j * n1 + a] = std::pow(x[j], static_cast<ld>(a));
  for (int i = 0; i < n1; ++i) C[i * n1 + i] = 1.0L;
  for (int c = 0; c < n1; ++c) {                 // Gauss-Jordan with partial pivoting
    int piv = c;
    for (int r = c + 1; r < n1; ++r)
      if (std::fabs(V[r * n1 + c]) > std::fabs(V[piv * n1 + c])) piv = r;
    for (int k = 0; k < n1; ++k) { std::swap(V[c * n1 + k], V[piv * n1 + k]); std::swap(C[c * n1 + k], C[piv * n1 + k]); }
    const ld d = V[c * n1 + c];
    for (int k = 0; k < n1; ++k) { V[c * n1 + k] /= d; C[c * n1 + k] /= d; }
    for (int r = 0; r < n1; ++r)
      if (r != c) {
        const ld f = V[r * n1 + c];
        for (int k = 0; k < n1; ++k) { V[r * n1 + k] -= f * V[c * n1 + k]; C[r * n1 + k] -= f * C[c * n1 + k]; }
      }
  }
  // C now holds V^{-1} with rows indexed by the monomial power: C[a][j]
  auto ffall = [](int a, int m) { ld r = 1.0L; for (int i = 0; i < m; ++i) r *= (a - i); return r; };  // a!/(a-m)!
  auto lder = [&](int j, int m, ld t) {         // l_j^{(m)}(t)
    ld v = 0.0L;
    for (int a = m; a < n1; ++a) v += C[a * n1 + j] * ffall(a, m) * std::pow(t, static_cast<ld>(a - m));
    return v;
  };
  for (int q = 0; q < n1; ++q) {
    T.w1[q] = static_cast<float>(w[q]);
    for (int j = 0; j < n1; ++j) {
      T.D1[q][j] = static_cast<float>(lder(j, 1, x[q]));
      T.D2[q][j] = static_cast<float>(lder(j, 2, x[q]));
      T.T1[q][j] = static_cast<double>(C[q * n1 + j]);
    }
  }
  for (int j = 0; j < n1; ++j) { T.Lend[0][j] = static_cast<float>(lder(j, 0, -1.0L)); T.Lend[1][j] = static_cast<float>(lder(j, 0, 1.0L)); }
  const ld h[3] = {hx, hy, hz};
  const ld he = std::sqrt(h[0] * h[0] + h[1] * h[1] + h[2] * h[2]);
  const ld W0 = h[0] * h[1] * h[2] / 8.0L;
  for (int d = 0; d < 3; ++d) T.sc[d] = static_cast<float>(2.0L / h[d]);
  T.W0 = static_cast<float>(W0);
  T.Jf[0] = static_cast<float>(h[1] * h[2] / 4.0L);
  T.Jf[1] = static_cast<float>(h[0] * h[2] / 4.0L);
  T.Jf[2] = static_cast<float>(h[0] * h[1] / 4.0L);
  T.he = static_cast<float>(he);
  T.nuf = static_cast<float>(he / (2.0L * p));
  // multi-indices 1 <= |k| <= p
  std::vector<std::array<int, 3>> ks;
  for (int n = 1; n <= p; ++n)
    for (int a = n; a >= 0; --a)
      for (int b = n - a; b >= 0; --b) ks.push_back({a, b, n - a - b});
  T.nk = static_cast<int>(ks.size());
  auto mono = [&](int a, int b, int c) { return a + n1 * (b + n1 * c); };
  for (int A = 0; A < T.nl; ++A) T.kmono[A] = -1;
  for (int k = 0; k < T.nk; ++k) {
    const auto& kk = ks[k];
    const int ord = kk[0] + kk[1] + kk[2];
    ld sc2 = 1.0L;
    for (int d = 0; d < 3; ++d) {
      T.kk[k][d] = static_cast<int8_t>(kk[d]);
      sc2 *= std::pow(2.0L / h[d], static_cast<ld>(2 * kk[d]));
    }
    T.wa[k] = static_cast<float>(std::pow(he, static_cast<ld>(2 * ord)) * sc2);
    T.hb[k] = static_cast<double>(std::pow(he, static_cast<ld>(2 * ord)));
    T.kmono[mono(kk[0], kk[1], kk[2])] = static_cast<int8_t>(k);
  }
  // G[A][B] = sum_k h_e^{2|k|-3} prod_d (2/h_d)^{2 k_d} W0 prod_d int_{-1}^{1} d^{k_d} xi^{A_d} d^{k_d} xi^{B_d}
  auto I1 = [&](int a, int b, int m) -> ld {
    if (a < m || b < m) return 0.0L;
    const int n = a + b - 2 * m;
    return (n % 2) ? 0.0L : ffall(a, m) * ffall(b, m) * 2.0L / (n + 1);
  };
  for (int A = 0; A < T.nl; ++A)
    for (int B = 0; B < T.nl; ++B) {
      const int Ad[3] = {A % n1, (A / n1) % n1, A / (n1 * n1)}, Bd[3] = {B % n1, (B / n1) % n1, B / (n1 * n1)};
      ld g = 0.0L;
      for (int k = 0; k < T.nk; ++k) {
        const auto& kk = ks[k];
        const int ord = kk[0] + kk[1] + kk[2];
        ld t = std::pow(he, static_cast<ld>(2 * ord - 3)) * W0;
        for (int d = 0; d < 3; ++d) t *= std::pow(2.0L / h[d], static_cast<ld>(2 * kk[d])) * I1(Ad[d], Bd[d], kk[d]);
        g += t;
      }
      T.G[A][B] = static_cast<double>(g);
    }
  // corners: sigma = (+-1, +-1, +-1) in the local vertex order of the mesh
  static const int SG[8][3] = {{-1, -1, -1}, {1, -1, -1}, {1, 1, -1}, {-1, 1, -1},
                               {-1, -1, 1}, {1, -1, 1}, {1, 1, 1}, {-1, 1, 1}};
  for (int m = 0; m < n1; ++m)
    for (int j = 0; j < n1; ++j) {
      T.E1[m][0][j] = static_cast<double>(lder(j, m, -1.0L));
      T.E1[m][1][j] = static_cast<double>(lder(j, m, 1.0L));
    }
  for (int k = 0; k < T.nk; ++k) {
    ld v = 1.0L;
    for (int d = 0; d < 3; ++d) v *= std::pow(2.0L / h[d], static_cast<ld>(ks[k][d]));
    T.hk[k] = static_cast<double>(v);
  }
  for (int l = 0; l < 8; ++l)
    for (int k = 0; k < T.nk; ++k) {
      const auto& kk = ks[k];
      // (x - x_l)^k / k! = prod_d (h_d/2)^{k_d} sum_{a_d <= k_d} xi^{a_d} (-sigma_d)^{k_d - a_d} / (a_d! (k_d - a_d)!)
      for (int a = 0; a < T.nk; ++a) {
        const auto& aa = ks[a];
        ld v = 1.0L;
        for (int d = 0; d < 3 && v != 0.0L; ++d) {
          if (aa[d] > kk[d]) { v = 0.0L; break; }
          const int r = kk[d] - aa[d];
          v *= std::pow(h[d] / 2.0L, static_cast<ld>(kk[d])) * std::pow(static_cast<ld>(-SG[l][d]), static_cast<ld>(r)) /
               (std::tgamma(static_cast<ld>(aa[d] + 1)) * std::tgamma(static_cast<ld>(r + 1)));
        }
        T.R[l][a][k] = static_cast<double>(v);
      }
    }
  // the sensor pass visits only the pairs of monomials with exponents of
  // equal parity in every direction: every other entry of G is an exact zero
  bool fits = true;
  for (int A = 0; A < T.nl; ++A)
    for (int B = 0; B < T.nl; ++B) {
      const bool pair = (A % n1 + B % n1) % 2 == 0 && ((A / n1) % n1 + (B / n1) % n1) % 2 == 0 &&
                        (A / (n1 * n1) + B / (n1 * n1)) % 2 == 0;
      fits = fits && (pair || T.G[A][B] == 0.0);
    }
  return fits;
}

// ---------------------------------------------------------------------------
// tetrahedra: the equispaced Lagrange basis (inverse Vandermonde in the
// monomials), the conical-product volume rule (Gauss-Legendre x Gauss-Jacobi
// (1-b) x Gauss-Jacobi (1-c)^2), Radon's symmetric 7-point face rule, the
// reference mass matrix, and the derivatives of the basis at the vertices
// ---------------------------------------------------------------------------
// Gauss rule for the weight (1 - x)^al on [-1, 1] (integer al >= 0): roots of
// P_n^{(al,0)} (recurrence, sign scan and bisection), weights from the moments
static double jacobi_a0(int n, int al, double x) {
  const double a = al, b = 0.0;
  double p0 = 1.0, p1 = (a + 1.0) + (a + b + 2.0) * (x - 1.0) / 2.0;
  if (n == 0) return p0;
  for (int k = 2; k <= n; ++k) {
    const double c = 2.0 * k + a + b;
    const double p2 = ((c - 1.0) * (c * (c - 2.0) * x + a * a - b * b) * p1 - 2.0 * (k + a - 1.0) * (k + b - 1.0) * c * p0) /
                      (2.0 * k * (k + a + b) * (c - 2.0));
    p0 = p1;
    p1 = p2;
  }
  return p1;
}
static void gauss_jacobi_a0(int n, int al, std::vector<double>& x, std::vector<double>& w) {
  x.clear();
  const int scan = 4000;
  double xa = -1.0, fa = jacobi_a0(n, al, xa);
  for (int i = 1; i <= scan && static_cast<int>(x.size()) < n; ++i) {
    const double xb = -1.0 + 2.0 * i / scan, fb = jacobi_a0(n, al, xb);
    if (fa == 0.0) { x.push_back(xa); }
    else if (fa * fb < 0.0) {
      double lo = xa, hi = xb, flo = fa;
      for (int it = 0; it < 200 && hi - lo > 0.0; ++it) {
        const double mid = 0.5 * (lo + hi);
        if (mid == lo || mid == hi) break;
        const double fm = jacobi_a0(n, al, mid);
        if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else { hi = mid; }
      }
      x.push_back(0.5 * (lo + hi));
    }
    xa = xb;
    fa = fb;
  }
  // moments int_{-1}^{1} x^k (1 - x)^al dx = sum_i C(al, i) (-1)^i int x^{k+i}
  std::vector<double> V(n * n), m(n, 0.0);
  for (int k = 0; k < n; ++k) {
    double binom = 1.0;
    for (int i = 0; i <= al; ++i) {
      if (i > 0) binom = binom * (al - i + 1) / i;
      if ((k + i) % 2 == 0) m[k] += ((i % 2) ? -1.0 : 1.0) * binom * 2.0 / (k + i + 1);
    }
    for (int i = 0; i < n; ++i) V[k * n + i] = std::pow(x[i], k);
  }
  solve_dense(V, m, n);
  w = m;
}

static void fill_tet_tables(TetTables& T, int p) {
  std::memset(&T, 0, sizeof(T));
  T.p = p;
  // monomials x^a y^b z^c, a + b + c <= p (by total degree, then decreasing a, then decreasing b)
  std::vector<std::array<int, 3>> mono;
  for (int n = 0; n <= p; ++n)
    for (int a = n; a >= 0; --a)
      for (int b = n - a; b >= 0; --b) mono.push_back({a, b, n - a - b});
  const int n = static_cast<int>(mono.size());
  T.nloc = n;
  T.nk = n - 1;
  std::vector<std::array<double, 3>> nodes;
  for (int k = 0; k <= p; ++k)
    for (int j = 0; j <= p - k; ++j)
      for (int i = 0; i <= p - j - k; ++i) nodes.push_back({double(i) / p, double(j) / p, double(k) / p});
  std::vector<double> V(n * n), C(n * n, 0.0);
  for (int r = 0; r < n; ++r) {
    for (int i = 0; i < n; ++i)
      V[r * n + i] = std::pow(nodes[r][0], mono[i][0]) * std::pow(nodes[r][1], mono[i][1]) * std::pow(nodes[r][2], mono[i][2]);
    C[r * n + r] = 1.0;
  }
  solve_dense(V, C, n);          // C[i][j]: coefficient of monomial i in phi_j
  auto ff = [](int a, int m) { double r = 1.0; for (int t = 0; t < m; ++t) r *= (a - t); return r; };
  auto der = [&](int j, int mx, int my, int mz, double x, double y, double z) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) {
      const auto& mm = mono[i];
      if (mm[0] < mx || mm[1] < my || mm[2] < mz) continue;
      s += C[i * n + j] * ff(mm[0], mx) * ff(mm[1], my) * ff(mm[2], mz) * std::pow(x, mm[0] - mx) *
           std::pow(y, mm[1] - my) * std::pow(z, mm[2] - mz);
    }
    return s;
  };
  // volume rule
  const int n1 = p + 1;
  std::vector<double> xa, wa, xb, wb, xc, wc;
  gauss_rule(n1, xa, wa);
  gauss_jacobi_a0(n1, 1, xb, wb);
  gauss_jacobi_a0(n1, 2, xc, wc);
  int q = 0;
  for (int ic = 0; ic < n1; ++ic)
    for (int ib = 0; ib < n1; ++ib)
      for (int ia = 0; ia < n1; ++ia, ++q) {
        const double a = 0.5 * (xa[ia] + 1.0), b = 0.5 * (xb[ib] + 1.0), c = 0.5 * (xc[ic] + 1.0);
        T.xq[q][0] = a * (1.0 - b) * (1.0 - c);
        T.xq[q][1] = b * (1.0 - c);
        T.xq[q][2] = c;
        T.wq[q] = 0.5 * wa[ia] * wb[ib] / 4.0 * wc[ic] / 8.0;
      }
  T.nq = q;
  for (int qq = 0; qq < q; ++qq)
    for (int j = 0; j < n; ++j) {
      const double x = T.xq[qq][0], y = T.xq[qq][1], z = T.xq[qq][2];
      T.B[qq][j] = der(j, 0, 0, 0, x, y, z);
      T.G[0][qq][j] = der(j, 1, 0, 0, x, y, z);
      T.G[1][qq][j] = der(j, 0, 1, 0, x, y, z);
      T.G[2][qq][j] = der(j, 0, 0, 1, x, y, z);
      T.Bs[qq][j] = static_cast<float>(T.B[qq][j]);
      for (int b = 0; b < 3; ++b) T.Gs[b][qq][j] = static_cast<float>(T.G[b][qq][j]);
    }
  for (int qq = 0; qq < q; ++qq) T.wqs[qq] = static_cast<float>(T.wq[qq]);
  static const int H[6][3] = {{2, 0, 0}, {1, 1, 0}, {1, 0, 1}, {0, 2, 0}, {0, 1, 1}, {0, 0, 2}};
  for (int h = 0; h < 6; ++h)
    for (int j = 0; j < n; ++j) T.H2[h][j] = der(j, H[h][0], H[h][1], H[h][2], 0.25, 0.25, 0.25);
  for (int j = 0; j < n; ++j) {
    T.Gc[0][j] = der(j, 1, 0, 0, 0.25, 0.25, 0.25);
    T.Gc[1][j] = der(j, 0, 1, 0, 0.25, 0.25, 0.25);
    T.Gc[2][j] = der(j, 0, 0, 1, 0.25, 0.25, 0.25);
  }
  // multi-indices 1 <= |k| <= p and the derivatives at the reference vertices
  static const double RV[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  std::vector<std::array<int, 3>> ks(mono.begin() + 1, mono.end());
  for (int k = 0; k < T.nk; ++k) {
    for (int d = 0; d < 3; ++d) T.kk[k][d] = static_cast<int8_t>(ks[k][d]);
    for (int l = 0; l < 4; ++l)
      for (int j = 0; j < n; ++j) T.TV[l][k][j] = der(j, ks[k][0], ks[k][1], ks[k][2], RV[l][0], RV[l][1], RV[l][2]);
  }
  // reference mass matrix (the volume rule is exact for degree 2p) and its inverse
  std::vector<double> M(n * n, 0.0), Mi(n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j)
      for (int qq = 0; qq < q; ++qq) M[i * n + j] += T.wq[qq] * T.B[qq][i] * T.B[qq][j];
    Mi[i * n + i] = 1.0;
  }
  solve_dense(M, Mi, n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) T.Minv[i][j] = static_cast<float>(Mi[i * n + j]);
  // Radon's 7-point rule of degree 5: the centroid and two orbits (a, a, 1 - 2a), a = (6 -+ sqrt 15) / 21
  double bary[TET_NFP][3], wr[TET_NFP];
  const double r15 = std::sqrt(15.0);
  bary[0][0] = bary[0][1] = bary[0][2] = 1.0 / 3.0;
  wr[0] = 9.0 / 40.0;
  for (int o = 0; o < 2; ++o) {
    const double a = o == 0 ? (6.0 - r15) / 21.0 : (6.0 + r15) / 21.0, b = 1.0 - 2.0 * a;
    const double w = o == 0 ? (155.0 - r15) / 1200.0 : (155.0 + r15) / 1200.0;
    const double P3[3][3] = {{a, a, b}, {a, b, a}, {b, a, a}};
    for (int i = 0; i < 3; ++i) {
      for (int d = 0; d < 3; ++d) bary[1 + 3 * o + i][d] = P3[i][d];
      wr[1 + 3 * o + i] = w;
    }
  }
  for (int g = 0; g < TET_NFP; ++g) T.wf[g] = static_cast<float>(0.5 * wr[g]);
  static const int FV[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
  for (int f = 0; f < 4; ++f)
    for (int g = 0; g < TET_NFP; ++g) {
      double x[3] = {0, 0, 0};
      for (int i = 0; i < 3; ++i)
        for (int d = 0; d < 3; ++d) x[d] += bary[g][i] * RV[FV[f][i]][d];
      for (int j = 0; j < n; ++j) T.Bf[f][g][j] = static_cast<float>(der(j, 0, 0, 0, x[0], x[1], x[2]));
    }
  // permutations sigma of the face's three vertices (lexicographic order):
  // the point with barycentrics lambda becomes the point with lambda o sigma
  static const int SIG[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
  for (int sg = 0; sg < 6; ++sg)
    for (int g = 0; g < TET_NFP; ++g) {
      int found = -1;
      for (int h = 0; h < TET_NFP && found < 0; ++h) {
        bool same = true;
        for (int j = 0; j < 3; ++j) same = same && std::fabs(bary[h][j] - bary[g][SIG[sg][j]]) < 1e-12;
        if (same) found = h;
      }
      T.perm[sg][g] = static_cast<int8_t>(found);
    }
}

static std::vector<double> fill_hp_tables(int p, bool lobatto) {
  const int n1 = p + 1;
  const HPOff o = hp_off(p);
  std::vector<double> out(o.size, 0.0);
  std::vector<ld> xq, wq, xn, wn;
  rule_ld(n1, false, xq, wq);
  if (lobatto) rule_ld(n1, true, xn, wn); else xn = xq;
  // C = V^{-1}, V[i][n] = P_n(xn_i): Gauss-Jordan with partial pivoting
  std::vector<ld> V(n1 * n1), C(n1 * n1, 0.0L), T;
  for (int i = 0; i < n1; ++i) {
    legendre_all(p, 0, xn[i], T);
    for (int n = 0; n < n1; ++n) V[i * n1 + n] = T[n];
    C[i * n1 + i] = 1.0L;
  }
  for (int c = 0; c < n1; ++c) {
    int piv = c;
    for (int r = c + 1; r < n1; ++r)
      if (std::fabs(V[r * n1 + c]) > std::fabs(V[piv * n1 + c])) piv = r;
    for (int k = 0; k < n1; ++k) {
      std::swap(V[c * n1 + k], V[piv * n1 + k]);
      std::swap(C[c * n1 + k], C[piv * n1 + k]);
    }
    const ld d = V[c * n1 + c];
    for (int k = 0; k < n1; ++k) { V[c * n1 + k] /= d; C[c * n1 + k] /= d; }
    for (int r = 0; r < n1; ++r) {
      if (r == c) continue;
      const ld f = V[r * n1 + c];
      if (f == 0.0L) continue;
      for (int k = 0; k < n1; ++k) { V[r * n1 + k] -= f * V[c * n1 + k]; C[r * n1 + k] -= f * C[c * n1 + k]; }
    }
  }
  // l_j^(m)(x) = sum_n C[n][j] P_n^(m)(x)   (C rows: modes n, columns: nodes j)
  auto lag = [&](ld x, std::vector<ld>& L) {       // L[m * n1 + j], m = 0..p
    legendre_all(p, p, x, T);
    L.assign(n1 * n1, 0.0L);
    for (int m = 0; m <= p; ++m)
      for (int j = 0; j < n1; ++j) {
        ld s = 0.0L;
        for (int n = m; n <= p; ++n) s += C[n * n1 + j] * T[m * n1 + n];
        L[m * n1 + j] = s;
      }
  };
  std::vector<ld> L;
  for (int q = 0; q < n1; ++q) {
    out[o.xq + q] = static_cast<double>(xq[q]);
    out[o.wq + q] = static_cast<double>(wq[q]);
    lag(xq[q], L);
    for (int m = 0; m <= p; ++m)
      for (int j = 0; j < n1; ++j) out[o.DQ + (m * n1 + j) * n1 + q] = static_cast<double>(L[m * n1 + j]);
  }
  for (int v = 0; v < 2; ++v) {
    lag(v == 0 ? -1.0L : 1.0L, L);
    for (int j = 0; j < n1; ++j)
      for (int m = 0; m <= p; ++m) out[o.DV + (v * n1 + j) * n1 + m] = static_cast<double>(L[m * n1 + j]);
  }
  for (int a = 0; a < n1; ++a) {
    lag(xn[a], L);
    for (int j = 0; j < n1; ++j) out[o.DN + a * n1 + j] = static_cast<double>(L[n1 + j]);
  }
  return out;
}

// Canonical CG numbering: vertex DOFs by vertex id, then edge DOFs (edges
// sorted by (min, max) vertex id, oriented min -> max), then cell-interior
// DOFs by cell id (lexicographic inside the cell).
static bool cg_number(cvw_mesh* m, const int32_t* cv) {
  const int p = m->degree;
  const int64_t E = m->E, Nv = m->Nv;
  const int nloc = m->nloc;
  m->h_cell_dof.assign(E * nloc, -1);
  if (m->cell == CVW_SEG) {
    for (int64_t e = 0; e < E; ++e) {
      m->h_cell_dof[e * nloc] = cv[e * 2];
      m->h_cell_dof[e * nloc + p] = cv[e * 2 + 1];
      for (int t = 1; t < p; ++t) m->h_cell_dof[e * nloc + t] = static_cast<int32_t>(Nv + e * (p - 1) + t - 1);
    }
    m->ndof = Nv + E * (p - 1);
    return true;
  }
  if (m->cell != CVW_QUAD) return false;
  const int n1 = p + 1;
  auto loc = [n1](int a, int b) { return a + n1 * b; };
  const int ca[4][2] = {{0, 0}, {p, 0}, {p, p}, {0, p}};
  std::vector<std::pair<int64_t, int64_t>> keys(E * 4);
  for (int64_t e = 0; e < E; ++e) {
    for (int lv = 0; lv < 4; ++lv) m->h_cell_dof[e * nloc + loc(ca[lv][0], ca[lv][1])] = cv[e * 4 + lv];
    for (int f = 0; f < 4; ++f) {
      const int64_t a = cv[e * 4 + f], b = cv[e * 4 + (f + 1) % 4];
      keys[e * 4 + f] = {std::min(a, b), std::max(a, b)};
    }
  }
  std::vector<std::pair<int64_t, int64_t>> uniq(keys);
  std::sort(uniq.begin(), uniq.end());
  uniq.erase(std::unique(uniq.begin(), uniq.end()), uniq.end());
  const int64_t n_edges = static_cast<int64_t>(uniq.size());
  auto edge_node = [p](int f, int t, int& a, int& b) {
    switch (f) {
      case 0: a = t; b = 0; break;
      case 1: a = p; b = t; break;
      case 2: a = p - t; b = p; break;
      default: a = 0; b = p - t; break;
    }
  };
  for (int64_t e = 0; e < E; ++e)
    for (int f = 0; f < 4; ++f) {
      const int64_t eid = std::lower_bound(uniq.begin(), uniq.end(), keys[e * 4 + f]) - uniq.begin();
      const bool same = cv[e * 4 + f] < cv[e * 4 + (f + 1) % 4];
      for (int t = 1; t < p; ++t) {
        const int g = same ? t - 1 : p - 1 - t;
        int a, b;
        edge_node(f, t, a, b);
        m->h_cell_dof[e * nloc + loc(a, b)] = static_cast<int32_t>(Nv + eid * (p - 1) + g);
      }
    }
  const int64_t base = Nv + n_edges * (p - 1);
  const int ni = (p - 1) * (p - 1);
  for (int64_t e = 0; e < E; ++e)
    for (int b = 1; b < p; ++b)
      for (int a = 1; a < p; ++a)
        m->h_cell_dof[e * nloc + loc(a, b)] = static_cast<int32_t>(base + e * ni + (a - 1) + (p - 1) * (b - 1));
  m->ndof = base + E * ni;
  return true;
}

}  // namespace cvw

using namespace cvw;

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
#define CVW_HIP(call)                                                              \
  do {                                                                             \
    hipError_t _e = (call);                                                        \
    if (_e != hipSuccess) {                                                        \
      set_error(std::string(#call) + ": " + hipGetErrorString(_e));                \
      return CVW_EDEVICE;                                                          \
    }                                                                              \
  } while (0)

// Device storage of a mesh under construction: one hipMalloc per array, or
// 256-byte aligned pieces of a caller-provided buffer (cvw_mesh_build_in), or
// only a byte count (cvw_mesh_plan).
struct MeshArena {
  char* base = nullptr;
  size_t size = 0, off = 0;
  bool count_only = false;
};
static thread_local MeshArena* g_arena = nullptr;

static cvw_status dev_alloc(void** dst, size_t bytes) {
  if (!g_arena) {
    if (hipMalloc(dst, bytes) != hipSuccess) { set_error("hipMalloc failed"); return CVW_ENOMEM; }
    return CVW_OK;
  }
  MeshArena& A = *g_arena;
  A.off = (A.off + 255) / 256 * 256;
  if (A.count_only) {
    *dst = nullptr;
    A.off += bytes;
    return CVW_OK;
  }
  // the plan is the rounded end of the last piece: check that, so that every
  // buffer smaller than the plan is refused
  if ((A.off + bytes + 255) / 256 * 256 > A.size) {
    set_error("device buffer too small (cvw_mesh_plan / cvw_batch_plan give the size)");
    return CVW_EINVAL;
  }
  *dst = A.base + A.off;
  A.off += bytes;
  return CVW_OK;
}

template <typename T>
static cvw_status upload(T** dst, const std::vector<T>& src) {
  if (src.empty()) { *dst = nullptr; return CVW_OK; }
  void* p = nullptr;
  const cvw_status st = dev_alloc(&p, src.size() * sizeof(T));
  if (st != CVW_OK) return st;
  *dst = static_cast<T*>(p);
  if (g_arena && g_arena->count_only) return CVW_OK;
  CVW_HIP(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return CVW_OK;
}

// Row sums of the mass matrix (CG: the integrals of the nodal basis
// functions, the lumped mass; 1D DG: the exact, diagonal element mass of the
// Gauss-node basis), float64.  Empty when the mesh has no time-stepping path.
static std::vector<double> diag_mass(const cvw_mesh* m, const cvw_mesh_desc* d) {
  std::vector<double> out;
  const int p = m->degree;
  const int64_t E = m->E;
  if (d->cell == CVW_SEG) {
    const std::vector<double> tab = fill_hp_tables(p, d->space == CVW_CG);
    const HPOff o = hp_off(p);
    const int n1 = p + 1;
    out.assign(d->space == CVW_CG ? m->ndof : E * n1, 0.0);
    for (int64_t e = 0; e < E; ++e) {
      const double jac = 0.5 * (d->cell_coords[e * 2 + 1] - d->cell_coords[e * 2]);
      for (int j = 0; j <= p; ++j) {
        double s = 0.0;
        for (int q = 0; q <= p; ++q) s += tab[o.wq + q] * tab[o.DQ + j * n1 + q];
        const int64_t I = d->space == CVW_CG ? m->h_cell_dof[e * n1 + j] : e * n1 + j;
        out[I] += jac * s;
      }
    }
    return out;
  }
  if (p < 1 || p > MAXP) return out;
  if (d->cell == CVW_QUAD && d->space == CVW_CG && p <= 2) {
    std::vector<double> xq, wq, xn;
    gauss_rule(p + 1, xq, wq);
    lobatto_nodes(p + 1, xn);
    const int N1 = p + 1;
    const double sxv[4] = {-1, 1, 1, -1}, syv[4] = {-1, -1, 1, 1};
    out.assign(m->ndof, 0.0);
    for (int64_t e = 0; e < E; ++e) {
      const double* X = d->cell_coords + e * 8;
      for (int qy = 0; qy < N1; ++qy)
        for (int qx = 0; qx < N1; ++qx) {
          double J[2][2] = {{0, 0}, {0, 0}};
          for (int v = 0; v < 4; ++v) {
            const double Nx = 0.25 * sxv[v] * (1 + syv[v] * xq[qy]), Ny = 0.25 * syv[v] * (1 + sxv[v] * xq[qx]);
            for (int c = 0; c < 2; ++c) {
              J[c][0] += Nx * X[2 * v + c];
              J[c][1] += Ny * X[2 * v + c];
            }
          }
          const double W = wq[qx] * wq[qy] * std::fabs(J[0][0] * J[1][1] - J[0][1] * J[1][0]);
          for (int b = 0; b < N1; ++b)
            for (int a = 0; a < N1; ++a)
              out[m->h_cell_dof[e * N1 * N1 + a + N1 * b]] +=
                  W * lagrange_deriv(xn, a, 0, xq[qx]) * lagrange_deriv(xn, b, 0, xq[qy]);
        }
    }
  }
  return out;
}

static void free_mesh(cvw_mesh* m) {
  if (!m) return;
  if (m->external) {                 // device arrays live in the caller's buffer
    delete m;
    return;
  }
  (void)hipFree(m->d_vtx_ptr);
  (void)hipFree(m->d_vtx_ent);
  (void)hipFree(m->d_cell_vtx);
  (void)hipFree(m->d_nbr);
  (void)hipFree(m->d_tens);
  (void)hipFree(m->d_lanes);
  (void)hipFree(m->d_cell_dof);
  (void)hipFree(m->d_dof_ptr);
  (void)hipFree(m->d_dof_ent);
  (void)hipFree(m->d_geo);
  (void)hipFree(m->d_he);
  (void)hipFree(m->d_cgt);
  (void)hipFree(m->d_hcell);
  (void)hipFree(m->d_segt);
  (void)hipFree(m->d_hp);
  (void)hipFree(m->d_trit);
  (void)hipFree(m->d_geot);
  (void)hipFree(m->d_geov);
  (void)hipFree(m->d_nbrf);
  (void)hipFree(m->d_hext);
  (void)hipFree(m->d_tett);
  (void)hipFree(m->d_geoth);
  (void)hipFree(m->d_nbrt);
  (void)hipFree(m->d_dinv_f);
  (void)hipFree(m->d_dinv_d);
  delete m;
}

extern "C" {

int cvw_abi_version(void) { return CVW_ABI_VERSION; }

const char* cvw_last_error(void) { return g_err.c_str(); }

void cvw_mesh_destroy(cvw_mesh* mesh) { free_mesh(mesh); }

cvw_status cvw_mesh_build(const cvw_mesh_desc* d, cvw_mesh** out) {
  if (!d || !out) { set_error("null argument"); return CVW_EINVAL; }
  *out = nullptr;
  if (!d->cell_vertices || !d->cell_coords) { set_error("null mesh arrays"); return CVW_EINVAL; }
  int ve, nf;
  if (d->cell == CVW_SEG && d->dim == 1) { ve = 2; nf = 2; }
  else if (d->cell == CVW_TRI && d->dim == 2) { ve = 3; nf = 3; }
  else if (d->cell == CVW_QUAD && d->dim == 2) { ve = 4; nf = 4; }
  else if (d->cell == CVW_HEX && d->dim == 3) { ve = 8; nf = 6; }
  else if (d->cell == CVW_TET && d->dim == 3) { ve = 4; nf = 4; }
  else { set_error("cell type / dimension mismatch"); return CVW_EINVAL; }
  if (d->cell == CVW_HEX && d->space != CVW_DG) { set_error("hexahedra: DG only"); return CVW_EUNSUPPORTED; }
  if (d->cell == CVW_TET && d->space != CVW_DG) { set_error("tetrahedra: DG only"); return CVW_EUNSUPPORTED; }
  if (d->degree < 1 || d->degree > (d->cell == CVW_SEG ? HP_MAXP : 16)) { set_error("degree out of range"); return CVW_EINVAL; }
  if (d->space != CVW_CG && d->space != CVW_DG) { set_error("space must be CG or DG"); return CVW_EINVAL; }
  if (d->n_cells <= 0 || d->n_vertices <= 0) { set_error("empty mesh"); return CVW_EINVAL; }
  // packed (cell, local index) entries: cell * 4 + local vertex, cell * n_loc + local CG node
  const int64_t nloc_d = d->cell == CVW_SEG ? d->degree + 1 : d->cell == CVW_QUAD ? (d->degree + 1) * (d->degree + 1)
                          : d->cell == CVW_HEX ? (d->degree + 1) * (d->degree + 1) * (d->degree + 1)
                          : d->cell == CVW_TET ? (d->degree + 1) * (d->degree + 2) * (d->degree + 3) / 6
                                               : (d->degree + 1) * (d->degree + 2) / 2;
  if (d->n_cells * std::max<int64_t>(8, nloc_d) >= (int64_t(1) << 31) || d->n_vertices >= (int64_t(1) << 31)) {
    set_error("mesh too large for 32-bit indices"); return CVW_EINVAL;
  }
  const int64_t E = d->n_cells, Nv = d->n_vertices;
  auto* m = new cvw_mesh();
  m->external = g_arena != nullptr;
  m->dim = d->dim; m->cell = d->cell; m->degree = d->degree; m->space = d->space;
  m->E = E; m->Nv = Nv; m->ve = ve; m->nf = nf;
  const int p = d->degree;
  if (d->cell == CVW_TRI) { m->nloc = (p + 1) * (p + 2) / 2; m->nq = (p + 1) * (p + 1); }
  else if (d->cell == CVW_QUAD) { m->nloc = (p + 1) * (p + 1); m->nq = (p + 1) * (p + 1); }
  else if (d->cell == CVW_HEX) { m->nloc = (p + 1) * (p + 1) * (p + 1); m->nq = m->nloc; }
  else if (d->cell == CVW_TET) { m->nloc = (p + 1) * (p + 2) * (p + 3) / 6; m->nq = (p + 1) * (p + 1) * (p + 1); }
  else { m->nloc = p + 1; m->nq = p + 1; }
  m->nk = (d->dim == 1) ? p : d->dim == 2 ? (p + 1) * (p + 2) / 2 - 1 : (p + 1) * (p + 2) * (p + 3) / 6 - 1;
  (void)hipGetDevice(&m->device);

  // ---- validation and vertex patches (CSR in ascending (cell, local vertex)) ----
  m->h_cell_vtx.assign(d->cell_vertices, d->cell_vertices + E * ve);
  std::vector<int32_t> cnt(Nv, 0);
  for (int64_t e = 0; e < E; ++e)
    for (int l = 0; l < ve; ++l) {
      const int32_t v = d->cell_vertices[e * ve + l];
      if (v < 0 || v >= Nv) { free_mesh(m); set_error("vertex id out of range"); return CVW_EINVAL; }
      for (int l2 = 0; l2 < l; ++l2)
        if (d->cell_vertices[e * ve + l2] == v) { free_mesh(m); set_error("repeated vertex in a cell"); return CVW_EINVAL; }
      ++cnt[v];
    }
  m->h_vtx_ptr.assign(Nv + 1, 0);
  for (int64_t v = 0; v < Nv; ++v) {
    if (cnt[v] == 0) { free_mesh(m); set_error("vertex not used by any cell"); return CVW_EINVAL; }
    m->h_vtx_ptr[v + 1] = m->h_vtx_ptr[v] + cnt[v];
  }
  m->nnz = m->h_vtx_ptr[Nv];
  m->h_vtx_cell.assign(m->nnz, 0);
  m->h_vtx_lv.assign(m->nnz, 0);
  std::vector<int32_t> fill(m->h_vtx_ptr.begin(), m->h_vtx_ptr.end() - 1);
  std::vector<int32_t> ent(m->nnz);
  for (int64_t e = 0; e < E; ++e)
    for (int l = 0; l < ve; ++l) {
      const int32_t v = d->cell_vertices[e * ve + l];
      const int32_t pos = fill[v]++;
      m->h_vtx_cell[pos] = static_cast<int32_t>(e);
      m->h_vtx_lv[pos] = l;
      ent[pos] = static_cast<int32_t>(e * (ve == 8 ? 8 : 4) + l);   // tetrahedra: cell * 4 + lv
    }

  // ---- geometry ----
  m->h_coords.assign(d->cell_coords, d->cell_coords + E * ve * d->dim);
  m->h_he.assign(E, 0.0);
  for (int64_t e = 0; e < E; ++e) {
    double hmax = 0.0;
    for (int i = 0; i < ve; ++i)
      for (int j = i + 1; j < ve; ++j) {
        double s = 0.0;
        for (int c = 0; c < d->dim; ++c) {
          const double dd = d->cell_coords[(e * ve + i) * d->dim + c] - d->cell_coords[(e * ve + j) * d->dim + c];
          s += dd * dd;
        }
        hmax = std::max(hmax, std::sqrt(s));
      }
    if (!(hmax > 0.0) || !std::isfinite(hmax)) { free_mesh(m); set_error("degenerate cell"); return CVW_EINVAL; }
    m->h_he[e] = hmax;
  }
  if (d->cell == CVW_QUAD) {
    // congruent axis-aligned rectangles?
    const double* X = d->cell_coords;
    const double hx0 = X[2] - X[0], hy0 = X[5] - X[3];
    bool uni = hx0 > 0 && hy0 > 0;
    const double tol = 1e-9;
    for (int64_t e = 0; e < E && uni; ++e) {
      const double* c = X + e * 8;
      const double hx = c[2] - c[0], hy = c[7] - c[1];
      uni = std::fabs(c[3] - c[1]) <= tol * hy0 && std::fabs(c[4] - c[2]) <= tol * hx0 &&
            std::fabs(c[5] - c[7]) <= tol * hy0 && std::fabs(c[6] - c[0]) <= tol * hx0 &&
            std::fabs(hx - hx0) <= tol * hx0 && std::fabs(hy - hy0) <= tol * hy0;
    }
    m->uniform = uni ? 1 : 0;
    if (uni) { m->hx = hx0; m->hy = hy0; m->he = std::sqrt(hx0 * hx0 + hy0 * hy0); }
  }

  if (d->cell == CVW_HEX) {
    // congruent axis-aligned boxes, vertices at the corners in the local order
    // (the face z = z0 counter-clockwise from the lowest corner, then z = z0 + hz)
    static const int SG[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0}, {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
    const double* X = d->cell_coords;
    const double h0[3] = {X[3] - X[0], X[10] - X[1], X[14] - X[2]};
    bool uni = h0[0] > 0 && h0[1] > 0 && h0[2] > 0;
    const double tol = 1e-9;
    for (int64_t e = 0; e < E && uni; ++e) {
      const double* c = X + e * 24;
      for (int v = 0; v < 8 && uni; ++v)
        for (int a = 0; a < 3 && uni; ++a) uni = std::fabs(c[v * 3 + a] - c[a] - SG[v][a] * h0[a]) <= tol * h0[a];
    }
    m->uniform = uni ? 1 : 0;
    if (uni) { m->hx = h0[0]; m->hy = h0[1]; m->hz = h0[2]; m->he = std::sqrt(h0[0] * h0[0] + h0[1] * h0[1] + h0[2] * h0[2]); }
  }

  // ---- ends of a line: vertices of one cell ----
  if (d->cell == CVW_SEG) {
    for (int64_t v = 0; v < Nv; ++v) m->open_ends += cnt[v] == 1 ? 1 : 0;
    // every other vertex joins the right vertex of one cell to the left vertex of another
    std::vector<int8_t> side(Nv, 0);
    for (int64_t e = 0; e < E; ++e)
      for (int l = 0; l < 2; ++l) {
        const int32_t v = d->cell_vertices[e * 2 + l];
        if (cnt[v] > 2 || (cnt[v] == 2 && (side[v] & (1 << l)))) {
          free_mesh(m); set_error("a line's vertex must join the right end of one cell to the left end of another");
          return CVW_EINVAL;
        }
        side[v] |= static_cast<int8_t>(1 << l);
      }
  }

  // ---- DG face neighbours ----
  if (d->space == CVW_DG && (d->cell == CVW_HEX || d->cell == CVW_TET)) {
    // a face of a hexahedron is its four vertices (local faces 2 axis + side);
    // of a tetrahedron its three vertices (face f opposite vertex f)
    static const int FVH[6][4] = {{0, 3, 7, 4}, {1, 2, 6, 5}, {0, 1, 5, 4}, {3, 2, 6, 7}, {0, 1, 2, 3}, {4, 5, 6, 7}};
    static const int FVT[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    const bool hexc = d->cell == CVW_HEX;
    const int nfv = hexc ? 4 : 3;
    struct HK { std::array<int32_t, 4> v; int32_t ef; };
    std::vector<HK> keys(E * nf);
    for (int64_t e = 0; e < E; ++e)
      for (int f = 0; f < nf; ++f) {
        HK k;
        k.v = {-1, -1, -1, -1};
        for (int i = 0; i < nfv; ++i) k.v[i] = d->cell_vertices[e * ve + (hexc ? FVH[f][i] : FVT[f][i])];
        std::sort(k.v.begin(), k.v.end());
        k.ef = static_cast<int32_t>(e * nf + f);
        keys[e * nf + f] = k;
      }
    std::sort(keys.begin(), keys.end(), [](const HK& a, const HK& b) { return a.v < b.v || (a.v == b.v && a.ef < b.ef); });
    m->h_nbr.assign(E * nf, -1);
    m->h_nbr_face.assign(E * nf, -1);
    for (size_t i = 0; i < keys.size();) {
      size_t j = i;
      while (j + 1 < keys.size() && keys[j + 1].v == keys[i].v) ++j;
      if (j - i + 1 > 2) { free_mesh(m); set_error("non-conforming mesh: face shared by more than two cells"); return CVW_EINVAL; }
      if (j == i + 1) {
        const int32_t a = keys[i].ef, b = keys[j].ef;
        m->h_nbr[a] = b / nf; m->h_nbr_face[a] = b % nf;
        m->h_nbr[b] = a / nf; m->h_nbr_face[b] = a % nf;
      }
      i = j + 1;
    }
    m->closed = std::all_of(m->h_nbr.begin(), m->h_nbr.end(), [](int32_t x) { return x >= 0; }) ? 1 : 0;
    for (int64_t i = 0; i < E * nf; ++i)
      if (m->h_nbr[i] < 0) { m->h_bface.push_back(static_cast<int32_t>(i / nf)); m->h_bface.push_back(static_cast<int32_t>(i % nf)); }
    m->n_bfaces = static_cast<int64_t>(m->h_bface.size() / 2);
    // the hexahedron cell pass reads the neighbour across face f through its face f ^ 1
    if (hexc)
      for (int64_t i = 0; i < E * 6; ++i)
        if (m->h_nbr[i] >= 0 && m->h_nbr_face[i] != ((i % 6) ^ 1)) { m->uniform = 0; break; }
  } else if (d->space == CVW_DG) {
    struct FK { int64_t key; int32_t ef; };
    std::vector<FK> keys(E * nf);
    for (int64_t e = 0; e < E; ++e)
      for (int f = 0; f < nf; ++f) {
        int64_t key;
        if (ve == 2) {
          key = d->cell_vertices[e * 2 + f];
        } else {
          const int64_t v0 = d->cell_vertices[e * ve + f], v1 = d->cell_vertices[e * ve + (f + 1) % ve];
          key = std::min(v0, v1) * Nv + std::max(v0, v1);
        }
        keys[e * nf + f] = {key, static_cast<int32_t>(e * nf + f)};
      }
    std::sort(keys.begin(), keys.end(), [](const FK& x, const FK& y) { return x.key < y.key || (x.key == y.key && x.ef < y.ef); });
    m->h_nbr.assign(E * nf, -1);
    m->h_nbr_face.assign(E * nf, -1);
    for (size_t i = 0; i < keys.size();) {
      size_t j = i;
      while (j + 1 < keys.size() && keys[j + 1].key == keys[i].key) ++j;
      if (j - i + 1 > 2) { free_mesh(m); set_error("non-conforming mesh: face shared by more than two cells"); return CVW_EINVAL; }
      if (j == i + 1) {
        const int32_t a = keys[i].ef, b = keys[j].ef;
        const int32_t ea = a / nf, fa = a % nf, eb = b / nf, fb = b % nf;
        if (ve > 2) {
          const int32_t a0 = d->cell_vertices[ea * ve + fa], a1 = d->cell_vertices[ea * ve + (fa + 1) % ve];
          const int32_t b0 = d->cell_vertices[eb * ve + fb], b1 = d->cell_vertices[eb * ve + (fb + 1) % ve];
          if (!(a0 == b1 && a1 == b0)) { free_mesh(m); set_error("inconsistently oriented shared face"); return CVW_EINVAL; }
        }
        m->h_nbr[a] = eb; m->h_nbr_face[a] = fb;
        m->h_nbr[b] = ea; m->h_nbr_face[b] = fa;
      }
      i = j + 1;
    }
    m->closed = std::all_of(m->h_nbr.begin(), m->h_nbr.end(), [](int32_t x) { return x >= 0; }) ? 1 : 0;
    for (int64_t i = 0; i < E * nf; ++i)
      if (m->h_nbr[i] < 0) {
        m->h_bface.push_back(static_cast<int32_t>(i / nf));
        m->h_bface.push_back(static_cast<int32_t>(i % nf));
      }
    m->n_bfaces = static_cast<int64_t>(m->h_bface.size() / 2);
    if (m->cell == CVW_SEG && m->closed) {
      // the 1D kernels read the neighbour across face f through its face 1 - f
      for (int64_t i = 0; i < E * 2; ++i)
        if (m->h_nbr_face[i] != 1 - (i % 2)) { m->closed = 0; break; }
    }
    if (m->cell == CVW_QUAD) {
      // the structured DG path reads the neighbour across face f through its face (f + 2) mod 4
      for (int64_t i = 0; i < E * 4; ++i)
        if (m->h_nbr[i] >= 0 && m->h_nbr_face[i] != (i % 4 + 2) % 4) { m->uniform = 0; break; }
    }
  }

  // ---- structured periodic DG grid (cells e = i + nx j, four cells at every
  // vertex): the fused sensor pass reads the neighbours by index arithmetic
  if (d->cell == CVW_QUAD && d->space == CVW_DG && m->uniform && m->closed) {
    const int64_t nx = m->h_nbr[2];                 // north neighbour of cell 0
    bool ok = nx >= 3 && E % nx == 0 && E / nx >= 3;
    const int64_t ny = ok ? E / nx : 0;
    for (int64_t e = 0; e < E && ok; ++e) {
      const int64_t i = e % nx, j = e / nx;
      ok = m->h_nbr[e * 4 + 0] == i + nx * ((j + ny - 1) % ny) && m->h_nbr[e * 4 + 1] == (i + 1) % nx + nx * j &&
           m->h_nbr[e * 4 + 2] == i + nx * ((j + 1) % ny) && m->h_nbr[e * 4 + 3] == (i + nx - 1) % nx + nx * j;
    }
    for (int64_t v = 0; v < Nv && ok; ++v) ok = m->h_vtx_ptr[v + 1] - m->h_vtx_ptr[v] == 4;
    if (ok) { m->grid_nx = nx; m->grid_ny = ny; }
  }

  // ---- CG numbering, DOF patches, per-cell geometry ----
  std::vector<int32_t> dptr, dent;
  std::vector<float> geo, hef;
  if (d->space == CVW_CG) {
    if (d->cell == CVW_TRI) { free_mesh(m); set_error("CG on triangles is not implemented"); return CVW_EUNSUPPORTED; }
    cg_number(m, d->cell_vertices);
    std::vector<int32_t> dc(m->ndof, 0);
    for (int32_t v : m->h_cell_dof) ++dc[v];
    dptr.assign(m->ndof + 1, 0);
    for (int64_t i = 0; i < m->ndof; ++i) dptr[i + 1] = dptr[i] + dc[i];
    dent.assign(E * m->nloc, 0);
    std::vector<int32_t> fp(dptr.begin(), dptr.end() - 1);
    for (int64_t e = 0; e < E; ++e)
      for (int j = 0; j < m->nloc; ++j) dent[fp[m->h_cell_dof[e * m->nloc + j]]++] = static_cast<int32_t>(e * m->nloc + j);
  }
  if (d->dim == 2) {
    geo.assign(E * 8, 0.0f);
    for (int64_t e = 0; e < E; ++e) {
      const double* X = d->cell_coords + e * ve * 2;
      geo[e * 8] = static_cast<float>(X[0]);
      geo[e * 8 + 1] = static_cast<float>(X[1]);
      for (int v = 1; v < ve && v < 4; ++v) {
        geo[e * 8 + 2 * v] = static_cast<float>(X[2 * v] - X[0]);
        geo[e * 8 + 2 * v + 1] = static_cast<float>(X[2 * v + 1] - X[1]);
      }
    }
  }
  hef.assign(m->h_he.begin(), m->h_he.end());

  // ---- reference tables ----
  if (d->cell == CVW_QUAD || d->cell == CVW_SEG)
    fill_tensor_tables(m->tens, std::min(p, MAXP), d->space == CVW_CG);
  if (d->space == CVW_CG && p <= 2) fill_cg_tables(m->cgt, p);

  // ---- upload ----
  cvw_status st;
  // hexahedra: each vertex's patch in the order of its octants (entry 8 v + l
  // is the cell whose local vertex l it is) when every vertex has exactly one
  // cell in each of its eight octants (closed conforming box meshes); the
  // vertex pass of the GPU path needs that order
  bool hex_oct = false;
  if (d->cell == CVW_HEX) {
    hex_oct = m->nnz == 8 * Nv;
    std::vector<int32_t> eo(hex_oct ? m->nnz : 0, -1);
    for (int64_t v = 0; v < Nv && hex_oct; ++v) {
      if (m->h_vtx_ptr[v + 1] - m->h_vtx_ptr[v] != 8) { hex_oct = false; break; }
      for (int32_t i = m->h_vtx_ptr[v]; i < m->h_vtx_ptr[v + 1] && hex_oct; ++i) {
        const int l = m->h_vtx_lv[i];
        if (eo[8 * v + l] >= 0) hex_oct = false;
        else eo[8 * v + l] = ent[i];
      }
    }
    if (hex_oct) ent.swap(eo);
  }
  std::vector<int32_t> ptr32(m->h_vtx_ptr.begin(), m->h_vtx_ptr.end());
  if ((st = upload(&m->d_vtx_ptr, ptr32)) != CVW_OK) { free_mesh(m); return st; }
  if ((st = upload(&m->d_vtx_ent, ent)) != CVW_OK) { free_mesh(m); return st; }
  if ((st = upload(&m->d_cell_vtx, m->h_cell_vtx)) != CVW_OK) { free_mesh(m); return st; }
  {
    // device neighbour table: boundary face b (ascending (cell, face)) as -(b + 1)
    std::vector<int32_t> dn(m->h_nbr);
    int32_t b = 0;
    for (auto& x : dn)
      if (x < 0) x = -(++b);
    if ((st = upload(&m->d_nbr, dn)) != CVW_OK) { free_mesh(m); return st; }
  }
  if ((st = upload(&m->d_cell_dof, m->h_cell_dof)) != CVW_OK) { free_mesh(m); return st; }
  if ((st = upload(&m->d_dof_ptr, dptr)) != CVW_OK) { free_mesh(m); return st; }
  if ((st = upload(&m->d_dof_ent, dent)) != CVW_OK) { free_mesh(m); return st; }
  if ((st = upload(&m->d_geo, geo)) != CVW_OK) { free_mesh(m); return st; }
  if ((st = upload(&m->d_he, hef)) != CVW_OK) { free_mesh(m); return st; }
  {
    std::vector<CGTables> t1(1, m->cgt);
    if ((st = upload(&m->d_cgt, t1)) != CVW_OK) { free_mesh(m); return st; }
  }
  if (d->cell == CVW_QUAD && d->space == CVW_DG && p <= MAXP) {
    std::vector<LaneRec> lr(16);
    fill_lane_tables(lr.data(), m->tens, p);
    if ((st = upload(&m->d_lanes, lr)) != CVW_OK) { free_mesh(m); return st; }
  }
  if (d->cell == CVW_SEG) {
    std::vector<double> hc(E);
    for (int64_t e = 0; e < E; ++e) hc[e] = d->cell_coords[e * 2 + 1] - d->cell_coords[e * 2];
    for (int64_t e = 0; e < E; ++e)
      if (!(hc[e] > 0)) { free_mesh(m); set_error("segment cells must have x1 > x0"); return CVW_EINVAL; }
    if ((st = upload(&m->d_hcell, hc)) != CVW_OK) { free_mesh(m); return st; }
    std::vector<SegTables> t1(1);
    fill_seg_tables(t1[0], std::min(p, MAXP), d->space == CVW_CG);
    if ((st = upload(&m->d_segt, t1)) != CVW_OK) { free_mesh(m); return st; }
    if ((st = upload(&m->d_hp, fill_hp_tables(p, d->space == CVW_CG))) != CVW_OK) { free_mesh(m); return st; }
  }
  if (d->cell == CVW_TRI && d->space == CVW_DG && p <= MAXP) {
    std::vector<double> gt(E * 8, 0.0);
    for (int64_t e = 0; e < E; ++e) {
      const double* X = d->cell_coords + e * 6;
      double* g = gt.data() + e * 8;
      g[0] = X[0]; g[1] = X[1];
      g[2] = X[2] - X[0]; g[3] = X[3] - X[1];
      g[4] = X[4] - X[0]; g[5] = X[5] - X[1];
      g[6] = m->h_he[e];
      if (!(g[2] * g[5] - g[4] * g[3] > 0.0)) {
        free_mesh(m); set_error("triangles must be counter-clockwise and non-degenerate"); return CVW_EINVAL;
      }
    }
    if ((st = upload(&m->d_geot, gt)) != CVW_OK) { free_mesh(m); return st; }
    // the vertex pass reads each triangle from all three of its vertices: a
    // 32-byte float32 record of what it needs (the inverse Jacobian and h_e)
    std::vector<float> gv(E * 8, 0.0f);
    for (int64_t e = 0; e < E; ++e) {
      const double* g = gt.data() + e * 8;
      const double det = g[2] * g[5] - g[4] * g[3];
      float* o = gv.data() + e * 8;
      o[0] = static_cast<float>(g[5] / det);       // A = J^{-1}, J = [[x1-x0, x2-x0], [y1-y0, y2-y0]]
      o[1] = static_cast<float>(-g[4] / det);
      o[2] = static_cast<float>(-g[3] / det);
      o[3] = static_cast<float>(g[2] / det);
      o[4] = static_cast<float>(g[6]);
    }
    if ((st = upload(&m->d_geov, gv)) != CVW_OK) { free_mesh(m); return st; }
    std::vector<int32_t> nf32(E * 3);
    int32_t nbf = 0;
    for (int64_t i = 0; i < E * 3; ++i) nf32[i] = m->h_nbr[i] < 0 ? -(++nbf) : m->h_nbr[i] * 4 + m->h_nbr_face[i];
    if ((st = upload(&m->d_nbrf, nf32)) != CVW_OK) { free_mesh(m); return st; }
    std::vector<TriTables> tt(1);
    fill_tri_tables(tt[0], p);
    if ((st = upload(&m->d_trit, tt)) != CVW_OK) { free_mesh(m); return st; }
  }
  if (d->cell == CVW_HEX && m->uniform && hex_oct && p <= HEX_MAXP) {
    std::vector<HexTables> ht(1);
    if (!fill_hex_tables(ht[0], p, m->hx, m->hy, m->hz)) { free_mesh(m); return CVW_EUNSUPPORTED; }
    if ((st = upload(&m->d_hext, ht)) != CVW_OK) { free_mesh(m); return st; }
  }
  if (d->cell == CVW_TET) {
    // per-cell geometry: vertex 0, J = [x1 - x0, x2 - x0, x3 - x0] (columns), diam; positive orientation
    std::vector<double> gt(E * 16, 0.0);
    for (int64_t e = 0; e < E; ++e) {
      const double* X = d->cell_coords + e * 12;
      double* g = gt.data() + e * 16;
      for (int a = 0; a < 3; ++a) {
        g[a] = X[a];
        for (int b = 0; b < 3; ++b) g[3 + 3 * a + b] = X[3 * (b + 1) + a] - X[a];
      }
      g[12] = m->h_he[e];
      const double* J = g + 3;
      const double det = J[0] * (J[4] * J[8] - J[5] * J[7]) - J[1] * (J[3] * J[8] - J[5] * J[6]) + J[2] * (J[3] * J[7] - J[4] * J[6]);
      if (!(det > 0.0)) { free_mesh(m); set_error("tetrahedra must be positively oriented and non-degenerate"); return CVW_EINVAL; }
    }
    if ((st = upload(&m->d_geoth, gt)) != CVW_OK) { free_mesh(m); return st; }
    if (E >= (int64_t(1) << 26)) { free_mesh(m); set_error("tetrahedral mesh too large for the packed neighbour codes"); return CVW_EINVAL; }
    // neighbour code: cell * 32 + its face * 8 + the permutation taking this face's
    // vertex order (face f opposite vertex f, increasing) to the neighbour's
    static const int FVT[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    static const int SIG[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    std::vector<int32_t> nc(E * 4, -1);
    for (int64_t e = 0; e < E; ++e)
      for (int f = 0; f < 4; ++f) {
        const int32_t e2 = m->h_nbr[e * 4 + f];
        if (e2 < 0) continue;
        const int f2 = m->h_nbr_face[e * 4 + f];
        int Gv[3], Hv[3];
        for (int i = 0; i < 3; ++i) {
          Gv[i] = d->cell_vertices[e * 4 + FVT[f][i]];
          Hv[i] = d->cell_vertices[static_cast<int64_t>(e2) * 4 + FVT[f2][i]];
        }
        // sigma(j) = i with H[j] = G[i]: the neighbour's barycentric j is the own barycentric sigma(j)
        int sg = -1;
        for (int c = 0; c < 6 && sg < 0; ++c) {
          bool ok = true;
          for (int j = 0; j < 3; ++j) ok = ok && Hv[j] == Gv[SIG[c][j]];
          if (ok) sg = c;
        }
        if (sg < 0) { free_mesh(m); set_error("tetrahedral faces do not match"); return CVW_EINVAL; }
        nc[e * 4 + f] = e2 * 32 + f2 * 8 + sg;
      }
    if ((st = upload(&m->d_nbrt, nc)) != CVW_OK) { free_mesh(m); return st; }
    if (p <= TET_MAXP) {
      std::vector<TetTables> tt(1);
      fill_tet_tables(tt[0], p);
      if ((st = upload(&m->d_tett, tt)) != CVW_OK) { free_mesh(m); return st; }
    }
  }
  {
    const std::vector<double> dm = diag_mass(m, d);
    for (double v : dm)
      if (!(v > 0)) { free_mesh(m); set_error("non-positive lumped mass (degenerate cell)"); return CVW_EINVAL; }
    if (!dm.empty()) {
      std::vector<double> inv_d(dm.size());
      std::vector<float> inv_f(dm.size());
      for (size_t i = 0; i < dm.size(); ++i) {
        inv_d[i] = 1.0 / dm[i];
        inv_f[i] = static_cast<float>(inv_d[i]);
      }
      m->n_mass = static_cast<int64_t>(dm.size());
      if ((st = upload(&m->d_dinv_d, inv_d)) != CVW_OK) { free_mesh(m); return st; }
      if ((st = upload(&m->d_dinv_f, inv_f)) != CVW_OK) { free_mesh(m); return st; }
    }
  }
  {
    std::vector<TensorTables> t1(1, m->tens);
    if ((st = upload(&m->d_tens, t1)) != CVW_OK) { free_mesh(m); return st; }
  }
  *out = m;
  return CVW_OK;
}

cvw_status cvw_mesh_get_info(const cvw_mesh* m, cvw_mesh_info* info) {
  if (!m || !info) { set_error("null argument"); return CVW_EINVAL; }
  info->n_cells = m->E; info->n_vertices = m->Nv; info->n_dof = m->ndof; info->nnz_vertex = m->nnz;
  info->n_loc = m->nloc; info->n_k = m->nk; info->n_q = m->nq; info->v_e = m->ve; info->n_faces = m->nf;
  info->uniform = m->uniform; info->hx = m->hx; info->hy = m->hy;
  info->grid_nx = m->grid_nx; info->grid_ny = m->grid_ny;
  info->n_bfaces = m->n_bfaces;
  return CVW_OK;
}

cvw_status cvw_mesh_plan(const cvw_mesh_desc* d, size_t* device_bytes) {
  if (!d || !device_bytes) { set_error("null argument"); return CVW_EINVAL; }
  MeshArena A;
  A.count_only = true;
  g_arena = &A;
  cvw_mesh* m = nullptr;
  const cvw_status st = cvw_mesh_build(d, &m);
  g_arena = nullptr;
  if (st != CVW_OK) return st;
  free_mesh(m);
  *device_bytes = (A.off + 255) / 256 * 256;
  return CVW_OK;
}

cvw_status cvw_mesh_build_in(const cvw_mesh_desc* d, void* device_buf, size_t bytes, cvw_mesh** out) {
  if (!d || !out || !device_buf) { set_error("null argument"); return CVW_EINVAL; }
  if (reinterpret_cast<uintptr_t>(device_buf) % 256 != 0) { set_error("device buffer not 256-byte aligned"); return CVW_EINVAL; }
  MeshArena A;
  A.base = static_cast<char*>(device_buf);
  A.size = bytes;
  g_arena = &A;
  const cvw_status st = cvw_mesh_build(d, out);
  g_arena = nullptr;
  return st;
}

cvw_status cvw_mesh_set_grid(cvw_mesh* m, int blocks) {
  if (!m) { set_error("null mesh"); return CVW_EINVAL; }
  m->eval_grid = blocks > 0 ? blocks : 0;
  return CVW_OK;
}

cvw_status cvw_mesh_export(const cvw_mesh* m, int which, void* dst, size_t bytes) {
  if (!m || !dst) { set_error("null argument"); return CVW_EINVAL; }
  const std::vector<int32_t>* src = nullptr;
  switch (which) {
    case CVW_EXPORT_VTX_PTR: src = &m->h_vtx_ptr; break;
    case CVW_EXPORT_VTX_CELL: src = &m->h_vtx_cell; break;
    case CVW_EXPORT_VTX_LV: src = &m->h_vtx_lv; break;
    case CVW_EXPORT_NBR: src = &m->h_nbr; break;
    case CVW_EXPORT_NBR_FACE: src = &m->h_nbr_face; break;
    case CVW_EXPORT_CELL_DOF: src = &m->h_cell_dof; break;
    case CVW_EXPORT_BFACE: src = &m->h_bface; break;
    default: set_error("unknown export selector"); return CVW_EINVAL;
  }
  if (bytes != src->size() * sizeof(int32_t)) { set_error("export size mismatch"); return CVW_EINVAL; }
  std::memcpy(dst, src->data(), bytes);
  return CVW_OK;
}

// ---------------------------------------------------------------------------
// workspace: [status 256 B][candidates n_k * Nv][stage 1][stage 2]
// ---------------------------------------------------------------------------
// learned-sensor network: float32 master parameters, Adam moments and the
// device compute copies, in one allocation
struct cvw_mlp {
  int device = 0;
  int64_t steps = 0;
  int external = 0;                  // mem is the caller's buffer (cvw_mlp_create_in): not freed here
  void* mem = nullptr;
  float* master = nullptr;
  float* m1 = nullptr;
  float* m2 = nullptr;
  float* b1 = nullptr;
  float* b2 = nullptr;
  float* b3 = nullptr;
  uint16_t* W1t = nullptr;
  uint16_t* W2t = nullptr;
  uint16_t* W2r = nullptr;
  uint16_t* w3 = nullptr;
  float* lo = nullptr;               // validity box of the features [48] each (-inf / +inf at creation)
  float* hi = nullptr;
  cvw::MlpDev dev() const { return {W1t, W2t, W2r, w3, b1, b2, b3}; }
  cvw::MlpDevMut mut() const { return {W1t, W2t, W2r, w3, b1, b2, b3}; }
};

static size_t state_elems(const cvw_mesh* m, int nv) {
  return static_cast<size_t>(nv) * (m->space == CVW_DG ? static_cast<size_t>(m->E) * m->nloc : static_cast<size_t>(m->ndof));
}
static size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// CVW_SENSOR_PATH=twopass in the environment keeps the two-pass plain sensor
// (vertex candidates in the workspace, then the cell pass) on structured grids
// too; both paths compute eq. gamma and are tested against the oracle
static bool twopass_forced() {
  const char* v = std::getenv("CVW_SENSOR_PATH");
  return v && std::strcmp(v, "twopass") == 0;
}
// the fused sensor pass applies: plain sensor on a structured periodic DG quadrilateral grid
static bool use_tile(const cvw_mesh* m, const cvw_params* prm) {
  return m->cell == CVW_QUAD && m->space == CVW_DG && m->grid_nx > 0 && prm->sensor == CVW_SENSOR_PLAIN &&
         !twopass_forced();
}


// true when the mesh has a time-stepping path (stages and steps)
static bool has_stage(const cvw_mesh* m) {
  return m->n_mass > 0 || (m->space == CVW_DG && (m->cell == CVW_QUAD || (m->cell == CVW_TRI && m->d_trit) ||
                                                  (m->cell == CVW_HEX && m->d_hext) || (m->cell == CVW_TET && m->d_tett)));
}

// float64 scratch of the totals: block partials of up to four variables and the results
constexpr size_t TOT_SCRATCH = (4 * 1024 + 4) * sizeof(double) + 224;

// CG scratch: P_h grad u (2D: two components; 1D: one per variable) and the
// element rows of every variable
static size_t pg_elems(const cvw_mesh* m, const cvw_params* prm) {
  return static_cast<size_t>(std::max(2, n_var(m, prm->flux))) * m->ndof;
}
static size_t rcell_elems(const cvw_mesh* m, const cvw_params* prm) {
  return static_cast<size_t>(n_var(m, prm->flux)) * m->E * m->nloc;
}

static size_t cg_extra(const cvw_mesh* m, const cvw_params* prm, size_t es) {
  size_t b = 0;
  if (m->space == CVW_CG) b += align256(pg_elems(m, prm) * es) + align256(rcell_elems(m, prm) * es);
  if (m->n_mass > 0) {
    // stage right-hand side R, and for CG the PCG vectors x, r, z, p, Ap (every
    // variable) and its block partials and scalars
    b += align256(state_elems(m, n_var(m, prm->flux)) * es);
    if (m->space == CVW_CG)
      b += 5 * align256(state_elems(m, n_var(m, prm->flux)) * es) + align256((pcg_partials(m->ndof) + 8) * sizeof(double));
  }
  return b;
}

size_t cvw_workspace_bytes(const cvw_mesh* m, const cvw_params* prm, int op) {
  if (!m || !prm) return 0;
  if (op == 3) return 256 + align256(static_cast<size_t>(m->E) * 4);   // positivity: count, cell list
  const size_t es = prm->dtype == CVW_F64 ? 8 : 4;
  // the vertex candidates go through the workspace except in the fused sensor pass
  const size_t cand = use_tile(m, prm) ? 0 : align256(static_cast<size_t>(m->nk) * m->Nv * es);
  size_t b = 256 + TOT_SCRATCH + cand + cg_extra(m, prm, es);
  if (prm->sensor == CVW_SENSOR_LEARNED)      // features, tile flags, audit partials and results
    b += align256(static_cast<size_t>(m->E) * MLP_IN * 2) + align256(static_cast<size_t>(sensor_tiles(m))) +
         align256(static_cast<size_t>(sensor_tiles(m)) * 16) + 256;
  if (prm->sensor == CVW_SENSOR_LEARNED || (m->cell == CVW_QUAD && m->space == CVW_DG) || m->cell == CVW_HEX ||
      m->cell == CVW_TET)
    b += align256(static_cast<size_t>(m->E) * 4);
  if (op == 1) b += 2 * align256(state_elems(m, n_var(m, prm->flux)) * es);
  if (op == 2)    // limiter: vertex candidates of every variable, gamma, the selected cells and their count
    b += align256(static_cast<size_t>(n_var(m, prm->flux)) * m->nk * m->Nv * es) +
         2 * align256(static_cast<size_t>(m->E) * 4) + 256 + align256(static_cast<size_t>(m->Nv)) +
         align256(static_cast<size_t>(m->Nv) * 4);
  return b;
}

static cvw_status check_common(const cvw_mesh* m, const cvw_params* prm, size_t ws_bytes, int op, void* ws) {
  if (!m || !prm) { set_error("null argument"); return CVW_EINVAL; }
  if (!ws) { set_error("null workspace"); return CVW_EINVAL; }
  if (ws_bytes < cvw_workspace_bytes(m, prm, op)) { set_error("workspace too small"); return CVW_EINVAL; }
  if (reinterpret_cast<uintptr_t>(ws) % 256) { set_error("workspace must be 256-byte aligned"); return CVW_EINVAL; }
  if (prm->flux < 0 || prm->flux > CVW_EULER) { set_error("unknown flux"); return CVW_EINVAL; }
  if (prm->sensor == CVW_SENSOR_LEARNED) {
    if (!(m->cell == CVW_QUAD && m->space == CVW_DG)) {
      set_error("learned sensor: DG quadrilaterals only"); return CVW_EUNSUPPORTED;
    }
    if (!prm->mlp || !(prm->sigma_ref > 0) || !std::isfinite(prm->sigma_ref)) {
      set_error("learned sensor needs a network and sigma_ref > 0"); return CVW_EINVAL;
    }
    if (prm->mlp->device != m->device) { set_error("network and mesh on different devices"); return CVW_EINVAL; }
    if (m->grid_nx <= 0) {
      set_error("learned sensor: structured periodic grids (its plain fallback is the fused pass)");
      return CVW_EUNSUPPORTED;
    }
    if (prm->audit_every < 0 || !(prm->audit_tol >= 0)) { set_error("bad audit parameters"); return CVW_EINVAL; }
  } else if (prm->sensor != CVW_SENSOR_PLAIN && prm->sensor != CVW_SENSOR_FIXED) {
    set_error("unknown sensor kind"); return CVW_EINVAL;
  }
  if (!(prm->eps_vertex > 0) || !(prm->eps_cell > 0) || prm->r < 1 || !(prm->q_sensor >= 1) || !(prm->q_beta >= 1) ||
      !(prm->lin_w_vertex > 0) || !(prm->lin_w_vertex * m->ve < 1)) {
    set_error("invalid method parameters"); return CVW_EINVAL;
  }
  const bool dgq = m->cell == CVW_QUAD && m->space == CVW_DG;
  const bool cgq = m->cell == CVW_QUAD && m->space == CVW_CG;
  const bool seg = m->cell == CVW_SEG;
  const bool dgt = m->cell == CVW_TRI && m->space == CVW_DG;
  if (m->cell == CVW_TET) {
    if (!m->d_tett) { set_error("DG tetrahedra: degree <= 2"); return CVW_EUNSUPPORTED; }
    if (!m->closed) { set_error("DG tetrahedra: meshes without boundary faces (periodic)"); return CVW_EUNSUPPORTED; }
    if (prm->dtype != CVW_F32) { set_error("DG tetrahedra run in float32"); return CVW_EUNSUPPORTED; }
    if (prm->flux != CVW_ADVECT_CONST && prm->flux != CVW_BURGERS && prm->flux != CVW_EULER) {
      set_error("DG tetrahedra: constant-velocity advection, Burgers and the Euler equations"); return CVW_EUNSUPPORTED;
    }
    return CVW_OK;
  }
  if (m->cell == CVW_HEX) {
    if (!m->closed) { set_error("DG hexahedra: meshes without boundary faces (periodic)"); return CVW_EUNSUPPORTED; }
    if (!m->uniform || !m->d_hext) {
      set_error("DG hexahedra: congruent axis-aligned boxes with one cell in each octant of every vertex, degree <= 2");
      return CVW_EUNSUPPORTED;
    }
    if (prm->dtype != CVW_F32) { set_error("DG hexahedra run in float32"); return CVW_EUNSUPPORTED; }
    if (prm->flux != CVW_ADVECT_CONST && prm->flux != CVW_BURGERS && prm->flux != CVW_EULER) {
      set_error("DG hexahedra: constant-velocity advection, Burgers and the Euler equations"); return CVW_EUNSUPPORTED;
    }
    return CVW_OK;
  }
  if (dgt) {
    if (m->degree > MAXP) { set_error("degree > 3 not on the GPU path"); return CVW_EUNSUPPORTED; }
    if (prm->dtype != CVW_F32) { set_error("DG triangles run in float32"); return CVW_EUNSUPPORTED; }
    if (!m->closed && !prm->bc_face_kind) {
      set_error("boundary faces need boundary data (cvw_params.bc_face_kind)"); return CVW_EINVAL;
    }
    return CVW_OK;
  }
  if (!dgq && !cgq && !seg) { set_error("this cell / space combination is not on the GPU path yet"); return CVW_EUNSUPPORTED; }
  if (seg) {
    if (prm->flux != CVW_ADVECT_CONST && prm->flux != CVW_BURGERS && prm->flux != CVW_EULER) {
      set_error("1D path: constant-velocity advection, Burgers and the Euler equations"); return CVW_EUNSUPPORTED;
    }
    if (seg_hp(m, prm) && prm->dtype != CVW_F64) {
      set_error("1D path: degrees above 3, the Euler equations and lines with ends run in float64");
      return CVW_EUNSUPPORTED;
    }
    if (m->open_ends > 0) {
      if (m->open_ends != 2) { set_error("a line has two ends"); return CVW_EINVAL; }
      for (int e = 0; e < 2; ++e) {
        const int b = prm->bc[e];
        if (b != CVW_BC_OUTFLOW && b != CVW_BC_WALL && b != CVW_BC_INFLOW) {
          set_error("a line with ends needs boundary data (outflow, wall or inflow) at both ends"); return CVW_EINVAL;
        }
        if (b == CVW_BC_WALL && prm->flux != CVW_EULER) {
          set_error("a reflecting wall needs the Euler equations"); return CVW_EINVAL;
        }
        if (b == CVW_BC_INFLOW) {
          const double* q = prm->bc_state[e];
          bool ok = std::isfinite(q[0]) && std::isfinite(q[1]) && std::isfinite(q[2]);
          if (prm->flux == CVW_EULER && ok) {
            const double pr = (prm->flux_param[0] - 1.0) * (q[2] - 0.5 * q[1] * q[1] / q[0]);
            ok = q[0] > 0.0 && pr > 0.0;
          }
          if (!ok) { set_error("inflow state not finite (or not of positive density and pressure)"); return CVW_EINVAL; }
        }
      }
    }
  }
  if (cgq) {
    if (m->degree > 2) { set_error("CG quadrilaterals: degree <= 2 on the GPU path"); return CVW_EUNSUPPORTED; }
    if (prm->dtype != CVW_F32) { set_error("CG quadrilaterals run in float32"); return CVW_EUNSUPPORTED; }
    if (prm->flux == CVW_EULER) { set_error("systems are not on the CG quadrilateral path"); return CVW_EUNSUPPORTED; }
  }
  if (dgq) {
    if (!m->uniform) { set_error("DG quadrilaterals: only congruent axis-aligned cells"); return CVW_EUNSUPPORTED; }
    if (m->degree > MAXP) { set_error("degree > 3 not on the GPU path"); return CVW_EUNSUPPORTED; }
    if (prm->dtype != CVW_F32) { set_error("DG quadrilaterals run in float32"); return CVW_EUNSUPPORTED; }
    if (prm->flux == CVW_ADVECT_ROT) { set_error("rotating velocity not on the DG quadrilateral path"); return CVW_EUNSUPPORTED; }
    if (!m->closed && !prm->bc_face_kind) {
      set_error("boundary faces need boundary data (cvw_params.bc_face_kind)"); return CVW_EINVAL;
    }
  }
  return CVW_OK;
}

struct WS {
  uint32_t* status;
  double* tot;                     // totals scratch
  void* cand;
  void* pg;
  void* rcell;
  void* rhs;                       // stage right-hand side (R)
  void* x, *r, *z, *p, *Ap;        // PCG vectors (CG)
  double* part;                    // PCG block partials, followed by its 8 scalars
  double* S;
  uint16_t* feat;                  // learned sensor: features [E][48], tile flags, audit partials and results
  uint8_t* tflag;
  double* apart;
  double* aout;
  float* gam;                      // DG quadrilaterals / learned sensor: gamma_e of the stage [E]
  void* st1;
  void* st2;
};
static WS carve(const cvw_mesh* m, const cvw_params* prm, void* ws) {
  const size_t es = prm->dtype == CVW_F64 ? 8 : 4;
  char* p = static_cast<char*>(ws);
  WS w{};
  w.status = reinterpret_cast<uint32_t*>(p);
  p += 256;
  w.tot = reinterpret_cast<double*>(p);
  p += TOT_SCRATCH;
  if (!use_tile(m, prm)) {
    w.cand = p;
    p += align256(static_cast<size_t>(m->nk) * m->Nv * es);
  }
  if (m->space == CVW_CG) {
    w.pg = p;
    p += align256(pg_elems(m, prm) * es);
    w.rcell = p;
    p += align256(rcell_elems(m, prm) * es);
  }
  if (m->n_mass > 0) {
    w.rhs = p;
    p += align256(state_elems(m, n_var(m, prm->flux)) * es);
    if (m->space == CVW_CG) {
      void** vecs[5] = {&w.x, &w.r, &w.z, &w.p, &w.Ap};
      for (void** v : vecs) {
        *v = p;
        p += align256(state_elems(m, n_var(m, prm->flux)) * es);
      }
      w.part = reinterpret_cast<double*>(p);
      w.S = w.part + pcg_partials(m->ndof);
      p += align256((pcg_partials(m->ndof) + 8) * sizeof(double));
    }
  }
  if (prm->sensor == CVW_SENSOR_LEARNED) {
    w.feat = reinterpret_cast<uint16_t*>(p);
    p += align256(static_cast<size_t>(m->E) * MLP_IN * 2);
    w.tflag = reinterpret_cast<uint8_t*>(p);
    p += align256(static_cast<size_t>(sensor_tiles(m)));
    w.apart = reinterpret_cast<double*>(p);
    p += align256(static_cast<size_t>(sensor_tiles(m)) * 16);
    w.aout = reinterpret_cast<double*>(p);
    p += 256;
  }
  if (prm->sensor == CVW_SENSOR_LEARNED || (m->cell == CVW_QUAD && m->space == CVW_DG) || m->cell == CVW_HEX ||
      m->cell == CVW_TET) {
    w.gam = reinterpret_cast<float*>(p);
    p += align256(static_cast<size_t>(m->E) * 4);
  }
  w.st1 = p;
  p += align256(state_elems(m, n_var(m, prm->flux)) * es);
  w.st2 = p;
  return w;
}

// the gamma the two-pass cell pass takes as given: the learned sensor's (in
// the workspace), else none (the cell pass runs the plain sensor itself)
static const float* learned_gamma_of(const cvw_params* prm, const WS& w) {
  return prm->sensor == CVW_SENSOR_LEARNED ? w.gam : nullptr;
}

// learned sensor: features of u, then the network, guarded: cells outside
// the network's feature box, with a non-finite output, or all cells once an
// audit has set the latch, are handed to the plain sensor (the fused pass
// over the flagged tiles only); gamma in the workspace
static cvw_status learned_gamma(const cvw_mesh* m, const cvw_params* prm, const void* u, const void* cand, const WS& w,
                                hipStream_t s, float* gamma = nullptr) {
  float* g = gamma ? gamma : w.gam;      // the caller's array, else the workspace's
  cvw_status st = dgquad_features(m, static_cast<const float*>(u), static_cast<const float*>(cand), prm->sigma_ref,
                                  w.feat, s);
  if (st != CVW_OK) return st;
  const MlpGuard G{prm->mlp->lo, prm->mlp->hi, w.status, w.tflag, m->grid_nx, (m->grid_nx + 15) / 16};
  if ((st = mlp_infer(prm->mlp->dev(), w.feat, m->E, g, s, &G)) != CVW_OK) return st;
  return dgquad_sensor_tile(m, prm, static_cast<const float*>(u), g, s, TILE_FALLBACK, w.tflag);
}

// audit of the learned sensor on state u: learned gamma (guarded) in the
// workspace, the plain gamma of every cell against it; the mean deviation
// above prm->audit_tol sets the latch (device side, no host synchronisation)
static cvw_status learned_audit(const cvw_mesh* m, const cvw_params* prm, const void* u, const WS& w, hipStream_t s) {
  cvw_status st = dgquad_candidates(m, prm, static_cast<const float*>(u), static_cast<float*>(w.cand), s);
  if (st != CVW_OK || (st = learned_gamma(m, prm, u, w.cand, w, s)) != CVW_OK) return st;
  if ((st = dgquad_sensor_tile(m, prm, static_cast<const float*>(u), nullptr, s, TILE_AUDIT, nullptr, w.gam,
                               w.apart)) != CVW_OK)
    return st;
  return dgquad_audit_finalize(m, w.apart, prm->audit_tol, w.status, w.aout, s);
}

static cvw_status candidates_any(const cvw_mesh* m, const cvw_params* prm, const void* u, void* cand,
                                 hipStream_t s) {
  if (m->cell == CVW_SEG) return seg_candidates(m, prm, u, cand, s);
  if (m->cell == CVW_HEX)
    return hex_candidates(m, prm, static_cast<const float*>(u), static_cast<float*>(cand), s);
  if (m->cell == CVW_TET)
    return tet_candidates(m, prm, static_cast<const float*>(u), static_cast<float*>(cand), s);
  if (m->cell == CVW_TRI)
    return tri_candidates(m, prm, static_cast<const float*>(u), static_cast<float*>(cand), s);
  if (m->space == CVW_CG)
    return cgquad_candidates(m, prm, static_cast<const float*>(u), static_cast<float*>(cand), s);
  return dgquad_candidates(m, prm, static_cast<const float*>(u), static_cast<float*>(cand), s);
}

cvw_status cvw_vertex_candidates(const cvw_mesh* m, const cvw_params* prm, const void* u, void* cand, void* ws,
                                 size_t ws_bytes, void* stream) {
  cvw_status st = check_common(m, prm, ws_bytes, 0, ws);
  if (st != CVW_OK) return st;
  if (!u || !cand) { set_error("null device pointer"); return CVW_EINVAL; }
  return candidates_any(m, prm, u, cand, static_cast<hipStream_t>(stream));
}

cvw_status cvw_sensor(const cvw_mesh* m, const cvw_params* prm, const void* u, void* gamma, void* alpha, void* ws,
                      size_t ws_bytes, void* stream) {
  cvw_status st = check_common(m, prm, ws_bytes, 0, ws);
  if (st != CVW_OK) return st;
  if (!u || !gamma) { set_error("null device pointer"); return CVW_EINVAL; }
  const WS w = carve(m, prm, ws);
  auto s = static_cast<hipStream_t>(stream);
  if (use_tile(m, prm)) {
    // fused pass; the shock-capturing weights, when asked for, from the cell pass with that gamma
    st = dgquad_sensor_tile(m, prm, static_cast<const float*>(u), static_cast<float*>(gamma), s);
    if (st != CVW_OK || !alpha) return st;
    return dgquad_eval(m, prm, MODE_SENSOR, static_cast<const float*>(u), nullptr, nullptr, static_cast<float*>(gamma),
                       static_cast<float*>(alpha), nullptr, w.status, 0.f, 0.f, 0.f, s,
                       static_cast<const float*>(gamma));
  }
  if (prm->sensor != CVW_SENSOR_FIXED) {
    st = candidates_any(m, prm, u, w.cand, s);
    if (st != CVW_OK) return st;
  }
  if (prm->sensor == CVW_SENSOR_LEARNED) {
    // the network (with its plain fallback) writes gamma; the cell pass only
    // when the shock-capturing weights are asked for
    if ((st = learned_gamma(m, prm, u, w.cand, w, s, static_cast<float*>(gamma))) != CVW_OK || !alpha) return st;
    return dgquad_eval(m, prm, MODE_SENSOR, static_cast<const float*>(u), nullptr, nullptr, static_cast<float*>(gamma),
                       static_cast<float*>(alpha), nullptr, w.status, 0.f, 0.f, 0.f, s,
                       static_cast<const float*>(gamma));
  }
  if (m->cell == CVW_SEG)
    return seg_eval(m, prm, MODE_SENSOR, u, w.cand, w.pg, w.rcell, nullptr, gamma, alpha, w.status, s);
  if (m->cell == CVW_TET)
    return tet_eval(m, prm, MODE_SENSOR, static_cast<const float*>(u), nullptr, nullptr, static_cast<float*>(gamma),
                    static_cast<float*>(alpha), static_cast<const float*>(w.cand), w.gam, w.status, 0.f, 0.f, 0.f, s);
  if (m->cell == CVW_HEX)
    return hex_eval(m, prm, MODE_SENSOR, static_cast<const float*>(u), nullptr, nullptr, static_cast<float*>(gamma),
                    static_cast<float*>(alpha), static_cast<const float*>(w.cand), w.gam, w.status, 0.f, 0.f, 0.f, s);
  if (m->cell == CVW_TRI)
    return tri_eval(m, prm, MODE_SENSOR, static_cast<const float*>(u), nullptr, nullptr, static_cast<float*>(gamma),
                    static_cast<float*>(alpha), static_cast<const float*>(w.cand), w.status, 0.f, 0.f, 0.f, s);
  if (m->space == CVW_CG)
    return cgquad_eval(m, prm, MODE_SENSOR, static_cast<const float*>(u), static_cast<const float*>(w.cand),
                       static_cast<float*>(w.pg), static_cast<float*>(w.rcell), nullptr, static_cast<float*>(gamma),
                       static_cast<float*>(alpha), w.status, s);
  return dgquad_eval(m, prm, MODE_SENSOR, static_cast<const float*>(u), nullptr, nullptr, static_cast<float*>(gamma),
                     static_cast<float*>(alpha), static_cast<const float*>(w.cand), w.status, 0.f, 0.f, 0.f, s,
                     learned_gamma_of(prm, w));
}

cvw_status cvw_limit(const cvw_mesh* m, const cvw_params* prm, const void* u, void* u_out, double threshold,
                     void* gamma_out, void* ws, size_t ws_bytes, void* stream) {
  cvw_status st = check_common(m, prm, ws_bytes, 2, ws);
  if (st != CVW_OK) return st;
  const bool tri = m->cell == CVW_TRI && m->space == CVW_DG;
  if (!(m->cell == CVW_QUAD && m->space == CVW_DG) && !tri) {
    set_error("HWENO limiter: DG quadrilaterals and triangles only"); return CVW_EUNSUPPORTED;
  }
  if (prm->sensor == CVW_SENSOR_LEARNED) {
    set_error("HWENO limiter: plain or fixed sensor"); return CVW_EUNSUPPORTED;
  }
  if (!u || !u_out) { set_error("null device pointer"); return CVW_EINVAL; }
  if (std::isnan(threshold)) { set_error("threshold is NaN"); return CVW_EINVAL; }
  const int nv = n_var(m, prm->flux);
  {
    // u_out is u or a separate array: a partial overlap would be read after written
    const uintptr_t a = reinterpret_cast<uintptr_t>(u), b = reinterpret_cast<uintptr_t>(u_out);
    const uintptr_t n = static_cast<uintptr_t>(m->E) * m->nloc * nv * sizeof(float);
    if (a != b && a < b + n && b < a + n) { set_error("u_out overlaps u without being u"); return CVW_EINVAL; }
  }
  const WS w = carve(m, prm, ws);
  auto s = static_cast<hipStream_t>(stream);
  char* lp = static_cast<char*>(w.st1);
  float* cand = reinterpret_cast<float*>(lp);
  lp += align256(static_cast<size_t>(nv) * m->nk * m->Nv * 4);
  float* gam = gamma_out ? static_cast<float*>(gamma_out) : reinterpret_cast<float*>(lp);
  lp += align256(static_cast<size_t>(m->E) * 4);
  int32_t* list = reinterpret_cast<int32_t*>(lp);
  lp += align256(static_cast<size_t>(m->E) * 4);
  uint32_t* count = reinterpret_cast<uint32_t*>(lp);
  lp += 256;
  uint8_t* vflag = reinterpret_cast<uint8_t*>(lp);
  lp += align256(static_cast<size_t>(m->Nv));
  int32_t* vlist = reinterpret_cast<int32_t*>(lp);
  const float* uf = static_cast<const float*>(u);
  if (tri) {
    // every variable's vertex candidates, the sensor values, the selection
    for (int v = 0; v < nv; ++v)
      if ((st = tri_candidates(m, prm, uf + static_cast<int64_t>(v) * m->E * m->nloc,
                               cand + static_cast<int64_t>(v) * m->Nv * m->nk, s)) != CVW_OK)
        return st;
    if ((st = tri_eval(m, prm, MODE_SENSOR, uf, nullptr, nullptr, gam, nullptr, cand, w.status, 0.f, 0.f, 0.f, s)) !=
        CVW_OK)
      return st;
    const bool all = threshold > 1.0 && (prm->sensor != CVW_SENSOR_FIXED || prm->fixed_gamma < threshold);
    if (!all) {
      if (u_out != u &&
          hipMemcpyAsync(u_out, u, static_cast<size_t>(m->E) * m->nloc * nv * sizeof(float), hipMemcpyDeviceToDevice,
                         s) != hipSuccess) {
        set_error("state copy failed"); return CVW_EDEVICE;
      }
      if ((st = limit_select(gam, m->E, threshold, count, list, s)) != CVW_OK) return st;
    }
    return tri_limit(m, prm, uf, static_cast<float*>(u_out), cand, count, all ? nullptr : list, s);
  }
  // the sensor field's vertex candidates (the other variables' follow inside
  // the limiter, where they are needed; every candidate is taken from the
  // state before the reconstruction writes, so u_out may be u)
  if ((st = dgquad_candidates(m, prm, uf, cand, s)) != CVW_OK) return st;
  // sensor values of the sensor field (variable 0): the fused pass where it
  // applies (the values of cvw_sensor), else the cell pass on the candidates
  if (use_tile(m, prm)) {
    if ((st = dgquad_sensor_tile(m, prm, uf, gam, s)) != CVW_OK) return st;
  } else if ((st = dgquad_eval(m, prm, MODE_SENSOR, uf, nullptr, nullptr, gam, nullptr, cand, w.status, 0.f, 0.f,
                               0.f, s)) != CVW_OK) {
    return st;
  }
  LimitNodes ln{};
  std::vector<double> x, wq;
  gauss_rule(m->degree + 1, x, wq);
  for (int i = 0; i <= m->degree; ++i) {
    ln.xi[i] = x[i];
    ln.w[i] = wq[i];
  }
  return dgquad_limit(m, prm, uf, static_cast<float*>(u_out), cand, gam, ln, threshold, count, list, vflag, vlist,
                      s);
}

cvw_status cvw_positivity(const cvw_mesh* m, const cvw_params* prm, const void* u, void* u_out, double eps0,
                          void* ws, size_t ws_bytes, void* stream) {
  if (!m || !prm) { set_error("null argument"); return CVW_EINVAL; }
  if (!ws) { set_error("null workspace"); return CVW_EINVAL; }
  if (ws_bytes < cvw_workspace_bytes(m, prm, 3)) { set_error("workspace too small"); return CVW_EINVAL; }
  if (reinterpret_cast<uintptr_t>(ws) % 256) { set_error("workspace must be 256-byte aligned"); return CVW_EINVAL; }
  const bool tri = m->cell == CVW_TRI && m->space == CVW_DG && m->d_trit;
  if (!(m->cell == CVW_QUAD && m->space == CVW_DG && m->uniform) && !tri) {
    set_error("positivity limiter: DG quadrilaterals (congruent axis-aligned cells) and DG triangles only");
    return CVW_EUNSUPPORTED;
  }
  if (prm->flux != CVW_EULER) { set_error("positivity limiter: Euler equations only"); return CVW_EUNSUPPORTED; }
  if (prm->dtype != CVW_F32) { set_error("the positivity limiter runs in float32"); return CVW_EUNSUPPORTED; }
  if (m->degree < 1 || m->degree > MAXP) { set_error("degree not on the GPU path"); return CVW_EUNSUPPORTED; }
  const double gam = prm->flux_param[0];
  if (!(gam > 1.0) || !std::isfinite(gam)) { set_error("gamma must be > 1"); return CVW_EINVAL; }
  if (!(eps0 > 0.0) || !std::isfinite(eps0)) { set_error("eps0 must be positive and finite"); return CVW_EINVAL; }
  if (!u || !u_out) { set_error("null device pointer"); return CVW_EINVAL; }
  {
    const uintptr_t a = reinterpret_cast<uintptr_t>(u), b = reinterpret_cast<uintptr_t>(u_out);
    const uintptr_t n = static_cast<uintptr_t>(m->E) * m->nloc * 4 * sizeof(float);
    if (a != b && a < b + n && b < a + n) { set_error("u_out overlaps u without being u"); return CVW_EINVAL; }
  }
  if (tri)
    return tri_positivity(m, static_cast<const float*>(u), static_cast<float*>(u_out), gam, eps0,
                          static_cast<hipStream_t>(stream));
  LimitNodes ln{};
  std::vector<double> x, wq;
  gauss_rule(m->degree + 1, x, wq);
  for (int i = 0; i <= m->degree; ++i) {
    ln.xi[i] = x[i];
    ln.w[i] = wq[i];
  }
  uint32_t* count = static_cast<uint32_t*>(ws);
  int32_t* list = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + 256);
  return dgquad_positivity(m, static_cast<const float*>(u), static_cast<float*>(u_out), ln, gam, eps0, count, list,
                           static_cast<hipStream_t>(stream));
}

cvw_status cvw_residual(const cvw_mesh* m, const cvw_params* prm, const void* u, void* R, void* gamma_out, void* ws,
                        size_t ws_bytes, void* stream) {
  cvw_status st = check_common(m, prm, ws_bytes, 0, ws);
  if (st != CVW_OK) return st;
  if (!u || !R) { set_error("null device pointer"); return CVW_EINVAL; }
  if (u == R) { set_error("R must not alias u"); return CVW_EINVAL; }
  const WS w = carve(m, prm, ws);
  auto s = static_cast<hipStream_t>(stream);
  if (use_tile(m, prm)) {
    st = dgquad_sensor_tile(m, prm, static_cast<const float*>(u), w.gam, s);
    if (st != CVW_OK) return st;
    return dgquad_eval(m, prm, MODE_RESIDUAL, static_cast<const float*>(u), nullptr, static_cast<float*>(R),
                       static_cast<float*>(gamma_out), nullptr, nullptr, w.status, 0.f, 0.f, 0.f, s, w.gam);
  }
  if (prm->sensor != CVW_SENSOR_FIXED) {
    st = candidates_any(m, prm, u, w.cand, s);
    if (st != CVW_OK) return st;
  }
  if (prm->sensor == CVW_SENSOR_LEARNED && (st = learned_gamma(m, prm, u, w.cand, w, s)) != CVW_OK) return st;
  if (m->cell == CVW_SEG)
    return seg_eval(m, prm, MODE_RESIDUAL, u, w.cand, w.pg, w.rcell, R, gamma_out, nullptr, w.status, s);
  if (m->cell == CVW_TET)
    return tet_eval(m, prm, MODE_RESIDUAL, static_cast<const float*>(u), nullptr, static_cast<float*>(R),
                    static_cast<float*>(gamma_out), nullptr, static_cast<const float*>(w.cand), w.gam, w.status, 0.f,
                    0.f, 0.f, s);
  if (m->cell == CVW_HEX)
    return hex_eval(m, prm, MODE_RESIDUAL, static_cast<const float*>(u), nullptr, static_cast<float*>(R),
                    static_cast<float*>(gamma_out), nullptr, static_cast<const float*>(w.cand), w.gam, w.status, 0.f,
                    0.f, 0.f, s);
  if (m->cell == CVW_TRI)
    return tri_eval(m, prm, MODE_RESIDUAL, static_cast<const float*>(u), nullptr, static_cast<float*>(R),
                    static_cast<float*>(gamma_out), nullptr, static_cast<const float*>(w.cand), w.status, 0.f, 0.f,
                    0.f, s);
  if (m->space == CVW_CG)
    return cgquad_eval(m, prm, MODE_RESIDUAL, static_cast<const float*>(u), static_cast<const float*>(w.cand),
                       static_cast<float*>(w.pg), static_cast<float*>(w.rcell), static_cast<float*>(R),
                       static_cast<float*>(gamma_out), nullptr, w.status, s);
  return dgquad_eval(m, prm, MODE_RESIDUAL, static_cast<const float*>(u), nullptr, static_cast<float*>(R),
                     static_cast<float*>(gamma_out), nullptr, static_cast<const float*>(w.cand), w.status, 0.f, 0.f,
                     0.f, s, learned_gamma_of(prm, w));
}

}  // extern "C"

namespace {

// Mass-matrix tolerances of the PCG solve (relative, preconditioned norm) and
// its launch-time iteration cap; converged iterations are no-ops on the device.
constexpr double PCG_TOL_F32 = 2e-7, PCG_TOL_F64 = 1e-14;
constexpr int PCG_MAXIT_F32 = 64, PCG_MAXIT_F64 = 160;

template <typename Real>
cvw_status generic_stage(const cvw_mesh* m, const cvw_params* prm, const WS& w, const Real* us, const Real* cand,
                         const Real* un, Real* uo, double dt, double a0, double b0, hipStream_t s) {
  cvw_status st;
  Real* rhs = static_cast<Real*>(w.rhs);
  if (m->cell == CVW_SEG)
    st = seg_eval(m, prm, MODE_RESIDUAL, us, cand, w.pg, w.rcell, rhs, nullptr, nullptr, w.status, s);
  else
    st = cgquad_eval(m, prm, MODE_RESIDUAL, reinterpret_cast<const float*>(us), reinterpret_cast<const float*>(cand),
                     static_cast<float*>(w.pg), static_cast<float*>(w.rcell), reinterpret_cast<float*>(rhs), nullptr,
                     nullptr, w.status, s);
  if (st != CVW_OK) return st;
  const bool f64 = std::is_same<Real, double>::value;
  const Real* dinv = f64 ? reinterpret_cast<const Real*>(m->d_dinv_d) : reinterpret_cast<const Real*>(m->d_dinv_f);
  const int64_t n = static_cast<int64_t>(state_elems(m, n_var(m, prm->flux)));
  if (m->space == CVW_CG) {
    Real* x = static_cast<Real*>(w.x);
    st = cg_mass_solve<Real>(m, rhs, x, static_cast<Real*>(w.r), static_cast<Real*>(w.z), static_cast<Real*>(w.p),
                             static_cast<Real*>(w.Ap), static_cast<Real*>(w.rcell), w.part, w.S, dinv,
                             f64 ? PCG_TOL_F64 : PCG_TOL_F32, f64 ? PCG_MAXIT_F64 : PCG_MAXIT_F32, w.status, s,
                             n_var(m, prm->flux));
    if (st != CVW_OK) return st;
    return stage_update<Real>(us, un, x, nullptr, uo, a0, b0, dt, n, s);
  }
  return stage_update<Real>(us, un, rhs, dinv, uo, a0, b0, dt, n, s, m->n_mass);
}

cvw_status any_stage(const cvw_mesh* m, const cvw_params* prm, const WS& w, const void* us, const void* cand,
                     const void* un, void* uo, double dt, double a0, double b0, hipStream_t s) {
  if (m->cell == CVW_TET)
    return tet_eval(m, prm, MODE_STAGE, static_cast<const float*>(us), static_cast<const float*>(un),
                    static_cast<float*>(uo), nullptr, nullptr, static_cast<const float*>(cand), w.gam, w.status,
                    static_cast<float>(dt), static_cast<float>(a0), static_cast<float>(b0), s);
  if (m->cell == CVW_HEX)
    return hex_eval(m, prm, MODE_STAGE, static_cast<const float*>(us), static_cast<const float*>(un),
                    static_cast<float*>(uo), nullptr, nullptr, static_cast<const float*>(cand), w.gam, w.status,
                    static_cast<float>(dt), static_cast<float>(a0), static_cast<float>(b0), s);
  if (m->cell == CVW_TRI)
    return tri_eval(m, prm, MODE_STAGE, static_cast<const float*>(us), static_cast<const float*>(un),
                    static_cast<float*>(uo), nullptr, nullptr, static_cast<const float*>(cand), w.status,
                    static_cast<float>(dt), static_cast<float>(a0), static_cast<float>(b0), s);
  if (m->cell == CVW_QUAD && m->space == CVW_DG) {
    if (use_tile(m, prm)) {
      const cvw_status st = dgquad_sensor_tile(m, prm, static_cast<const float*>(us), w.gam, s);
      if (st != CVW_OK) return st;
      return dgquad_eval(m, prm, MODE_STAGE, static_cast<const float*>(us), static_cast<const float*>(un),
                         static_cast<float*>(uo), nullptr, nullptr, nullptr, w.status, static_cast<float>(dt),
                         static_cast<float>(a0), static_cast<float>(b0), s, w.gam);
    }
    if (prm->sensor == CVW_SENSOR_LEARNED) {
      const cvw_status st = learned_gamma(m, prm, us, cand, w, s);
      if (st != CVW_OK) return st;
    }
    return dgquad_eval(m, prm, MODE_STAGE, static_cast<const float*>(us), static_cast<const float*>(un),
                       static_cast<float*>(uo), nullptr, nullptr, static_cast<const float*>(cand), w.status,
                       static_cast<float>(dt), static_cast<float>(a0), static_cast<float>(b0), s,
                       learned_gamma_of(prm, w));
  }
  if (prm->dtype == CVW_F64)
    return generic_stage<double>(m, prm, w, static_cast<const double*>(us), static_cast<const double*>(cand),
                                 static_cast<const double*>(un), static_cast<double*>(uo), dt, a0, b0, s);
  return generic_stage<float>(m, prm, w, static_cast<const float*>(us), static_cast<const float*>(cand),
                              static_cast<const float*>(un), static_cast<float*>(uo), dt, a0, b0, s);
}

}  // namespace

extern "C" {

cvw_status cvw_rk_stage(const cvw_mesh* m, const cvw_params* prm, const void* u_stage, const void* cand,
                        const void* u_n, void* u_out, double dt, double a0, double b0, void* ws, size_t ws_bytes,
                        void* stream) {
  cvw_status st = check_common(m, prm, ws_bytes, 0, ws);
  if (st != CVW_OK) return st;
  if (!has_stage(m)) { set_error("no Runge-Kutta stage for this mesh (degree out of range)"); return CVW_EUNSUPPORTED; }
  if (!u_stage || (!cand && !use_tile(m, prm)) || !u_out || (a0 != 0.0 && !u_n)) {
    set_error("null device pointer"); return CVW_EINVAL;
  }
  if (u_out == u_stage || u_out == cand) { set_error("u_out must not alias u_stage or cand"); return CVW_EINVAL; }
  if (!std::isfinite(dt) || !std::isfinite(a0) || !std::isfinite(b0)) { set_error("non-finite stage coefficients"); return CVW_EINVAL; }
  const WS w = carve(m, prm, ws);
  return any_stage(m, prm, w, u_stage, cand, u_n, u_out, dt, a0, b0, static_cast<hipStream_t>(stream));
}

cvw_status cvw_rk_stage_gamma(const cvw_mesh* m, const cvw_params* prm, const void* u_stage, const void* gamma,
                              const void* u_n, void* u_out, double dt, double a0, double b0, void* ws,
                              size_t ws_bytes, void* stream) {
  cvw_status st = check_common(m, prm, ws_bytes, 0, ws);
  if (st != CVW_OK) return st;
  if (!(m->cell == CVW_QUAD && m->space == CVW_DG)) { set_error("a given gamma: DG quadrilaterals only"); return CVW_EUNSUPPORTED; }
  if (!u_stage || !gamma || !u_out || (a0 != 0.0 && !u_n)) { set_error("null device pointer"); return CVW_EINVAL; }
  if (u_out == u_stage || u_out == gamma) { set_error("u_out must not alias u_stage or gamma"); return CVW_EINVAL; }
  if (!std::isfinite(dt) || !std::isfinite(a0) || !std::isfinite(b0)) { set_error("non-finite stage coefficients"); return CVW_EINVAL; }
  const WS w = carve(m, prm, ws);
  return dgquad_eval(m, prm, MODE_STAGE, static_cast<const float*>(u_stage), static_cast<const float*>(u_n),
                     static_cast<float*>(u_out), nullptr, nullptr, nullptr, w.status, static_cast<float>(dt),
                     static_cast<float>(a0), static_cast<float>(b0), static_cast<hipStream_t>(stream),
                     static_cast<const float*>(gamma));
}

cvw_status cvw_step(const cvw_mesh* m, const cvw_params* prm, void* u, double dt, int n_steps, void* ws,
                    size_t ws_bytes, void* stream) {
  cvw_status st = check_common(m, prm, ws_bytes, 1, ws);
  if (st != CVW_OK) return st;
  if (!has_stage(m)) { set_error("no Runge-Kutta stage for this mesh (degree out of range)"); return CVW_EUNSUPPORTED; }
  if (!u) { set_error("null device pointer"); return CVW_EINVAL; }
  if (n_steps < 0 || !(dt > 0) || !std::isfinite(dt)) { set_error("bad dt or step count"); return CVW_EINVAL; }
  const WS w = carve(m, prm, ws);
  auto s = static_cast<hipStream_t>(stream);
  const bool f64 = prm->dtype == CVW_F64;
  // stage coefficients in the precision of the kernels (SSP-RK3, Shu-Osher form)
  const double third = f64 ? 1.0 / 3.0 : static_cast<double>(1.0f / 3.0f);
  const double two3 = f64 ? 2.0 / 3.0 : static_cast<double>(2.0f / 3.0f);
  const struct { const void* in; void* out; double a0, b0; } stages[3] = {
      {u, w.st1, 0.0, 1.0}, {w.st1, w.st2, 0.75, 0.25}, {w.st2, u, third, two3}};
  for (int n = 0; n < n_steps; ++n) {
    if (prm->sensor == CVW_SENSOR_LEARNED && prm->audit_every > 0 && n % prm->audit_every == 0 &&
        (st = learned_audit(m, prm, u, w, s)) != CVW_OK)
      return st;
    for (const auto& sg : stages) {
      if (prm->sensor != CVW_SENSOR_FIXED && !use_tile(m, prm)) {
        st = candidates_any(m, prm, sg.in, w.cand, s);
        if (st != CVW_OK) return st;
      }
      st = any_stage(m, prm, w, sg.in, w.cand, u, sg.out, dt, sg.a0, sg.b0, s);
      if (st != CVW_OK) return st;
    }
  }
  return CVW_OK;
}

cvw_status cvw_learned_audit(const cvw_mesh* m, const cvw_params* prm, const void* u, double* out_host, void* ws,
                             size_t ws_bytes, void* stream) {
  cvw_status st = check_common(m, prm, ws_bytes, 0, ws);
  if (st != CVW_OK) return st;
  if (prm->sensor != CVW_SENSOR_LEARNED) { set_error("audit: the learned sensor's parameters"); return CVW_EINVAL; }
  if (!u || !out_host) { set_error("null argument"); return CVW_EINVAL; }
  const WS w = carve(m, prm, ws);
  auto s = static_cast<hipStream_t>(stream);
  if ((st = learned_audit(m, prm, u, w, s)) != CVW_OK) return st;
  double r[2];
  uint32_t words[3];
  CVW_HIP(hipMemcpyAsync(r, w.aout, sizeof(r), hipMemcpyDeviceToHost, s));
  CVW_HIP(hipMemcpyAsync(words, w.status, sizeof(words), hipMemcpyDeviceToHost, s));
  CVW_HIP(hipStreamSynchronize(s));
  out_host[0] = r[0];
  out_host[1] = r[1];
  out_host[2] = static_cast<double>(words[WS_FALLBACK_COUNT]);
  out_host[3] = words[WS_LEARNED_OFF] ? 1.0 : 0.0;
  return CVW_OK;
}

cvw_status cvw_poll_status(const cvw_mesh* m, void* ws, size_t ws_bytes, uint32_t* flags, void* stream) {
  if (!m || !ws || !flags || ws_bytes < 256) { set_error("bad argument"); return CVW_EINVAL; }
  auto s = static_cast<hipStream_t>(stream);
  uint32_t h = 0;
  CVW_HIP(hipMemcpyAsync(&h, ws, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  CVW_HIP(hipStreamSynchronize(s));
  const uint32_t zero[2] = {0, 0};             // the status bits and the hand-over count; the latch stays
  CVW_HIP(hipMemcpyAsync(ws, zero, sizeof(zero), hipMemcpyHostToDevice, s));
  CVW_HIP(hipStreamSynchronize(s));
  *flags = h;
  return h ? CVW_ENUMERIC : CVW_OK;
}

cvw_status cvw_totals(const cvw_mesh* m, const cvw_params* prm, const void* u, double* out_host, void* ws,
                      size_t ws_bytes, void* stream) {
  cvw_status st = check_common(m, prm, ws_bytes, 0, ws);
  if (st != CVW_OK) return st;
  if (!u || !out_host) { set_error("null pointer"); return CVW_EINVAL; }
  if (m->space != CVW_DG || (m->cell != CVW_QUAD && m->cell != CVW_TRI)) {
    set_error("totals are implemented for DG quadrilaterals and triangles"); return CVW_EUNSUPPORTED;
  }
  const int nv = n_var(m, prm->flux);
  const WS w = carve(m, prm, ws);
  double* part = w.tot;
  double* res = part + 4 * 1024;
  auto s = static_cast<hipStream_t>(stream);
  st = m->cell == CVW_TRI ? tri_totals(m, nv, static_cast<const float*>(u), part, res, s)
                          : totals_f32(m, nv, static_cast<const float*>(u), part, res, s);
  if (st != CVW_OK) return st;
  CVW_HIP(hipMemcpyAsync(out_host, res, nv * sizeof(double), hipMemcpyDeviceToHost, s));
  CVW_HIP(hipStreamSynchronize(s));
  return CVW_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// batched stages over many meshes
// ---------------------------------------------------------------------------
struct cvw_batch {
  int n = 0;
  int device = 0;
  int external = 0;                               // device arrays in a caller buffer (cvw_batch_build_in)
  int grid = 0;                                   // blocks per launch (<= 0: one per item)
  std::vector<const cvw_mesh*> meshes;
  std::vector<cvw_params> prms;
  std::vector<void*> u;
  std::vector<double> dt;
  std::vector<size_t> off_cand, off_st1, off_st2, off_gam;   // off_gam 0: no fused sensor pass
  size_t ws_bytes = 0;
  // work lists: fused sensor pass and vertex pass per degree, cell pass per (degree, flux)
  struct List { int P = 0, flux = 0, n = 0; int2* d = nullptr; };
  std::vector<List> slists, vlists, elists;
  cvw::BatchInst* d_inst = nullptr;
  cvw::TensorTables* d_tabs = nullptr;            // [4], index = degree
  cvw::LaneRec* d_lanes = nullptr;                // [4][16]
  // captured graph
  void* graph_ws = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

static void batch_drop_graph(cvw_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_ws = nullptr;
}

static void batch_free(cvw_batch* b) {
  if (!b) return;
  batch_drop_graph(b);
  if (!b->external) {
    for (auto& l : b->slists) (void)hipFree(l.d);
    for (auto& l : b->vlists) (void)hipFree(l.d);
    for (auto& l : b->elists) (void)hipFree(l.d);
    (void)hipFree(b->d_inst);
    (void)hipFree(b->d_tabs);
    (void)hipFree(b->d_lanes);
  }
  delete b;
}

// one pass of every stage kernel on stream s (used eagerly and under capture)
static cvw_status batch_launch_stage(const cvw_batch* b, int stage, hipStream_t s) {
  for (const auto& l : b->slists) {
    const cvw_status st = batch_sensor_pass(l.P, b->d_inst, l.d, l.n, stage, b->grid > 0 ? b->grid : l.n, s);
    if (st != CVW_OK) return st;
  }
  for (const auto& l : b->vlists) {
    const cvw_status st = batch_vertex_pass(l.P, b->d_inst, l.d, l.n, b->d_tabs, stage,
                                            b->grid > 0 ? b->grid : l.n, s);
    if (st != CVW_OK) return st;
  }
  for (const auto& l : b->elists) {
    const cvw_status st = batch_eval_pass(l.P, l.flux, b->d_inst, l.d, l.n, b->d_tabs, b->d_lanes, stage,
                                          b->grid > 0 ? b->grid : l.n, s);
    if (st != CVW_OK) return st;
  }
  return CVW_OK;
}

static cvw_status batch_upload_descriptors(cvw_batch* b, void* ws) {
  std::vector<BatchInst> h(b->n);
  char* base = static_cast<char*>(ws);
  for (int i = 0; i < b->n; ++i) {
    const cvw_mesh* m = b->meshes[i];
    BatchInst& I = h[i];
    std::memset(&I, 0, sizeof(I));
    float* u = static_cast<float*>(b->u[i]);
    float* s1 = reinterpret_cast<float*>(base + b->off_st1[i]);
    float* s2 = reinterpret_cast<float*>(base + b->off_st2[i]);
    I.u_in[0] = u;  I.u_out[0] = s1;
    I.u_in[1] = s1; I.u_out[1] = s2;
    I.u_in[2] = s2; I.u_out[2] = u;
    I.u = u;
    I.cand = b->off_cand[i] ? reinterpret_cast<float*>(base + b->off_cand[i]) : nullptr;
    I.cell_vtx = m->d_cell_vtx;
    I.nbr = m->d_nbr;
    I.vptr = m->d_vtx_ptr;
    I.vent = m->d_vtx_ent;
    I.E = m->E;
    I.Nv = m->Nv;
    I.vt = make_vertex_tables(m->tens, m->hx, m->hy, m->he, m->degree);
    I.g = make_cell_geo(m->hx, m->hy, m->he, m->degree);
    I.dt = static_cast<float>(b->dt[i]);
    I.P = m->degree;
    I.flux = b->prms[i].flux;
    I.status = reinterpret_cast<uint32_t*>(base);
    I.ms = make_scalars(&b->prms[i]);
    I.gam = b->off_gam[i] ? reinterpret_cast<float*>(base + b->off_gam[i]) : nullptr;
    if (I.gam) I.sa = make_sensor_tile_args(m);
  }
  CVW_HIP(hipMemcpy(b->d_inst, h.data(), h.size() * sizeof(BatchInst), hipMemcpyHostToDevice));
  return CVW_OK;
}

extern "C" {

cvw_status cvw_batch_build(const cvw_batch_instance* inst, int n, cvw_batch** out) {
  if (!inst || !out || n <= 0) { set_error("bad argument"); return CVW_EINVAL; }
  *out = nullptr;
  auto* b = new cvw_batch();
  b->n = n;
  b->external = g_arena != nullptr;
  (void)hipGetDevice(&b->device);
  size_t off = 256;
  struct Item { double cost; int inst, blk; };
  std::vector<Item> sitems[MAXP + 1], vitems[MAXP + 1];
  std::vector<Item> eitems[MAXP + 1][CVW_EULER + 1];
  for (int i = 0; i < n; ++i) {
    const cvw_mesh* m = inst[i].mesh;
    const cvw_params* prm = &inst[i].params;
    if (!m || !inst[i].u) { batch_free(b); set_error("null mesh or state"); return CVW_EINVAL; }
    if (m->device != b->device) { batch_free(b); set_error("instances on different devices"); return CVW_EINVAL; }
    if (m->cell != CVW_QUAD || m->space != CVW_DG || !m->uniform || !m->closed || m->degree > MAXP) {
      batch_free(b); set_error("batched stages: DG on congruent axis-aligned periodic quadrilaterals, p <= 3");
      return CVW_EUNSUPPORTED;
    }
    if (prm->dtype != CVW_F32) { batch_free(b); set_error("batched stages run in float32"); return CVW_EUNSUPPORTED; }
    if (prm->flux != CVW_ADVECT_CONST && prm->flux != CVW_BURGERS && prm->flux != CVW_KPP) {
      batch_free(b); set_error("batched stages: scalar fluxes (constant advection, Burgers, KPP)");
      return CVW_EUNSUPPORTED;
    }
    if (prm->sensor != CVW_SENSOR_PLAIN && prm->sensor != CVW_SENSOR_FIXED) {
      batch_free(b); set_error("batched stages: plain or fixed sensor"); return CVW_EUNSUPPORTED;
    }
    if (!(inst[i].dt > 0) || !std::isfinite(inst[i].dt)) { batch_free(b); set_error("bad dt"); return CVW_EINVAL; }
    b->meshes.push_back(m);
    b->prms.push_back(*prm);
    b->u.push_back(inst[i].u);
    b->dt.push_back(inst[i].dt);
    // the plain sensor on a structured periodic grid takes the fused pass
    // (gamma of the stage in the workspace), like a single instance's stage;
    // otherwise the vertex candidates go through the workspace
    const bool tile = use_tile(m, prm);
    b->off_cand.push_back(tile ? 0 : off);
    if (!tile) off += align256(static_cast<size_t>(m->Nv) * m->nk * 4);
    b->off_gam.push_back(tile ? off : 0);
    if (tile) off += align256(static_cast<size_t>(m->E) * 4);
    b->off_st1.push_back(off);
    off += align256(static_cast<size_t>(m->E) * m->nloc * 4);
    b->off_st2.push_back(off);
    off += align256(static_cast<size_t>(m->E) * m->nloc * 4);
    // estimated cost of a block: proportional to the nodes per cell
    const double c = static_cast<double>(m->nloc);
    const int cpt = cells_per_tile(m->degree);
    const int neb = static_cast<int>((m->E + cpt - 1) / cpt);
    if (tile) {
      for (int64_t k = 0; k < sensor_tiles(m); ++k) sitems[m->degree].push_back({c, i, static_cast<int>(k)});
    } else if (prm->sensor != CVW_SENSOR_FIXED) {
      const int nvb = static_cast<int>((m->Nv + VTX_PER_BLOCK - 1) / VTX_PER_BLOCK);
      for (int k = 0; k < nvb; ++k) vitems[m->degree].push_back({c, i, k});
    }
    for (int k = 0; k < neb; ++k) eitems[m->degree][prm->flux].push_back({c, i, k});
  }
  b->ws_bytes = off;
  // longest items first (ties: instance, block), each list uploaded once
  auto upload_list = [&](std::vector<Item>& v, int P, int flux, std::vector<cvw_batch::List>& dst) -> cvw_status {
    if (v.empty()) return CVW_OK;
    std::stable_sort(v.begin(), v.end(), [](const Item& x, const Item& y) { return x.cost > y.cost; });
    std::vector<int2> h(v.size());
    for (size_t k = 0; k < v.size(); ++k) h[k] = make_int2(v[k].inst, v[k].blk);
    cvw_batch::List l;
    l.P = P;
    l.flux = flux;
    l.n = static_cast<int>(h.size());
    const cvw_status st = upload(&l.d, h);
    if (st != CVW_OK) return st;
    dst.push_back(l);
    return CVW_OK;
  };
  cvw_status st;
  for (int P = MAXP; P >= 1; --P) {
    if ((st = upload_list(sitems[P], P, 0, b->slists)) != CVW_OK) { batch_free(b); return st; }
    if ((st = upload_list(vitems[P], P, 0, b->vlists)) != CVW_OK) { batch_free(b); return st; }
    for (int f = 0; f <= CVW_EULER; ++f)
      if ((st = upload_list(eitems[P][f], P, f, b->elists)) != CVW_OK) { batch_free(b); return st; }
  }
  std::vector<TensorTables> tabs(MAXP + 1);
  std::vector<LaneRec> lanes(16 * (MAXP + 1));
  for (int P = 1; P <= MAXP; ++P) {
    fill_tensor_tables(tabs[P], P, false);
    fill_lane_tables(lanes.data() + 16 * P, tabs[P], P);
  }
  if ((st = upload(&b->d_tabs, tabs)) != CVW_OK) { batch_free(b); return st; }
  if ((st = upload(&b->d_lanes, lanes)) != CVW_OK) { batch_free(b); return st; }
  {
    void* p = nullptr;
    if ((st = dev_alloc(&p, n * sizeof(BatchInst))) != CVW_OK) { batch_free(b); return st; }
    b->d_inst = static_cast<BatchInst*>(p);
  }
  *out = b;
  return CVW_OK;
}

cvw_status cvw_batch_plan(const cvw_batch_instance* inst, int n, size_t* device_bytes) {
  if (!device_bytes) { set_error("null argument"); return CVW_EINVAL; }
  MeshArena A;
  A.count_only = true;
  g_arena = &A;
  cvw_batch* b = nullptr;
  const cvw_status st = cvw_batch_build(inst, n, &b);
  g_arena = nullptr;
  if (st != CVW_OK) return st;
  batch_free(b);
  *device_bytes = (A.off + 255) / 256 * 256;
  return CVW_OK;
}

cvw_status cvw_batch_build_in(const cvw_batch_instance* inst, int n, void* device_buffer, size_t bytes,
                              cvw_batch** out) {
  if (!device_buffer || !out) { set_error("null argument"); return CVW_EINVAL; }
  if (reinterpret_cast<uintptr_t>(device_buffer) % 256) { set_error("device buffer must be 256-byte aligned"); return CVW_EINVAL; }
  MeshArena A;
  A.base = static_cast<char*>(device_buffer);
  A.size = bytes;
  g_arena = &A;
  const cvw_status st = cvw_batch_build(inst, n, out);
  g_arena = nullptr;
  return st;
}

void cvw_batch_destroy(cvw_batch* batch) { batch_free(batch); }

size_t cvw_batch_workspace_bytes(const cvw_batch* batch) { return batch ? batch->ws_bytes : 0; }

cvw_status cvw_batch_set_grid(cvw_batch* batch, int blocks) {
  if (!batch) { set_error("null batch"); return CVW_EINVAL; }
  batch->grid = blocks;
  batch_drop_graph(batch);
  return CVW_OK;
}

cvw_status cvw_batch_step(cvw_batch* b, int n_steps, int use_graph, void* ws, size_t ws_bytes, void* stream) {
  if (!b || !ws) { set_error("null argument"); return CVW_EINVAL; }
  if (ws_bytes < b->ws_bytes) { set_error("workspace too small"); return CVW_EINVAL; }
  if (reinterpret_cast<uintptr_t>(ws) % 256) { set_error("workspace must be 256-byte aligned"); return CVW_EINVAL; }
  if (n_steps < 0) { set_error("negative step count"); return CVW_EINVAL; }
  auto s = static_cast<hipStream_t>(stream);
  cvw_status st = CVW_OK;
  if (ws != b->graph_ws) {
    // descriptors point into this workspace; written before any launch that reads them
    CVW_HIP(hipStreamSynchronize(s));
    batch_drop_graph(b);
    if ((st = batch_upload_descriptors(b, ws)) != CVW_OK) return st;
    b->graph_ws = ws;
  }
  if (!use_graph) {
    for (int k = 0; k < n_steps; ++k)
      for (int stage = 0; stage < 3; ++stage)
        if ((st = batch_launch_stage(b, stage, s)) != CVW_OK) return st;
    return CVW_OK;
  }
  if (!b->exec) {
    hipStream_t cap;
    CVW_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    CVW_HIP(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal));
    for (int stage = 0; stage < 3 && st == CVW_OK; ++stage) st = batch_launch_stage(b, stage, cap);
    hipGraph_t g = nullptr;
    const hipError_t e1 = hipStreamEndCapture(cap, &g);
    (void)hipStreamDestroy(cap);
    if (st != CVW_OK) { if (g) (void)hipGraphDestroy(g); return st; }
    if (e1 != hipSuccess || !g) { set_error("graph capture failed"); return CVW_EDEVICE; }
    hipGraphExec_t ex = nullptr;
    if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) != hipSuccess) {
      (void)hipGraphDestroy(g);
      set_error("graph instantiation failed");
      return CVW_EDEVICE;
    }
    b->graph = g;
    b->exec = ex;
  }
  for (int k = 0; k < n_steps; ++k) CVW_HIP(hipGraphLaunch(b->exec, s));
  return CVW_OK;
}

cvw_status cvw_batch_poll_status(void* ws, size_t ws_bytes, uint32_t* flags, void* stream) {
  if (!ws || !flags || ws_bytes < 256) { set_error("bad argument"); return CVW_EINVAL; }
  auto s = static_cast<hipStream_t>(stream);
  uint32_t h = 0;
  CVW_HIP(hipMemcpyAsync(&h, ws, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  CVW_HIP(hipStreamSynchronize(s));
  const uint32_t zero = 0;
  CVW_HIP(hipMemcpyAsync(ws, &zero, sizeof(uint32_t), hipMemcpyHostToDevice, s));
  CVW_HIP(hipStreamSynchronize(s));
  *flags = h;
  return h ? CVW_ENUMERIC : CVW_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// learned-sensor network
// ---------------------------------------------------------------------------
namespace {

constexpr size_t MLP_BF16 = static_cast<size_t>(MLP_IN) * MLP_HID + 2 * MLP_HID * MLP_HID + MLP_HID;

cvw_status mlp_refresh(cvw_mlp* m, hipStream_t s) {
  // compute copies from the master weights (no gradient, no update)
  return mlp_update(nullptr, 0, m->master, m->m1, m->m2, 0.0f, 0.9, 0.999, 1e-8f, 1.0, 1.0, nullptr, m->mut(), s);
}

bool finite_params(const float* p) {
  for (int i = 0; i < MLP_NPARAM; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

extern "C" {

size_t cvw_mlp_device_bytes(void) {
  const size_t nf = 3 * static_cast<size_t>(MLP_NPARAM) + 2 * MLP_HID + 1;
  return align256(nf * 4) + align256(MLP_BF16 * 2) + align256(2 * MLP_IN * 4);
}

static cvw_status mlp_create_at(const float* params, void* buf, cvw_mlp** out) {
  if (!params || !out) { set_error("null argument"); return CVW_EINVAL; }
  *out = nullptr;
  if (!finite_params(params)) { set_error("non-finite network parameters"); return CVW_EINVAL; }
  auto* m = new cvw_mlp();
  (void)hipGetDevice(&m->device);
  const size_t nf = 3 * static_cast<size_t>(MLP_NPARAM) + 2 * MLP_HID + 1;
  const size_t bytes = cvw_mlp_device_bytes();
  if (buf) {
    m->mem = buf;
    m->external = 1;
  } else if (hipMalloc(&m->mem, bytes) != hipSuccess) {
    delete m; set_error("hipMalloc failed"); return CVW_ENOMEM;
  }
  float* f = static_cast<float*>(m->mem);
  m->master = f;
  m->m1 = f + MLP_NPARAM;
  m->m2 = f + 2 * MLP_NPARAM;
  m->b1 = f + 3 * MLP_NPARAM;
  m->b2 = m->b1 + MLP_HID;
  m->b3 = m->b2 + MLP_HID;
  uint16_t* h = reinterpret_cast<uint16_t*>(static_cast<char*>(m->mem) + align256(nf * 4));
  m->W1t = h;
  m->W2t = m->W1t + MLP_IN * MLP_HID;
  m->W2r = m->W2t + MLP_HID * MLP_HID;
  m->w3 = m->W2r + MLP_HID * MLP_HID;
  m->lo = reinterpret_cast<float*>(static_cast<char*>(m->mem) + align256(nf * 4) + align256(MLP_BF16 * 2));
  m->hi = m->lo + MLP_IN;
  std::vector<float> box(2 * MLP_IN);
  for (int i = 0; i < MLP_IN; ++i) {
    box[i] = -INFINITY;
    box[MLP_IN + i] = INFINITY;
  }
  if (hipMemset(m->mem, 0, bytes) != hipSuccess ||
      hipMemcpy(m->lo, box.data(), box.size() * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(m->master, params, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      mlp_refresh(m, nullptr) != CVW_OK || hipDeviceSynchronize() != hipSuccess) {
    if (!m->external) (void)hipFree(m->mem);
    delete m;
    set_error("network upload failed");
    return CVW_EDEVICE;
  }
  *out = m;
  return CVW_OK;
}

cvw_status cvw_mlp_create(const float* params, cvw_mlp** out) { return mlp_create_at(params, nullptr, out); }

cvw_status cvw_mlp_create_in(const float* params, void* device_buffer, size_t bytes, cvw_mlp** out) {
  if (!device_buffer) { set_error("null device buffer"); return CVW_EINVAL; }
  if (reinterpret_cast<uintptr_t>(device_buffer) % 256) { set_error("device buffer must be 256-byte aligned"); return CVW_EINVAL; }
  if (bytes < cvw_mlp_device_bytes()) { set_error("device buffer too small for the network (cvw_mlp_device_bytes)"); return CVW_EINVAL; }
  return mlp_create_at(params, device_buffer, out);
}

void cvw_mlp_destroy(cvw_mlp* mlp) {
  if (!mlp) return;
  if (!mlp->external) (void)hipFree(mlp->mem);
  delete mlp;
}

cvw_status cvw_mlp_get_params(const cvw_mlp* mlp, float* params) {
  if (!mlp || !params) { set_error("null argument"); return CVW_EINVAL; }
  CVW_HIP(hipDeviceSynchronize());
  CVW_HIP(hipMemcpy(params, mlp->master, MLP_NPARAM * sizeof(float), hipMemcpyDeviceToHost));
  return CVW_OK;
}

cvw_status cvw_mlp_set_params(cvw_mlp* mlp, const float* params) {
  if (!mlp || !params) { set_error("null argument"); return CVW_EINVAL; }
  if (!finite_params(params)) { set_error("non-finite network parameters"); return CVW_EINVAL; }
  CVW_HIP(hipDeviceSynchronize());
  CVW_HIP(hipMemcpy(mlp->master, params, MLP_NPARAM * sizeof(float), hipMemcpyHostToDevice));
  CVW_HIP(hipMemset(mlp->m1, 0, 2 * MLP_NPARAM * sizeof(float)));
  mlp->steps = 0;
  const cvw_status st = mlp_refresh(mlp, nullptr);
  if (st != CVW_OK) return st;
  CVW_HIP(hipDeviceSynchronize());
  return CVW_OK;
}

cvw_status cvw_mlp_set_range(cvw_mlp* mlp, const float* lo, const float* hi) {
  if (!mlp || !lo || !hi) { set_error("null argument"); return CVW_EINVAL; }
  for (int i = 0; i < MLP_IN; ++i)
    if (std::isnan(lo[i]) || std::isnan(hi[i]) || lo[i] > hi[i]) { set_error("bad feature range"); return CVW_EINVAL; }
  if (hipMemcpy(mlp->lo, lo, MLP_IN * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(mlp->hi, hi, MLP_IN * sizeof(float), hipMemcpyHostToDevice) != hipSuccess) {
    set_error("range upload failed"); return CVW_EDEVICE;
  }
  return CVW_OK;
}

cvw_status cvw_mlp_features(const cvw_mesh* mesh, const cvw_params* prm, const void* u, const void* cand,
                            void* feat, void* stream) {
  if (!mesh || !prm || !u || !cand || !feat) { set_error("null argument"); return CVW_EINVAL; }
  if (mesh->cell != CVW_QUAD || mesh->space != CVW_DG || !mesh->uniform || mesh->degree > MAXP) {
    set_error("features: DG on congruent axis-aligned quadrilaterals, p <= 3"); return CVW_EUNSUPPORTED;
  }
  if (prm->dtype != CVW_F32) { set_error("features: float32 state"); return CVW_EUNSUPPORTED; }
  if (!(prm->sigma_ref > 0) || !std::isfinite(prm->sigma_ref)) { set_error("sigma_ref must be > 0"); return CVW_EINVAL; }
  if (reinterpret_cast<uintptr_t>(feat) % 16) { set_error("features must be 16-byte aligned"); return CVW_EINVAL; }
  return dgquad_features(mesh, static_cast<const float*>(u), static_cast<const float*>(cand), prm->sigma_ref,
                         static_cast<uint16_t*>(feat), static_cast<hipStream_t>(stream));
}

cvw_status cvw_mlp_infer(const cvw_mlp* mlp, const void* feat, int64_t n, void* gamma, void* stream) {
  if (!mlp || n < 0) { set_error("bad argument"); return CVW_EINVAL; }
  if (n == 0) return CVW_OK;
  if (!feat || !gamma) { set_error("null device pointer"); return CVW_EINVAL; }
  if (reinterpret_cast<uintptr_t>(feat) % 16) { set_error("features must be 16-byte aligned"); return CVW_EINVAL; }
  return mlp_infer(mlp->dev(), static_cast<const uint16_t*>(feat), n, static_cast<float*>(gamma),
                   static_cast<hipStream_t>(stream));
}

size_t cvw_mlp_train_workspace_bytes(int batch) {
  if (batch <= 0) return 0;
  return align256(static_cast<size_t>((batch + 31) / 32) * MLP_NPARAM * sizeof(float));
}

cvw_status cvw_mlp_train_step(cvw_mlp* mlp, const void* feat, const void* target, const void* idx, int batch,
                              float lr, void* grad_out, void* ws, size_t ws_bytes, void* stream) {
  if (!mlp || !feat || !target || !idx || !ws) { set_error("null argument"); return CVW_EINVAL; }
  if (batch < 1 || batch > 65536) { set_error("batch must be in [1, 65536]"); return CVW_EINVAL; }
  if (!(lr >= 0) || !std::isfinite(lr)) { set_error("bad learning rate"); return CVW_EINVAL; }
  if (ws_bytes < cvw_mlp_train_workspace_bytes(batch)) { set_error("workspace too small"); return CVW_EINVAL; }
  if (reinterpret_cast<uintptr_t>(feat) % 16) { set_error("features must be 16-byte aligned"); return CVW_EINVAL; }
  auto s = static_cast<hipStream_t>(stream);
  float* part = static_cast<float*>(ws);
  cvw_status st = mlp_train(mlp->dev(), static_cast<const uint16_t*>(feat), static_cast<const float*>(target),
                            static_cast<const int32_t*>(idx), batch, part, s);
  if (st != CVW_OK) return st;
  const double b1 = 0.9, b2 = 0.999;
  const int64_t t = lr > 0 ? mlp->steps + 1 : mlp->steps;
  const double bc1 = lr > 0 ? 1.0 - std::pow(b1, static_cast<double>(t)) : 1.0;
  const double bc2 = lr > 0 ? 1.0 - std::pow(b2, static_cast<double>(t)) : 1.0;
  st = mlp_update(part, (batch + 31) / 32, mlp->master, mlp->m1, mlp->m2, lr, b1, b2, 1e-8f, bc1, bc2,
                  static_cast<float*>(grad_out), mlp->mut(), s);
  if (st == CVW_OK) mlp->steps = t;
  return st;
}

}  // extern "C"
