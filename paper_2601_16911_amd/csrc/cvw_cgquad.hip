// CG on bilinear (possibly jittered) quadrilaterals, Lagrange basis at the
// Gauss-Lobatto points, (p+1)^2 Gauss volume rule, p = 1, 2, on gfx950.
//
// Four kernels per residual evaluation, one thread per item:
//
//  * cgq_vertex_kernel   -- per mesh vertex: Hermite data D^k u_h^e(x_i) of the
//    cells of the patch C(x_i) (exact physical derivatives through the
//    bilinear map, including the map's Hessian in the second derivatives),
//    pointwise indicators and Jiang-Shu weights, vertex candidate data.
//  * cgq_pg_kernel       -- per global DOF: P_h grad u at the node = mean of
//    the broken gradients of the cells sharing the node (nodal averaging
//    reading of the Scott-Zhang / Clement projection).
//  * cgq_cell_kernel     -- per cell: element semi-norms on the (p+2)^2 Gauss
//    rule, WENO weights, gamma_e, lambda_e and nu_e, the shock-capturing
//    weights alpha_q, and the element residual
//      r_j = sum_q W_q grad phi_j . ( -f(u_q) + nu_e alpha_q (grad u_q - gamma_e P_h grad u_q) )
//    written to an element vector.
//  * cgq_assemble_kernel -- per global DOF: R_I = sum of the element entries
//    of the cells sharing I, in ascending (cell, local node) order (no atomics).
#include "cvw_device.h"

namespace cvw {

namespace {

template <int P>
struct CGDims {
  static constexpr int N1 = P + 1, NLOC = N1 * N1, NK = (P + 1) * (P + 2) / 2 - 1;
  static constexpr int NS = P + 2;      // semi-norm rule points per direction
};

// physical derivatives from reference ones: ref = (u_xi, u_eta, u_xixi, u_xieta, u_etaeta);
// out in multi-index order (1,0),(0,1),(2,0),(1,1),(0,2)
template <int P, typename Real>
__device__ __forceinline__ Real chain(const Geo& G, const float Jf[2][2], const Real* ref, Real* out) {
  const Real J00 = Jf[0][0], J01 = Jf[0][1], J10 = Jf[1][0], J11 = Jf[1][1];
  const Real det = J00 * J11 - J01 * J10;
  const Real inv = Real(1) / det;
  // A[b][a] = dxi_b / dx_a
  const Real A00 = J11 * inv, A01 = -J01 * inv, A10 = -J10 * inv, A11 = J00 * inv;
  out[0] = A00 * ref[0] + A10 * ref[1];
  out[1] = A01 * ref[0] + A11 * ref[1];
  if constexpr (P >= 2) {
    // g_b = sum_m A[b][m] h_m ; G = sum_b u_b g_b
    const Real g0 = A00 * Real(G.h[0]) + A01 * Real(G.h[1]);
    const Real g1 = A10 * Real(G.h[0]) + A11 * Real(G.h[1]);
    const Real Gs = ref[0] * g0 + ref[1] * g1;
    auto second = [&](Real Aa0, Real Aa1, Real Ac0, Real Ac1) {
      // A_{0a} A_{0c} u_xixi + (A_{0a} A_{1c} + A_{1a} A_{0c}) u_xieta + A_{1a} A_{1c} u_etaeta - G (A_{0a} A_{1c} + A_{1a} A_{0c})
      const Real mix = Aa0 * Ac1 + Aa1 * Ac0;
      return Aa0 * Ac0 * ref[2] + mix * ref[3] + Aa1 * Ac1 * ref[4] - Gs * mix;
    };
    // column a of A: (A[0][a], A[1][a])
    out[2] = second(A00, A10, A00, A10);
    out[3] = second(A00, A10, A01, A11);
    out[4] = second(A01, A11, A01, A11);
  }
  return det < Real(0) ? -det : det;
}

template <int P>
__device__ __forceinline__ void load_cell(const float* __restrict__ u, const int32_t* __restrict__ cdof, int64_t e,
                                          float* ue) {
  constexpr int NLOC = CGDims<P>::NLOC;
#pragma unroll
  for (int j = 0; j < NLOC; ++j) ue[j] = u[cdof[e * NLOC + j]];
}

// reference derivatives of a tensor Q_P function with 1D tables T[m][i] (x) and S[m][j] (y):
// (u_xi, u_eta, u_xixi, u_xieta, u_etaeta) and the value
template <int P, typename Real, typename UT>
__device__ __forceinline__ void ref_derivs(const UT* ue, const Real (*Tx)[MAXP + 1], const Real (*Ty)[MAXP + 1],
                                           Real* ref, Real& val) {
  constexpr int N1 = P + 1;
  Real R[3][N1];   // R[m][b] = sum_a Tx[m][a] u_ab
#pragma unroll
  for (int m = 0; m < 3; ++m)
#pragma unroll
    for (int b = 0; b < N1; ++b) {
      Real s = Real(0);
      if (m <= P) {
#pragma unroll
        for (int a = 0; a < N1; ++a) s = fma(Tx[m][a], Real(ue[a + N1 * b]), s);
      }
      R[m][b] = s;
    }
  auto col = [&](int m, int n) {
    Real s = Real(0);
#pragma unroll
    for (int b = 0; b < N1; ++b) s = fma(Ty[n][b], R[m][b], s);
    return s;
  };
  val = col(0, 0);
  ref[0] = col(1, 0);
  ref[1] = col(0, 1);
  if constexpr (P >= 2) {
    ref[2] = col(2, 0);
    ref[3] = col(1, 1);
    ref[4] = col(0, 2);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void cgq_vertex_kernel(const float* __restrict__ u, float* __restrict__ cand,
                                                         const int32_t* __restrict__ vptr,
                                                         const int32_t* __restrict__ vent,
                                                         const int32_t* __restrict__ cdof,
                                                         const float* __restrict__ geo, const float* __restrict__ hev,
                                                         const CGTables* __restrict__ tab, int64_t Nv,
                                                         MethodScalars ms) {
  constexpr int NK = CGDims<P>::NK, NLOC = CGDims<P>::NLOC;
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= Nv) return;
  double acc[NK];
#pragma unroll
  for (int t = 0; t < NK; ++t) acc[t] = 0.0;
  double wsum = 0.0;
  for (int it = vptr[i]; it < vptr[i + 1]; ++it) {
    const int ent = vent[it];
    const int64_t e = ent >> 2;
    const int lv = ent & 3;
    float uf[NLOC];
    load_cell<P>(u, cdof, e, uf);
    // data relative to one nodal value: constant data gives exactly zero derivatives
    double ue[NLOC];
#pragma unroll
    for (int j = 0; j < NLOC; ++j) ue[j] = static_cast<double>(uf[j]) - static_cast<double>(uf[0]);
    const Geo G = load_geo(geo, e);
    const float xi = (lv == 1 || lv == 2) ? 1.0f : -1.0f;
    const float eta = (lv >= 2) ? 1.0f : -1.0f;
    // derivatives of the sensor field in float64 (high derivatives of smooth data cancel)
    const double(*Tx)[MAXP + 1] = (xi > 0) ? tab->Lpd : tab->Lmd;
    const double(*Ty)[MAXP + 1] = (eta > 0) ? tab->Lpd : tab->Lmd;
    double ref[5], val;
    ref_derivs<P, double>(ue, Tx, Ty, ref, val);
    float px, py, J[2][2];
    geo_eval(G, xi, eta, px, py, J);
    double D[5];
    chain<P, double>(G, J, ref, D);
    const double he2 = static_cast<double>(hev[e]) * hev[e];
    double b2 = 0.0;
#pragma unroll
    for (int t = 0; t < NK; ++t) b2 = fma((t < 2 ? he2 : he2 * he2) * D[t], D[t], b2);
    double w;
    if (ms.fast_exp) {
      const double den = ms.eps_vd + sqrt(b2);
      w = 1.0 / (den * den);
    } else {
      w = pow(ms.eps_vd + pow(sqrt(b2), static_cast<double>(ms.q_beta)), -static_cast<double>(ms.r));
    }
#pragma unroll
    for (int t = 0; t < NK; ++t) acc[t] = fma(w, D[t], acc[t]);
    wsum += w;
  }
  const double inv = 1.0 / wsum;
#pragma unroll
  for (int t = 0; t < NK; ++t) cand[i * NK + t] = static_cast<float>(acc[t] * inv);
}

// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void cgq_pg_kernel(const float* __restrict__ u, float* __restrict__ pg,
                                                     const int32_t* __restrict__ dptr,
                                                     const int32_t* __restrict__ dent,
                                                     const int32_t* __restrict__ cdof, const float* __restrict__ geo,
                                                     const CGTables* __restrict__ tab, int64_t ndof) {
  constexpr int N1 = P + 1, NLOC = N1 * N1;
  const int64_t I = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (I >= ndof) return;
  float gx = 0.0f, gy = 0.0f;
  const int beg = dptr[I], end = dptr[I + 1];
  for (int it = beg; it < end; ++it) {
    const int ent = dent[it];
    const int64_t e = ent / NLOC;
    const int j = ent - static_cast<int>(e) * NLOC;
    const int a = j % N1, b = j / N1;
    float ue[NLOC];
    load_cell<P>(u, cdof, e, ue);
    float uxi = 0.0f, ueta = 0.0f;
#pragma unroll
    for (int k = 0; k < N1; ++k) {
      uxi = fmaf(tab->Dn[a][k], ue[k + N1 * b], uxi);
      ueta = fmaf(tab->Dn[b][k], ue[a + N1 * k], ueta);
    }
    const Geo G = load_geo(geo, e);
    float px, py, J[2][2];
    geo_eval(G, tab->xn[a], tab->xn[b], px, py, J);
    const float det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    const float inv = 1.0f / det;
    gx += (J[1][1] * uxi - J[1][0] * ueta) * inv;
    gy += (-J[0][1] * uxi + J[0][0] * ueta) * inv;
  }
  const float cnt = static_cast<float>(end - beg);
  pg[I] = gx / cnt;
  pg[ndof + I] = gy / cnt;
}

// ---------------------------------------------------------------------------
template <int P, int FLUX>
__global__ __launch_bounds__(128) void cgq_cell_kernel(const float* __restrict__ u, const float* __restrict__ cand,
                                                       const float* __restrict__ pg, const int32_t* __restrict__ cdof,
                                                       const int32_t* __restrict__ cell_vtx,
                                                       const float* __restrict__ geo, const float* __restrict__ hev,
                                                       const CGTables* __restrict__ tab, int64_t E, int64_t ndof,
                                                       MethodScalars ms, int mode, float* __restrict__ rcell,
                                                       float* __restrict__ gamma_out, float* __restrict__ alpha_out,
                                                       uint32_t* __restrict__ status) {
  constexpr int N1 = P + 1, NLOC = N1 * N1, NK = CGDims<P>::NK, NS = CGDims<P>::NS;
  const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (e >= E) return;
  float ue[NLOC];
  load_cell<P>(u, cdof, e, ue);
  // sensor-field data relative to one nodal value (exact zero derivatives for constants)
  double us[NLOC];
#pragma unroll
  for (int j = 0; j < NLOC; ++j) us[j] = static_cast<double>(ue[j]) - static_cast<double>(ue[0]);
  const Geo G = load_geo(geo, e);
  const float he = hev[e];
  const float he2 = he * he;

  // ---- sensor gamma_e ---------------------------------------------------------
  float gam;
  if (ms.sensor_kind == CVW_SENSOR_FIXED) {
    gam = ms.fixed_gamma;
  } else {
    float c[4][NK];
    int vid[4];
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      vid[l] = cell_vtx[e * 4 + l];
#pragma unroll
      for (int t = 0; t < NK; ++t) c[l][t] = cand[static_cast<int64_t>(vid[l]) * NK + t];
    }
    double n2 = 0.0;
    double b2[4] = {0.0, 0.0, 0.0, 0.0};
    double M[4][4];
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
      for (int k = 0; k < 4; ++k) M[l][k] = 0.0;
    const double he2d = static_cast<double>(he) * he;
    for (int qy = 0; qy < NS; ++qy)
      for (int qx = 0; qx < NS; ++qx) {
        double Tx[3][MAXP + 1], Ty[3][MAXP + 1];
#pragma unroll
        for (int m = 0; m < 3; ++m)
#pragma unroll
          for (int a = 0; a <= MAXP; ++a) {
            Tx[m][a] = tab->Dsd[m][qx][a];
            Ty[m][a] = tab->Dsd[m][qy][a];
          }
        double ref[5], val;
        ref_derivs<P, double>(us, Tx, Ty, ref, val);
        float px, py, J[2][2];
        geo_eval(G, tab->xs[qx], tab->xs[qy], px, py, J);
        double Du[5];
        const double W = static_cast<double>(tab->ws[qx]) * tab->ws[qy] * chain<P, double>(G, J, ref, Du);
        double wk[5];
        wk[0] = wk[1] = W;
        wk[2] = wk[3] = wk[4] = W * he2d;
        double s2 = 0.0;
#pragma unroll
        for (int t = 0; t < NK; ++t) s2 = fma(wk[t] * Du[t], Du[t], s2);
        n2 += s2;
        double dl[4][NK];
#pragma unroll
        for (int l = 0; l < 4; ++l) {
          const double dx = static_cast<double>(px) - G.d[l][0], dy = static_cast<double>(py) - G.d[l][1];
          double Ds[5];
          if constexpr (P == 1) {
            Ds[0] = c[l][0];
            Ds[1] = c[l][1];
          } else {
            Ds[0] = c[l][0] + c[l][2] * dx + c[l][3] * dy;
            Ds[1] = c[l][1] + c[l][3] * dx + c[l][4] * dy;
            Ds[2] = c[l][2];
            Ds[3] = c[l][3];
            Ds[4] = c[l][4];
          }
          double sb = 0.0;
#pragma unroll
          for (int t = 0; t < NK; ++t) {
            sb = fma(wk[t] * Ds[t], Ds[t], sb);
            dl[l][t] = Du[t] - Ds[t];
          }
          b2[l] += sb;
        }
        // M[l][k] = sum_q sum_t w (Du - Ds_l)(Du - Ds_k)
#pragma unroll
        for (int l = 0; l < 4; ++l)
#pragma unroll
          for (int k = l; k < 4; ++k) {
            double sm = 0.0;
#pragma unroll
            for (int t = 0; t < NK; ++t) sm = fma(wk[t] * dl[l][t], dl[k][t], sm);
            M[l][k] += sm;
          }
      }
    double beta[5];
    beta[0] = sqrt(n2);
#pragma unroll
    for (int l = 0; l < 4; ++l) beta[l + 1] = sqrt(b2[l]);
    double om[5], osum = 0.0;
#pragma unroll
    for (int l = 0; l < 5; ++l) {
      const double lin = (l == 0) ? 1.0 - 4.0 * ms.lin_wd : ms.lin_wd;
      double w;
      if (ms.fast_exp) {
        const double den = ms.eps_cd + beta[l];
        w = lin / (den * den);
      } else {
        w = lin * pow(ms.eps_cd + pow(beta[l], static_cast<double>(ms.q_beta)), -static_cast<double>(ms.r));
      }
      om[l] = w;
      osum += w;
    }
    double d2 = 0.0;
#pragma unroll
    for (int l = 0; l < 4; ++l)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const double mlk = (k >= l) ? M[l][k] : M[k][l];
        d2 += (om[l + 1] / osum) * (om[k + 1] / osum) * mlk;
      }
    d2 = fmax(d2, 0.0);
    if (n2 > 0.0) {
      const float mr = fminf(1.0f, static_cast<float>(sqrt(d2 / n2)));
      gam = 1.0f - (ms.fast_exp ? mr : powf(mr, ms.q_sensor));
    } else {
      gam = 1.0f;
    }
  }

  // ---- wave speed, SC weights (volume rule) ------------------------------------
  float pgn[2][NLOC];
#pragma unroll
  for (int j = 0; j < NLOC; ++j) {
    const int64_t I = cdof[e * NLOC + j];
    pgn[0][j] = pg[I];
    pgn[1][j] = pg[ndof + I];
  }
  float atil[NLOC], fq[NLOC], Wq[NLOC];
  float lam = 0.0f;
  float S = 0.0f, T = 0.0f;
  for (int qy = 0; qy < N1; ++qy)
    for (int qx = 0; qx < N1; ++qx) {
      const int q = qx + N1 * qy;
      double Tx[3][MAXP + 1], Ty[3][MAXP + 1];
#pragma unroll
      for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int a = 0; a <= MAXP; ++a) {
          Tx[m][a] = tab->Dvd[m][qx][a];
          Ty[m][a] = tab->Dvd[m][qy][a];
        }
      double refd[5], vald;
      ref_derivs<P, double>(us, Tx, Ty, refd, vald);
      vald += static_cast<double>(ue[0]);
      float px, py, J[2][2];
      geo_eval(G, tab->xv[qx], tab->xv[qy], px, py, J);
      double Dud[5];
      const float W = tab->wv[qx] * tab->wv[qy] * static_cast<float>(chain<P, double>(G, J, refd, Dud));
      double a2d = 0.0;
      const double he2d = static_cast<double>(he) * he;
#pragma unroll
      for (int t = 0; t < NK; ++t) a2d = fma((t < 2 ? he2d : he2d * he2d) * Dud[t], Dud[t], a2d);
      const float a2 = static_cast<float>(a2d);
      const float val = static_cast<float>(vald);
      float Du[2] = {static_cast<float>(Dud[0]), static_cast<float>(Dud[1])};
      float pgx = 0.0f, pgy = 0.0f;
#pragma unroll
      for (int b = 0; b < N1; ++b)
#pragma unroll
        for (int a = 0; a < N1; ++a) {
          const float phi = tab->Dv[0][qx][a] * tab->Dv[0][qy][b];
          pgx = fmaf(phi, pgn[0][a + N1 * b], pgx);
          pgy = fmaf(phi, pgn[1][a + N1 * b], pgy);
        }
      const float f = Du[0] * Du[0] + Du[1] * Du[1] - gam * (Du[0] * pgx + Du[1] * pgy);
      atil[q] = sqrtf(a2);
      fq[q] = f;
      Wq[q] = W;
      S = fmaf(W, f, S);
      T = fmaf(W * atil[q], f, T);
      if (ms.lam_g <= 0.0f) {
        const float uu[1] = {val};
        lam = fmaxf(lam, wave_speed<FLUX>(ms, uu, G.x0 + px, G.y0 + py));
      }
    }
  if (ms.lam_g > 0.0f) lam = ms.lam_g;
  const float nu = lam * he / (2.0f * P);
  const bool sc_active = ms.sc_on && (static_cast<double>(gam) < ms.c_gammad) && (S > 0.0f) && (T > 0.0f);
  const float ratio = sc_active ? S / T : 0.0f;

  if (mode == MODE_SENSOR) {
    gamma_out[e] = gam;
    if (alpha_out) {
#pragma unroll
      for (int q = 0; q < NLOC; ++q) alpha_out[e * NLOC + q] = sc_active ? atil[q] * ratio : 1.0f;
    }
    return;
  }
  if (gamma_out) gamma_out[e] = gam;

  // ---- element residual ---------------------------------------------------------
  float r[NLOC];
#pragma unroll
  for (int j = 0; j < NLOC; ++j) r[j] = 0.0f;
  bool bad = false;
  for (int qy = 0; qy < N1; ++qy)
    for (int qx = 0; qx < N1; ++qx) {
      const int q = qx + N1 * qy;
      float Tx[2][MAXP + 1], Ty[2][MAXP + 1];
#pragma unroll
      for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int a = 0; a <= MAXP; ++a) {
          Tx[m][a] = tab->Dv[m][qx][a];
          Ty[m][a] = tab->Dv[m][qy][a];
        }
      float uq = 0.0f, uxi = 0.0f, ueta = 0.0f, pgx = 0.0f, pgy = 0.0f;
#pragma unroll
      for (int b = 0; b < N1; ++b)
#pragma unroll
        for (int a = 0; a < N1; ++a) {
          const float v = ue[a + N1 * b];
          const float phi = Tx[0][a] * Ty[0][b];
          uq = fmaf(phi, v, uq);
          uxi = fmaf(Tx[1][a] * Ty[0][b], v, uxi);
          ueta = fmaf(Tx[0][a] * Ty[1][b], v, ueta);
          pgx = fmaf(phi, pgn[0][a + N1 * b], pgx);
          pgy = fmaf(phi, pgn[1][a + N1 * b], pgy);
        }
      float px, py, J[2][2];
      geo_eval(G, tab->xv[qx], tab->xv[qy], px, py, J);
      const float det = J[0][0] * J[1][1] - J[0][1] * J[1][0];
      const float inv = 1.0f / det;
      const float A00 = J[1][1] * inv, A01 = -J[0][1] * inv, A10 = -J[1][0] * inv, A11 = J[0][0] * inv;
      const float ux = A00 * uxi + A10 * ueta, uy = A01 * uxi + A11 * ueta;
      const float uu[1] = {uq};
      float fx[1], fy[1];
      phys_flux<FLUX>(ms, uu, G.x0 + px, G.y0 + py, fx, fy);
      const float alpha = sc_active ? atil[q] * ratio : 1.0f;
      const float cst = nu * alpha;
      const float Gx = -fx[0] + cst * (ux - gam * pgx);
      const float Gy = -fy[0] + cst * (uy - gam * pgy);
      // grad phi_j . G = (A^T grad_ref phi_j) . G = grad_ref phi_j . (A G)
      const float W = Wq[q];
      const float Hx = W * (A00 * Gx + A01 * Gy), Hy = W * (A10 * Gx + A11 * Gy);
#pragma unroll
      for (int b = 0; b < N1; ++b)
#pragma unroll
        for (int a = 0; a < N1; ++a)
          r[a + N1 * b] = fmaf(Tx[1][a] * Ty[0][b], Hx, fmaf(Tx[0][a] * Ty[1][b], Hy, r[a + N1 * b]));
    }
#pragma unroll
  for (int j = 0; j < NLOC; ++j) {
    bad = bad || !isfinite(r[j]);
    rcell[e * NLOC + j] = r[j];
  }
  (void)fq;
  if (bad) atomicOr(status, ST_NONFINITE);
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void cg_assemble_kernel(const float* __restrict__ rcell, float* __restrict__ R,
                                                          const int32_t* __restrict__ dptr,
                                                          const int32_t* __restrict__ dent, int64_t ndof) {
  const int64_t I = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (I >= ndof) return;
  float s = 0.0f;
  for (int it = dptr[I]; it < dptr[I + 1]; ++it) {
    const int ent = dent[it];
    s += rcell[ent];                      // ent = cell * nloc + local node
  }
  R[I] = s;
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static unsigned nblk(int64_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

cvw_status cgquad_candidates(const cvw_mesh* m, const cvw_params* prm, const float* u, float* cand, hipStream_t s) {
  const MethodScalars ms = make_scalars(prm);
  if (m->degree == 1)
    hipLaunchKernelGGL(cgq_vertex_kernel<1>, dim3(nblk(m->Nv, 256)), dim3(256), 0, s, u, cand, m->d_vtx_ptr,
                       m->d_vtx_ent, m->d_cell_dof, m->d_geo, m->d_he, m->d_cgt, m->Nv, ms);
  else
    hipLaunchKernelGGL(cgq_vertex_kernel<2>, dim3(nblk(m->Nv, 256)), dim3(256), 0, s, u, cand, m->d_vtx_ptr,
                       m->d_vtx_ent, m->d_cell_dof, m->d_geo, m->d_he, m->d_cgt, m->Nv, ms);
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

template <int P, int FLUX>
static void launch_cgq_cell(const cvw_mesh* m, const MethodScalars& ms, int mode, const float* u, const float* cand,
                            const float* pg, float* rcell, float* gamma, float* alpha, uint32_t* status,
                            hipStream_t s) {
  hipLaunchKernelGGL((cgq_cell_kernel<P, FLUX>), dim3(nblk(m->E, 128)), dim3(128), 0, s, u, cand, pg,
                     m->d_cell_dof, m->d_cell_vtx, m->d_geo, m->d_he, m->d_cgt, m->E, m->ndof, ms, mode, rcell,
                     gamma, alpha, status);
}

template <int P>
static cvw_status cgq_cell_p(const cvw_mesh* m, const MethodScalars& ms, int flux, int mode, const float* u,
                             const float* cand, const float* pg, float* rcell, float* gamma, float* alpha,
                             uint32_t* status, hipStream_t s) {
  switch (flux) {
    case CVW_ADVECT_CONST: launch_cgq_cell<P, CVW_ADVECT_CONST>(m, ms, mode, u, cand, pg, rcell, gamma, alpha, status, s); break;
    case CVW_ADVECT_ROT: launch_cgq_cell<P, CVW_ADVECT_ROT>(m, ms, mode, u, cand, pg, rcell, gamma, alpha, status, s); break;
    case CVW_BURGERS: launch_cgq_cell<P, CVW_BURGERS>(m, ms, mode, u, cand, pg, rcell, gamma, alpha, status, s); break;
    case CVW_KPP: launch_cgq_cell<P, CVW_KPP>(m, ms, mode, u, cand, pg, rcell, gamma, alpha, status, s); break;
    default: set_error("systems are not on the CG quadrilateral path"); return CVW_EUNSUPPORTED;
  }
  return CVW_OK;
}

cvw_status cgquad_eval(const cvw_mesh* m, const cvw_params* prm, int mode, const float* u, const float* cand,
                       float* pg, float* rcell, float* R, float* gamma, float* alpha, uint32_t* status,
                       hipStream_t s) {
  const MethodScalars ms = make_scalars(prm);
  if (m->degree == 1)
    hipLaunchKernelGGL(cgq_pg_kernel<1>, dim3(nblk(m->ndof, 256)), dim3(256), 0, s, u, pg, m->d_dof_ptr,
                       m->d_dof_ent, m->d_cell_dof, m->d_geo, m->d_cgt, m->ndof);
  else
    hipLaunchKernelGGL(cgq_pg_kernel<2>, dim3(nblk(m->ndof, 256)), dim3(256), 0, s, u, pg, m->d_dof_ptr,
                       m->d_dof_ent, m->d_cell_dof, m->d_geo, m->d_cgt, m->ndof);
  cvw_status st = (m->degree == 1)
                      ? cgq_cell_p<1>(m, ms, prm->flux, mode, u, cand, pg, rcell, gamma, alpha, status, s)
                      : cgq_cell_p<2>(m, ms, prm->flux, mode, u, cand, pg, rcell, gamma, alpha, status, s);
  if (st != CVW_OK) return st;
  if (mode != MODE_SENSOR)
    hipLaunchKernelGGL(cg_assemble_kernel, dim3(nblk(m->ndof, 256)), dim3(256), 0, s, rcell, R, m->d_dof_ptr,
                       m->d_dof_ent, m->ndof);
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

}  // namespace cvw
