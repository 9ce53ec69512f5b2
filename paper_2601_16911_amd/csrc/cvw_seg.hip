// One-dimensional CG (Gauss-Lobatto nodes) and DG (Gauss nodes) elements of
// degree p <= 3 with the (p+1)-point Gauss volume rule, in float64 or float32,
// for scalar laws on closed lines (higher degrees, the Euler equations and
// lines with ends go to the one-wave-per-cell kernels of cvw_seghp.hip).
// One thread per vertex / DOF / cell:
//
//  * seg_vertex_kernel   -- Hermite data D^k u_h^e at the vertex from the two
//    cells sharing it, Jiang-Shu weights, vertex candidate (eq. taylorcand);
//  * seg_pg_kernel       -- CG: P_h u' at the DOFs (nodal average);
//  * seg_cell_kernel     -- element semi-norms, WENO weights, gamma_e,
//    lambda_e, nu_e, alpha_q and the element residual (volume + DG
//    interface terms);
//  * seg_assemble_kernel -- CG: R_I = sum of the element entries sharing I.
#include "cvw_device.h"

namespace cvw {

template <typename Real, int FLUX>
__device__ __forceinline__ Real flux1(const MethodScalars& ms, Real u) {
  if constexpr (FLUX == CVW_ADVECT_CONST) return Real(ms.fpd[0]) * u;
  else return Real(0.5) * Real(ms.fpd[0]) * u * u;
}
template <typename Real, int FLUX>
__device__ __forceinline__ Real speed1(const MethodScalars& ms, Real u) {
  if constexpr (FLUX == CVW_ADVECT_CONST) return fabs(Real(ms.fpd[0]));
  else return fabs(u * Real(ms.fpd[0]));
}
template <typename Real, int FLUX>
__device__ __forceinline__ Real numflux1(const MethodScalars& ms, Real um, Real up, Real n) {
  Real lam;
  if (ms.lam_gd > 0.0) lam = Real(ms.lam_gd);
  else lam = fmax(speed1<Real, FLUX>(ms, um), speed1<Real, FLUX>(ms, up));
  return Real(0.5) * (flux1<Real, FLUX>(ms, um) + flux1<Real, FLUX>(ms, up)) * n - Real(0.5) * lam * (up - um);
}

template <int P, typename Real, bool CG>
__device__ __forceinline__ void seg_load(const Real* __restrict__ u, const int32_t* __restrict__ cdof, int64_t e,
                                         Real* ue) {
#pragma unroll
  for (int j = 0; j <= P; ++j) ue[j] = CG ? u[cdof[e * (P + 1) + j]] : u[e * (P + 1) + j];
}

template <int P, typename Real, bool CG>
__global__ __launch_bounds__(256) void seg_vertex_kernel(const Real* __restrict__ u, Real* __restrict__ cand,
                                                         const int32_t* __restrict__ vptr,
                                                         const int32_t* __restrict__ vent,
                                                         const int32_t* __restrict__ cdof,
                                                         const double* __restrict__ hcell,
                                                         const SegTables* __restrict__ tab, int64_t Nv,
                                                         MethodScalars ms) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= Nv) return;
  double acc[P];
#pragma unroll
  for (int k = 0; k < P; ++k) acc[k] = 0.0;
  double wsum = 0.0;
  for (int it = vptr[i]; it < vptr[i + 1]; ++it) {
    const int ent = vent[it];
    const int64_t e = ent >> 2;
    const int lv = ent & 3;
    Real ue[P + 1];
    seg_load<P, Real, CG>(u, cdof, e, ue);
    const double h = hcell[e], s = 2.0 / h;
    double D[P], b2 = 0.0, sc = 1.0;
#pragma unroll
    for (int k = 1; k <= P; ++k) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j <= P; ++j)
        v = fma(tab->Lv[lv][k][j], static_cast<double>(ue[j]) - static_cast<double>(ue[0]), v);
      sc *= s;
      D[k - 1] = v * sc;
      double hk = 1.0;
      for (int r = 0; r < k; ++r) hk *= h * h;
      b2 = fma(hk * D[k - 1], D[k - 1], b2);
    }
    double w;
    if (ms.fast_exp) {
      const double den = ms.eps_vd + sqrt(b2);
      w = 1.0 / (den * den);
    } else {
      w = pow(ms.eps_vd + pow(sqrt(b2), static_cast<double>(ms.q_beta)), -static_cast<double>(ms.r));
    }
#pragma unroll
    for (int k = 0; k < P; ++k) acc[k] = fma(w, D[k], acc[k]);
    wsum += w;
  }
#pragma unroll
  for (int k = 0; k < P; ++k) cand[i * P + k] = static_cast<Real>(acc[k] / wsum);
}

template <int P, typename Real>
__global__ __launch_bounds__(256) void seg_pg_kernel(const Real* __restrict__ u, Real* __restrict__ pg,
                                                     const int32_t* __restrict__ dptr, const int32_t* __restrict__ dent,
                                                     const int32_t* __restrict__ cdof,
                                                     const double* __restrict__ hcell,
                                                     const SegTables* __restrict__ tab, int64_t ndof) {
  const int64_t I = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (I >= ndof) return;
  Real g = Real(0);
  const int beg = dptr[I], end = dptr[I + 1];
  for (int it = beg; it < end; ++it) {
    const int ent = dent[it];
    const int64_t e = ent / (P + 1);
    const int a = ent - static_cast<int>(e) * (P + 1);
    Real ue[P + 1];
    seg_load<P, Real, true>(u, cdof, e, ue);
    Real d = Real(0);
#pragma unroll
    for (int j = 0; j <= P; ++j) d = fma(Real(tab->Dn[a][j]), ue[j], d);
    g += d * Real(2.0 / hcell[e]);
  }
  pg[I] = g / Real(end - beg);
}

template <int P, typename Real, bool CG, int FLUX>
__global__ __launch_bounds__(128) void seg_cell_kernel(const Real* __restrict__ u, const Real* __restrict__ cand,
                                                       const Real* __restrict__ pg, const int32_t* __restrict__ cdof,
                                                       const int32_t* __restrict__ cell_vtx,
                                                       const int32_t* __restrict__ nbr,
                                                       const double* __restrict__ hcell,
                                                       const SegTables* __restrict__ tab, int64_t E, MethodScalars ms,
                                                       int mode, Real* __restrict__ rcell, Real* __restrict__ gamma_out,
                                                       Real* __restrict__ alpha_out, uint32_t* __restrict__ status) {
  constexpr int NQ = P + 1;
  const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (e >= E) return;
  Real ue[P + 1];
  seg_load<P, Real, CG>(u, cdof, e, ue);
  const double h = hcell[e], s = 2.0 / h;
  double hp[P + 1];   // h^{2k}
  hp[0] = 1.0;
#pragma unroll
  for (int k = 1; k <= P; ++k) hp[k] = hp[k - 1] * h * h;
  // derivatives of u at the volume points (float64)
  double Du[NQ][P];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double sc = 1.0;
#pragma unroll
    for (int k = 1; k <= P; ++k) {
      double v = 0.0;
#pragma unroll
      for (int j = 0; j <= P; ++j) v = fma(tab->D[k][q][j], static_cast<double>(ue[j]) - static_cast<double>(ue[0]), v);
      sc *= s;
      Du[q][k - 1] = v * sc;
    }
  }
  // ---- sensor (semi-norms on the Gauss rule, exact for these polynomials) ----
  double gam;
  if (ms.sensor_kind == CVW_SENSOR_FIXED) {
    gam = ms.fixed_gammad;
  } else {
    double c[2][P];
#pragma unroll
    for (int l = 0; l < 2; ++l) {
      const int64_t vid = cell_vtx[e * 2 + l];
#pragma unroll
      for (int k = 0; k < P; ++k) c[l][k] = static_cast<double>(cand[vid * P + k]);
    }
    double n2 = 0.0, b2[2] = {0.0, 0.0}, M[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      const double W = tab->wq[q] * 0.5 * h;
      double dl[2][P];
#pragma unroll
      for (int l = 0; l < 2; ++l) {
        const double dx = (tab->xq[q] - (l == 0 ? -1.0 : 1.0)) * 0.5 * h;
#pragma unroll
        for (int m = 1; m <= P; ++m) {
          double v = 0.0, pw = 1.0;
#pragma unroll
          for (int k = m; k <= P; ++k) {
            v = fma(c[l][k - 1], pw, v);
            pw *= dx / (k - m + 1);
          }
          const double wk = W * hp[m] / h;   // h^{2|k| - d}, d = 1
          b2[l] = fma(wk * v, v, b2[l]);
          dl[l][m - 1] = Du[q][m - 1] - v;
        }
      }
#pragma unroll
      for (int m = 1; m <= P; ++m) {
        const double wk = W * hp[m] / h;
        n2 = fma(wk * Du[q][m - 1], Du[q][m - 1], n2);
        M[0][0] = fma(wk * dl[0][m - 1], dl[0][m - 1], M[0][0]);
        M[0][1] = fma(wk * dl[0][m - 1], dl[1][m - 1], M[0][1]);
        M[1][1] = fma(wk * dl[1][m - 1], dl[1][m - 1], M[1][1]);
      }
    }
    const double beta[3] = {sqrt(n2), sqrt(b2[0]), sqrt(b2[1])};
    double om[3], osum = 0.0;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const double lin = (l == 0) ? 1.0 - 2.0 * ms.lin_wd : ms.lin_wd;
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
    const double o1 = om[1] / osum, o2 = om[2] / osum;
    const double d2 = fmax(o1 * o1 * M[0][0] + 2.0 * o1 * o2 * M[0][1] + o2 * o2 * M[1][1], 0.0);
    if (n2 > 0.0) {
      const double mr = fmin(1.0, sqrt(d2 / n2));
      gam = 1.0 - (ms.fast_exp ? mr : pow(mr, static_cast<double>(ms.q_sensor)));
    } else {
      gam = 1.0;
    }
  }
  // ---- lambda, nu, SC weights ----
  Real uq[NQ], ux[NQ], pgq[NQ];
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    Real v = Real(0), p = Real(0);
#pragma unroll
    for (int j = 0; j <= P; ++j) {
      v = fma(Real(tab->D[0][q][j]), ue[j], v);
      if constexpr (CG) p = fma(Real(tab->D[0][q][j]), pg[cdof[e * (P + 1) + j]], p);
    }
    uq[q] = v;
    ux[q] = static_cast<Real>(Du[q][0]);
    pgq[q] = p;
  }
  double lam = 0.0;
  if (ms.lam_gd > 0.0) lam = ms.lam_gd;
  else {
#pragma unroll
    for (int q = 0; q < NQ; ++q) lam = fmax(lam, static_cast<double>(speed1<Real, FLUX>(ms, uq[q])));
  }
  const double nu = lam * h / (2.0 * P);
  double atil[NQ], S = 0.0, T = 0.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    double a2 = 0.0;
#pragma unroll
    for (int k = 1; k <= P; ++k) a2 = fma(hp[k] * Du[q][k - 1], Du[q][k - 1], a2);
    atil[q] = sqrt(a2);
    const double W = tab->wq[q] * 0.5 * h;
    const double g = Du[q][0];
    const double f = CG ? g * g - gam * g * static_cast<double>(pgq[q]) : (1.0 - gam) * g * g;
    S = fma(W, f, S);
    T = fma(W * atil[q], f, T);
  }
  const bool act = ms.sc_on && (gam < ms.c_gammad) && (S > 0.0) && (T > 0.0);
  if (mode == MODE_SENSOR) {
    gamma_out[e] = static_cast<Real>(gam);
    if (alpha_out) {
#pragma unroll
      for (int q = 0; q < NQ; ++q) alpha_out[e * NQ + q] = static_cast<Real>(act ? atil[q] * S / T : 1.0);
    }
    return;
  }
  if (gamma_out) gamma_out[e] = static_cast<Real>(gam);
  // ---- element residual ----
  Real r[P + 1];
#pragma unroll
  for (int j = 0; j <= P; ++j) r[j] = Real(0);
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const Real alpha = static_cast<Real>(act ? atil[q] * S / T : 1.0);
    const Real g = CG ? ux[q] - static_cast<Real>(gam) * pgq[q] : static_cast<Real>(1.0 - gam) * ux[q];
    const Real G = -flux1<Real, FLUX>(ms, uq[q]) + static_cast<Real>(nu) * alpha * g;
    const Real WG = Real(tab->wq[q]) * G;   // W_q * (2/h) = w_q: the Jacobians cancel
#pragma unroll
    for (int j = 0; j <= P; ++j) r[j] = fma(Real(tab->D[1][q][j]), WG, r[j]);
  }
  if constexpr (!CG) {
    // interface terms: own trace u(-1) / u(+1), neighbour's opposite trace
#pragma unroll
    for (int f = 0; f < 2; ++f) {
      const int64_t en = nbr[e * 2 + f];
      Real um = Real(0), up = Real(0);
      Real un[P + 1];
      seg_load<P, Real, false>(u, cdof, en, un);
#pragma unroll
      for (int j = 0; j <= P; ++j) {
        um = fma(Real(tab->Lv[f][0][j]), ue[j], um);
        up = fma(Real(tab->Lv[1 - f][0][j]), un[j], up);
      }
      const Real fs = numflux1<Real, FLUX>(ms, um, up, f == 0 ? Real(-1) : Real(1));
#pragma unroll
      for (int j = 0; j <= P; ++j) r[j] = fma(Real(tab->Lv[f][0][j]), fs, r[j]);
    }
  }
  bool bad = false;
#pragma unroll
  for (int j = 0; j <= P; ++j) {
    bad = bad || !isfinite(static_cast<double>(r[j]));
    rcell[e * (P + 1) + j] = r[j];
  }
  if (bad) atomicOr(status, ST_NONFINITE);
}

template <typename Real>
__global__ __launch_bounds__(256) void seg_assemble_kernel(const Real* __restrict__ rcell, Real* __restrict__ R,
                                                           const int32_t* __restrict__ dptr,
                                                           const int32_t* __restrict__ dent, int64_t ndof) {
  const int64_t I = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (I >= ndof) return;
  Real s = Real(0);
  for (int it = dptr[I]; it < dptr[I + 1]; ++it) {
    const int ent = dent[it];
    s += rcell[ent];                      // ent = cell * nloc + local node
  }
  R[I] = s;
}

// ---------------------------------------------------------------------------
static unsigned nb1(int64_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

template <int P, typename Real, bool CG>
static void seg_cand_l(const cvw_mesh* m, const MethodScalars& ms, const void* u, void* cand, hipStream_t s) {
  hipLaunchKernelGGL((seg_vertex_kernel<P, Real, CG>), dim3(nb1(m->Nv, 256)), dim3(256), 0, s,
                     static_cast<const Real*>(u), static_cast<Real*>(cand), m->d_vtx_ptr, m->d_vtx_ent,
                     m->d_cell_dof, m->d_hcell, m->d_segt, m->Nv, ms);
}

template <int P, typename Real>
static void seg_cand_p(const cvw_mesh* m, const MethodScalars& ms, const void* u, void* cand, hipStream_t s) {
  if (m->space == CVW_CG) seg_cand_l<P, Real, true>(m, ms, u, cand, s);
  else seg_cand_l<P, Real, false>(m, ms, u, cand, s);
}

template <typename Real>
static cvw_status seg_cand_r(const cvw_mesh* m, const MethodScalars& ms, const void* u, void* cand, hipStream_t s) {
  switch (m->degree) {
    case 1: seg_cand_p<1, Real>(m, ms, u, cand, s); break;
    case 2: seg_cand_p<2, Real>(m, ms, u, cand, s); break;
    case 3: seg_cand_p<3, Real>(m, ms, u, cand, s); break;
    default: set_error("degree > 3 not on the GPU path"); return CVW_EUNSUPPORTED;
  }
  return CVW_OK;
}

cvw_status seg_candidates(const cvw_mesh* m, const cvw_params* prm, const void* u, void* cand, hipStream_t s) {
  if (seg_hp(m, prm))
    return seghp_candidates(m, prm, static_cast<const double*>(u), static_cast<double*>(cand), s);
  const MethodScalars ms = make_scalars(prm);
  const cvw_status st = prm->dtype == CVW_F64 ? seg_cand_r<double>(m, ms, u, cand, s)
                                              : seg_cand_r<float>(m, ms, u, cand, s);
  if (st != CVW_OK) return st;
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

template <int P, typename Real, bool CG, int FLUX>
static void seg_eval_l(const cvw_mesh* m, const MethodScalars& ms, int mode, const void* u, const void* cand,
                       void* pg, void* rcell, void* R, void* gamma, void* alpha, uint32_t* status, hipStream_t s) {
  if constexpr (CG) {
    hipLaunchKernelGGL((seg_pg_kernel<P, Real>), dim3(nb1(m->ndof, 256)), dim3(256), 0, s,
                       static_cast<const Real*>(u), static_cast<Real*>(pg), m->d_dof_ptr, m->d_dof_ent,
                       m->d_cell_dof, m->d_hcell, m->d_segt, m->ndof);
  }
  hipLaunchKernelGGL((seg_cell_kernel<P, Real, CG, FLUX>), dim3(nb1(m->E, 128)), dim3(128), 0, s,
                     static_cast<const Real*>(u), static_cast<const Real*>(cand), static_cast<const Real*>(pg),
                     m->d_cell_dof, m->d_cell_vtx, m->d_nbr, m->d_hcell, m->d_segt, m->E, ms, mode,
                     static_cast<Real*>(CG ? rcell : R), static_cast<Real*>(gamma), static_cast<Real*>(alpha),
                     status);
  if constexpr (CG) {
    if (mode != MODE_SENSOR)
      hipLaunchKernelGGL((seg_assemble_kernel<Real>), dim3(nb1(m->ndof, 256)), dim3(256), 0, s,
                         static_cast<const Real*>(rcell), static_cast<Real*>(R), m->d_dof_ptr, m->d_dof_ent,
                         m->ndof);
  }
}

template <int P, typename Real, bool CG>
static cvw_status seg_eval_f(const cvw_mesh* m, const MethodScalars& ms, int flux, int mode, const void* u,
                             const void* cand, void* pg, void* rcell, void* R, void* gamma, void* alpha,
                             uint32_t* status, hipStream_t s) {
  if (flux == CVW_ADVECT_CONST)
    seg_eval_l<P, Real, CG, CVW_ADVECT_CONST>(m, ms, mode, u, cand, pg, rcell, R, gamma, alpha, status, s);
  else if (flux == CVW_BURGERS)
    seg_eval_l<P, Real, CG, CVW_BURGERS>(m, ms, mode, u, cand, pg, rcell, R, gamma, alpha, status, s);
  else {
    set_error("1D path: constant-velocity advection and Burgers only");
    return CVW_EUNSUPPORTED;
  }
  return CVW_OK;
}

template <typename Real>
static cvw_status seg_eval_r(const cvw_mesh* m, const MethodScalars& ms, int flux, int mode, const void* u,
                             const void* cand, void* pg, void* rcell, void* R, void* gamma, void* alpha,
                             uint32_t* status, hipStream_t s) {
  const bool cg = m->space == CVW_CG;
  switch (m->degree) {
    case 1: return cg ? seg_eval_f<1, Real, true>(m, ms, flux, mode, u, cand, pg, rcell, R, gamma, alpha, status, s)
                      : seg_eval_f<1, Real, false>(m, ms, flux, mode, u, cand, pg, rcell, R, gamma, alpha, status, s);
    case 2: return cg ? seg_eval_f<2, Real, true>(m, ms, flux, mode, u, cand, pg, rcell, R, gamma, alpha, status, s)
                      : seg_eval_f<2, Real, false>(m, ms, flux, mode, u, cand, pg, rcell, R, gamma, alpha, status, s);
    case 3: return cg ? seg_eval_f<3, Real, true>(m, ms, flux, mode, u, cand, pg, rcell, R, gamma, alpha, status, s)
                      : seg_eval_f<3, Real, false>(m, ms, flux, mode, u, cand, pg, rcell, R, gamma, alpha, status, s);
    default: set_error("degree > 3 not on the GPU path"); return CVW_EUNSUPPORTED;
  }
}

cvw_status seg_eval(const cvw_mesh* m, const cvw_params* prm, int mode, const void* u, const void* cand, void* pg,
                    void* rcell, void* R, void* gamma, void* alpha, uint32_t* status, hipStream_t s) {
  if (seg_hp(m, prm))
    return seghp_eval(m, prm, mode, static_cast<const double*>(u), static_cast<const double*>(cand),
                      static_cast<double*>(pg), static_cast<double*>(rcell), static_cast<double*>(R),
                      static_cast<double*>(gamma), static_cast<double*>(alpha), status, s);
  const MethodScalars ms = make_scalars(prm);
  const cvw_status st =
      prm->dtype == CVW_F64 ? seg_eval_r<double>(m, ms, prm->flux, mode, u, cand, pg, rcell, R, gamma, alpha, status, s)
                            : seg_eval_r<float>(m, ms, prm->flux, mode, u, cand, pg, rcell, R, gamma, alpha, status, s);
  if (st != CVW_OK) return st;
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

}  // namespace cvw
