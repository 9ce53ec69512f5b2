// One-dimensional CG (Gauss-Lobatto nodes) and DG (Gauss nodes) elements of
// any degree 1 <= p <= 32 in float64, for scalar laws and the Euler
// equations (rho, m, E), on periodic lines and on lines with ends carrying
// boundary data (an inflow state, a reflecting wall or outflow), the setting
// of the paper's shock-tube and blast-wave runs (Sec. 5.4: degrees up to 32
// on eight elements).
//
// One 64-lane wave per vertex, cell or DOF patch; the lanes hold derivative
// orders (vertex pass), Gauss points (cell pass: sensor, weights, fluxes) and
// nodes (residual rows).  Derivatives of every order come from host-built
// tables of the Lagrange basis (hp_off layout) and meet the shared data of
// the cell in LDS.  Every reduction over lanes runs in a fixed order and is
// broadcast from lane 0, so all lanes see the same value.
//
//  * hp_vertex_kernel   -- Hermite data D^k s^e(x_i), k = 1..p, of each cell at
//    the vertex, pointwise smoothness indicator (eq. pointsnorm), Jiang-Shu
//    weights and the vertex candidate (eq. taylorcand).  The patch of an end
//    vertex is its one cell.
//  * hp_pg_kernel       -- CG: P_h u' at the DOFs, every variable.
//  * hp_cell_kernel     -- element semi-norms of the cell and of its two
//    vertex Taylor candidates (eq. snorm), the reconstruction weights and
//    gamma_e (eqs. finalweno, gamma), lambda_e and nu_e (eq. lostab),
//    alpha_q (eqs. dissrateorig to alpha_prelim), the element residual (eq.
//    sdstab) with interface and boundary fluxes.
//  * hp_assemble_kernel -- CG: R_I = sum of the element rows sharing I.
// (The CG mass solve of a line runs in one workgroup, cvw_cgstep.hip.)
#include "cvw_device.h"

namespace cvw {

namespace {

constexpr int N1MAX = HP_MAXP + 1;

// sum over the 64 lanes in a fixed order, broadcast from lane 0
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  return __shfl(v, 0, 64);
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_down(v, off, 64));
  return __shfl(v, 0, 64);
}

__device__ __forceinline__ double ipow(double x, int k) {
  double r = 1.0;
  for (int i = 0; i < k; ++i) r *= x;
  return r;
}

// physical flux f(u) and the largest wave speed |f'(u)| (systems: |v| + c)
__device__ __forceinline__ void hp_flux(const SegHPArgs& A, const double* u, double* f) {
  if (A.flux == CVW_EULER) {
    const double g = A.ms.fpd[0];
    const double v = u[1] / u[0];
    const double pr = (g - 1.0) * (u[2] - 0.5 * u[1] * v);
    f[0] = u[1];
    f[1] = u[1] * v + pr;
    f[2] = (u[2] + pr) * v;
  } else if (A.flux == CVW_BURGERS) {
    f[0] = 0.5 * A.ms.fpd[0] * u[0] * u[0];
  } else {
    f[0] = A.ms.fpd[0] * u[0];
  }
}
__device__ __forceinline__ double hp_speed(const SegHPArgs& A, const double* u) {
  if (A.flux == CVW_EULER) {
    const double g = A.ms.fpd[0];
    const double v = u[1] / u[0];
    const double pr = (g - 1.0) * (u[2] - 0.5 * u[1] * v);
    return fabs(v) + sqrt(fmax(g * pr / u[0], 0.0));
  }
  if (A.flux == CVW_BURGERS) return fabs(A.ms.fpd[0] * u[0]);
  return fabs(A.ms.fpd[0]);
}

// interface flux in the direction n = +-1 (um: this cell's trace, up: the
// other side): HLL with the Davis speed bounds for the Euler equations,
// local Lax-Friedrichs for scalar laws
__device__ __forceinline__ void hp_numflux(const SegHPArgs& A, const double* um, const double* up, double n, double* F) {
  double fm[3], fp[3];
  hp_flux(A, um, fm);
  hp_flux(A, up, fp);
  if (A.flux == CVW_EULER) {
    const double g = A.ms.fpd[0];
    auto vc = [&](const double* u, double& vn, double& c) {
      const double v = u[1] / u[0];
      const double pr = (g - 1.0) * (u[2] - 0.5 * u[1] * v);
      vn = v * n;
      c = sqrt(fmax(g * pr / u[0], 0.0));
    };
    double vm, cm, vp, cp;
    vc(um, vm, cm);
    vc(up, vp, cp);
    const double SL = fmin(vm - cm, vp - cp), SR = fmax(vm + cm, vp + cp);
    for (int v = 0; v < 3; ++v) {
      const double Fm = fm[v] * n, Fp = fp[v] * n;
      F[v] = SL >= 0.0 ? Fm : (SR <= 0.0 ? Fp : (SR * Fm - SL * Fp + SL * SR * (up[v] - um[v])) / (SR - SL));
    }
    return;
  }
  double lam;
  if (A.ms.lam_gd > 0.0) lam = A.ms.lam_gd;
  else if (A.flux == CVW_BURGERS) lam = fmax(fabs(um[0]), fabs(up[0])) * fabs(A.ms.fpd[0] * n);
  else lam = fabs(A.ms.fpd[0] * n);
  F[0] = 0.5 * (fm[0] + fp[0]) * n - 0.5 * lam * (up[0] - um[0]);
}

// exterior state at an end: inflow imposes the given state, a wall mirrors
// the momentum, outflow copies the trace
__device__ __forceinline__ void hp_ghost(const SegHPArgs& A, const double* ub, int end, double* ug) {
  const int kind = end == 0 ? A.bc[0] : A.bc[1];
#pragma unroll
  for (int v = 0; v < 3; ++v) ug[v] = kind == CVW_BC_INFLOW ? (end == 0 ? A.bcs[0][v] : A.bcs[1][v]) : ub[v];
  if (kind == CVW_BC_WALL) ug[1] = -ub[1];
}

// index of local node j of cell e in variable v's block of the state
__device__ __forceinline__ int64_t hp_idx(const SegHPArgs& A, int64_t e, int j) {
  return A.cg ? static_cast<int64_t>(A.cell_dof[e * (A.p + 1) + j]) : e * (A.p + 1) + j;
}

}  // namespace

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void hp_vertex_kernel(SegHPArgs A, const double* __restrict__ u,
                                                       double* __restrict__ cand) {
  __shared__ double su[N1MAX];
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x;
  const int p = A.p, n1 = p + 1;
  const HPOff o = hp_off(p);
  const int k = lane + 1;                 // derivative order held by this lane
  double acc = 0.0, wsum = 0.0;
  for (int it = A.vptr[i]; it < A.vptr[i + 1]; ++it) {
    const int ent = A.vent[it];
    const int64_t e = ent >> 2;
    const int lv = ent & 3;
    __syncthreads();
    if (lane < n1) su[lane] = u[hp_idx(A, e, lane)];
    __syncthreads();
    const double h = A.hcell[e];
    double H = 0.0, hH = 0.0;
    if (k <= p) {
      // derivatives annihilate constants: take them of the data relative to its first node
      const double u0 = su[0];
#pragma unroll 8
      for (int j = 0; j < n1; ++j) H = fma(A.tab[o.DV + (lv * n1 + j) * n1 + k], su[j] - u0, H);
      hH = ipow(2.0, k) * H;               // h^k D^k s = 2^k d^k s / dxi^k
      H *= ipow(2.0 / h, k);
    }
    const double beta = sqrt(wave_sum(hH * hH));
    double w;
    if (A.ms.fast_exp) {
      const double den = A.ms.eps_vd + beta;
      w = 1.0 / (den * den);
    } else {
      w = pow(A.ms.eps_vd + pow(beta, static_cast<double>(A.ms.q_beta)), -static_cast<double>(A.ms.r));
    }
    acc = fma(w, H, acc);
    wsum += w;
  }
  if (k <= p) cand[i * p + lane] = acc / wsum;
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void hp_pg_kernel(SegHPArgs A, const double* __restrict__ u,
                                                    double* __restrict__ pg) {
  const int64_t I = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (I >= A.ndof) return;
  const int n1 = A.p + 1;
  const HPOff o = hp_off(A.p);
  const int beg = A.dptr[I], end = A.dptr[I + 1];
  for (int v = 0; v < A.nv; ++v) {
    const double* uv = u + v * A.ndof;
    double g = 0.0;
    for (int it = beg; it < end; ++it) {
      const int ent = A.dent[it];
      const int64_t e = ent / n1;
      const int a = ent - static_cast<int>(e) * n1;
      double d = 0.0;
      for (int j = 0; j < n1; ++j) d = fma(A.tab[o.DN + a * n1 + j], uv[A.cell_dof[e * n1 + j]], d);
      g += d * (2.0 / A.hcell[e]);
    }
    pg[v * A.ndof + I] = g / (end - beg);
  }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(64) void hp_cell_kernel(SegHPArgs A, const double* __restrict__ u,
                                                     const double* __restrict__ cand, const double* __restrict__ pg,
                                                     int mode, double* __restrict__ rout,
                                                     double* __restrict__ gamma_out, double* __restrict__ alpha_out,
                                                     uint32_t* __restrict__ status) {
  __shared__ double su[3][N1MAX];         // the cell's nodal values, every variable
  __shared__ double spg[3][N1MAX];        // CG: P_h u' at the cell's nodes
  __shared__ double sc[2][HP_MAXP];       // vertex candidates (physical derivatives 1..p)
  __shared__ double sG[3][N1MAX];         // w_q times the volume integrand at the Gauss points
  __shared__ double sF[2][3];             // interface / boundary fluxes of the two faces
  __shared__ int sHas[2];
  const int64_t e = blockIdx.x;
  const int lane = threadIdx.x;
  const int p = A.p, n1 = p + 1, nv = A.nv;
  const HPOff o = hp_off(p);
  const bool plain = A.ms.sensor_kind != CVW_SENSOR_FIXED;
  const int64_t vstride = A.cg ? A.ndof : A.E * n1;
  if (lane < n1) {
    const int64_t ix = hp_idx(A, e, lane);
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      if (v >= nv) break;
      su[v][lane] = u[v * vstride + ix];
      if (A.cg) spg[v][lane] = pg[v * A.ndof + ix];
    }
  }
  if (plain && lane < p) {
    sc[0][lane] = cand[static_cast<int64_t>(A.cell_vtx[e * 2]) * p + lane];
    sc[1][lane] = cand[static_cast<int64_t>(A.cell_vtx[e * 2 + 1]) * p + lane];
  }
  __syncthreads();
  const double h = A.hcell[e], s = 2.0 / h;
  const bool qok = lane < n1;
  const int q = qok ? lane : 0;
  const double xq = A.tab[o.xq + q], wq = A.tab[o.wq + q];
  const double W = qok ? wq * 0.5 * h : 0.0;
  const double dx0 = (xq + 1.0) * 0.5 * h, dx1 = (xq - 1.0) * 0.5 * h;   // from the left / right vertex

  // ---- derivatives of the sensor variable, order by order ----
  const double u0 = su[0][0];
  double n2 = 0.0, b2a = 0.0, b2b = 0.0, M00 = 0.0, M01 = 0.0, M11 = 0.0, a2 = 0.0, du1 = 0.0;
  double sm = 1.0, hm2 = 1.0;
  for (int m = 1; m <= p; ++m) {
    sm *= s;
    hm2 *= h * h;
    double D = 0.0;
    const double* dq = A.tab + o.DQ + (m * n1) * n1 + q;
#pragma unroll 8
    for (int j = 0; j < n1; ++j) D = fma(dq[j * n1], su[0][j] - u0, D);
    D = qok ? D * sm : 0.0;
    if (m == 1) du1 = D;
    a2 = fma(hm2 * D, D, a2);
    if (plain) {
      // m-th derivatives of the two vertex Taylor candidates at x_q
      double t0 = sc[0][p - 1], t1 = sc[1][p - 1];
      for (int kk = p - 1; kk >= m; --kk) {
        t0 = fma(t0, dx0 / (kk - m + 1), sc[0][kk - 1]);
        t1 = fma(t1, dx1 / (kk - m + 1), sc[1][kk - 1]);
      }
      if (!qok) { t0 = 0.0; t1 = 0.0; }
      const double wk = W * hm2 / h;      // h^{2m - 1}: the weight of eq. (snorm) in 1D
      n2 = fma(wk * D, D, n2);
      b2a = fma(wk * t0, t0, b2a);
      b2b = fma(wk * t1, t1, b2b);
      const double d0 = D - t0, d1 = D - t1;
      M00 = fma(wk * d0, d0, M00);
      M01 = fma(wk * d0, d1, M01);
      M11 = fma(wk * d1, d1, M11);
    }
  }

  // ---- gamma_e ----
  double gam;
  if (!plain) {
    gam = A.ms.fixed_gammad;
  } else {
    n2 = wave_sum(n2);
    b2a = wave_sum(b2a);
    b2b = wave_sum(b2b);
    M00 = wave_sum(M00);
    M01 = wave_sum(M01);
    M11 = wave_sum(M11);
    const double beta[3] = {sqrt(n2), sqrt(b2a), sqrt(b2b)};
    double om[3], osum = 0.0;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      const double lin = l == 0 ? 1.0 - 2.0 * A.ms.lin_wd : A.ms.lin_wd;
      double w;
      if (A.ms.fast_exp) {
        const double den = A.ms.eps_cd + beta[l];
        w = lin / (den * den);
      } else {
        w = lin * pow(A.ms.eps_cd + pow(beta[l], static_cast<double>(A.ms.q_beta)), -static_cast<double>(A.ms.r));
      }
      om[l] = w;
      osum += w;
    }
    const double o1 = om[1] / osum, o2 = om[2] / osum;
    const double d2 = fmax(o1 * o1 * M00 + 2.0 * o1 * o2 * M01 + o2 * o2 * M11, 0.0);
    if (n2 > 0.0) {
      const double mr = fmin(1.0, sqrt(d2 / n2));
      gam = 1.0 - (A.ms.fast_exp ? mr : pow(mr, static_cast<double>(A.ms.q_sensor)));
    } else {
      gam = 1.0;
    }
  }

  // ---- values, first derivatives and P_h u' at x_q; lambda_e, nu_e ----
  double uq[3] = {0.0, 0.0, 0.0}, gq[3] = {0.0, 0.0, 0.0}, pq[3] = {0.0, 0.0, 0.0};
  {
    const double* d0 = A.tab + o.DQ + q;
    const double* d1 = A.tab + o.DQ + n1 * n1 + q;
    for (int j = 0; j < n1; ++j) {
      const double l0 = d0[j * n1], l1 = d1[j * n1];
#pragma unroll
      for (int v = 0; v < 3; ++v) {
        if (v >= nv) break;
        uq[v] = fma(l0, su[v][j], uq[v]);
        gq[v] = fma(l1, su[v][j], gq[v]);
        if (A.cg) pq[v] = fma(l0, spg[v][j], pq[v]);
      }
    }
#pragma unroll
    for (int v = 0; v < 3; ++v) gq[v] *= s;
  }
  double lam;
  if (A.ms.lam_gd > 0.0) lam = A.ms.lam_gd;
  else lam = wave_max(qok ? hp_speed(A, uq) : 0.0);
  const double nu = lam * h / (2.0 * p);

  // ---- shock-capturing weights (density) ----
  const double atil = sqrt(a2);
  const double f = A.cg ? du1 * du1 - gam * du1 * pq[0] : (1.0 - gam) * du1 * du1;
  const double S = wave_sum(W * f), T = wave_sum(W * atil * f);
  const bool act = A.ms.sc_on && (gam < A.ms.c_gammad) && (S > 0.0) && (T > 0.0);
  const double alpha = act ? atil * S / T : 1.0;
  if (mode == MODE_SENSOR) {
    if (lane == 0) gamma_out[e] = gam;
    if (alpha_out && qok) alpha_out[e * n1 + q] = alpha;
    return;
  }
  if (gamma_out && lane == 0) gamma_out[e] = gam;

  // ---- volume integrand at x_q ----
  if (qok) {
    double fl[3] = {0.0, 0.0, 0.0};
    hp_flux(A, uq, fl);
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      if (v >= nv) break;
      const double g = A.cg ? gq[v] - gam * pq[v] : (1.0 - gam) * gq[v];
      sG[v][q] = wq * (-fl[v] + nu * alpha * g);      // W_q (2/h) = w_q
    }
  }
  // ---- interface and boundary fluxes ----
  if (lane < 2) {
    const int fc = lane;
    const int32_t vid = A.cell_vtx[e * 2 + fc];
    const bool at_end = A.vptr[vid + 1] - A.vptr[vid] == 1;
    const double n = fc == 0 ? -1.0 : 1.0;
    double um[3] = {0.0, 0.0, 0.0}, up[3] = {0.0, 0.0, 0.0};
    for (int j = 0; j < n1; ++j) {
      const double l = A.tab[o.DV + (fc * n1 + j) * n1];
#pragma unroll
      for (int v = 0; v < 3; ++v)
        if (v < nv) um[v] = fma(l, su[v][j], um[v]);
    }
    int has = 0;
    if (at_end) {
      hp_ghost(A, um, fc, up);
      has = 1;
    } else if (!A.cg) {
      const int64_t en = A.nbr[e * 2 + fc];
      for (int j = 0; j < n1; ++j) {
        const double l = A.tab[o.DV + ((1 - fc) * n1 + j) * n1];
#pragma unroll
        for (int v = 0; v < 3; ++v)
          if (v < nv) up[v] = fma(l, u[v * vstride + en * n1 + j], up[v]);
      }
      has = 1;
    }
    double F[3] = {0.0, 0.0, 0.0};
    if (has) hp_numflux(A, um, up, n, F);
#pragma unroll
    for (int v = 0; v < 3; ++v) sF[fc][v] = F[v];
    sHas[fc] = has;
  }
  __syncthreads();
  // ---- element rows ----
  if (lane < n1) {
    const int j = lane;
    const double* d1 = A.tab + o.DQ + (n1 + j) * n1;
    const double l0 = A.tab[o.DV + j * n1], l1 = A.tab[o.DV + (n1 + j) * n1];
    bool bad = false;
#pragma unroll
    for (int v = 0; v < 3; ++v) {
      if (v >= nv) break;
      double r = 0.0;
#pragma unroll 8
      for (int qq = 0; qq < n1; ++qq) r = fma(d1[qq], sG[v][qq], r);
      if (sHas[0]) r = fma(l0, sF[0][v], r);
      if (sHas[1]) r = fma(l1, sF[1][v], r);
      bad = bad || !isfinite(r);
      rout[v * A.E * n1 + e * n1 + j] = r;
    }
    if (bad) atomicOr(status, ST_NONFINITE);
  }
}

// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void hp_assemble_kernel(SegHPArgs A, const double* __restrict__ rcell,
                                                          double* __restrict__ R) {
  const int64_t I = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (I >= A.ndof) return;
  const int64_t cs = A.E * (A.p + 1);
  for (int v = 0; v < A.nv; ++v) {
    double s = 0.0;
    for (int it = A.dptr[I]; it < A.dptr[I + 1]; ++it) s += rcell[v * cs + A.dent[it]];
    R[v * A.ndof + I] = s;
  }
}

// ---------------------------------------------------------------------------
static unsigned nbh(int64_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

cvw_status seghp_candidates(const cvw_mesh* m, const cvw_params* prm, const double* u, double* cand, hipStream_t s) {
  const SegHPArgs A = seghp_args(m, prm);
  hipLaunchKernelGGL(hp_vertex_kernel, dim3(static_cast<unsigned>(m->Nv)), dim3(64), 0, s, A, u, cand);
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

cvw_status seghp_eval(const cvw_mesh* m, const cvw_params* prm, int mode, const double* u, const double* cand,
                      double* pg, double* rcell, double* R, double* gamma, double* alpha, uint32_t* status,
                      hipStream_t s) {
  const SegHPArgs A = seghp_args(m, prm);
  if (A.cg) hipLaunchKernelGGL(hp_pg_kernel, dim3(nbh(m->ndof, 256)), dim3(256), 0, s, A, u, pg);
  hipLaunchKernelGGL(hp_cell_kernel, dim3(static_cast<unsigned>(m->E)), dim3(64), 0, s, A, u, cand, pg, mode,
                     A.cg ? rcell : R, gamma, alpha, status);
  if (A.cg && mode != MODE_SENSOR)
    hipLaunchKernelGGL(hp_assemble_kernel, dim3(nbh(m->ndof, 256)), dim3(256), 0, s, A, rcell, R);
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

}  // namespace cvw
