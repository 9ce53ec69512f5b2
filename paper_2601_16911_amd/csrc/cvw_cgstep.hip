// Time stepping for the CG paths and the 1D DG path.
//
// CG (Sec. 2.1, eq. sdstab): the stage needs L = -M^{-1} R with the
// consistent global mass matrix M.  M is inverted by a preconditioned
// conjugate gradient iteration that stays on the device: its scalars live in
// a small device array, each kernel reads them, and once the preconditioned
// residual has dropped below the tolerance every later kernel of the fixed
// launch sequence returns at once.  No host synchronisation, so a stage can
// be captured in a graph.  Preconditioner: the inverse row sums of M (the
// integrals of the nodal basis functions; positive for Gauss-Lobatto nodes).
// Dot products are reduced in float64 in a fixed order (deterministic).  On
// a line (segments) the same iteration runs inside one workgroup.
//
// 1D DG: Gauss nodes with the (p+1)-point Gauss rule make the element mass
// exactly diagonal, so the stage divides by it directly.
#include "cvw_device.h"

namespace cvw {

enum { S_RZ = 0, S_PAP = 1, S_RZ0 = 2, S_ALPHA = 3, S_BETA = 4, S_DONE = 5, S_TOL2 = 6, S_ITER = 7 };
constexpr int PCG_THREADS = 256;

__device__ __forceinline__ bool pcg_done(const double* S) { return S[S_DONE] != 0.0; }

// block sum of one double per thread (PCG_THREADS threads); result valid in every thread
__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = PCG_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

// ycell_e = M_e x_e on bilinear quadrilaterals; the (p+1)^2 Gauss rule
// integrates phi_i phi_j |det J| exactly (degree 2p + 1 per direction)
template <int P>
__global__ __launch_bounds__(128) void cgq_mass_kernel(const float* __restrict__ x, float* __restrict__ ycell,
                                                       const int32_t* __restrict__ cdof, const float* __restrict__ geo,
                                                       const CGTables* __restrict__ tab, int64_t E,
                                                       const double* __restrict__ S) {
  constexpr int N1 = P + 1, NLOC = N1 * N1;
  if (pcg_done(S)) return;
  const int64_t e = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (e >= E) return;
  float xe[NLOC], y[NLOC];
#pragma unroll
  for (int j = 0; j < NLOC; ++j) {
    xe[j] = x[cdof[e * NLOC + j]];
    y[j] = 0.0f;
  }
  const Geo G = load_geo(geo, e);
#pragma unroll
  for (int qy = 0; qy < N1; ++qy)
#pragma unroll
    for (int qx = 0; qx < N1; ++qx) {
      float px, py, J[2][2];
      geo_eval(G, tab->xv[qx], tab->xv[qy], px, py, J);
      const float W = tab->wv[qx] * tab->wv[qy] * fabsf(J[0][0] * J[1][1] - J[0][1] * J[1][0]);
      float xq = 0.0f;
#pragma unroll
      for (int b = 0; b < N1; ++b)
#pragma unroll
        for (int a = 0; a < N1; ++a) xq = fmaf(tab->Dv[0][qx][a] * tab->Dv[0][qy][b], xe[a + N1 * b], xq);
      const float Wx = W * xq;
#pragma unroll
      for (int b = 0; b < N1; ++b)
#pragma unroll
        for (int a = 0; a < N1; ++a) y[a + N1 * b] = fmaf(tab->Dv[0][qx][a] * tab->Dv[0][qy][b], Wx, y[a + N1 * b]);
    }
#pragma unroll
  for (int j = 0; j < NLOC; ++j) ycell[e * NLOC + j] = y[j];
}

// Ap_I = sum of the element entries sharing I (ascending (cell, node) order);
// block partial of p . Ap
template <typename Real>
__global__ __launch_bounds__(PCG_THREADS) void pcg_gather_dot_kernel(const Real* __restrict__ ycell,
                                                                     const Real* __restrict__ p, Real* __restrict__ Ap,
                                                                     double* __restrict__ part,
                                                                     const int32_t* __restrict__ dptr,
                                                                     const int32_t* __restrict__ dent,
                                                                     int64_t n, const double* __restrict__ S) {
  __shared__ double sh[PCG_THREADS];
  if (pcg_done(S)) return;
  const int64_t I = blockIdx.x * static_cast<int64_t>(PCG_THREADS) + threadIdx.x;
  double d = 0.0;
  if (I < n) {
    Real s = Real(0);
    for (int it = dptr[I]; it < dptr[I + 1]; ++it) {
      const int ent = dent[it];
      s += ycell[ent];                    // ent = cell * nloc + local node
    }
    Ap[I] = s;
    d = static_cast<double>(p[I]) * static_cast<double>(s);
  }
  const double b = block_sum(d, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = b;
}

// x = 0, r = b, z = D r, p = z; block partial of r . z
template <typename Real>
__global__ __launch_bounds__(PCG_THREADS) void pcg_init_kernel(const Real* __restrict__ b,
                                                               const Real* __restrict__ dinv, Real* __restrict__ x,
                                                               Real* __restrict__ r, Real* __restrict__ z,
                                                               Real* __restrict__ p, double* __restrict__ part,
                                                               int64_t n) {
  __shared__ double sh[PCG_THREADS];
  const int64_t i = blockIdx.x * static_cast<int64_t>(PCG_THREADS) + threadIdx.x;
  double d = 0.0;
  if (i < n) {
    const Real bi = b[i];
    const Real zi = dinv[i] * bi;
    x[i] = Real(0);
    r[i] = bi;
    z[i] = zi;
    p[i] = zi;
    d = static_cast<double>(bi) * static_cast<double>(zi);
  }
  const double s = block_sum(d, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// x += alpha p, r -= alpha Ap, z = D r; block partial of r . z
template <typename Real>
__global__ __launch_bounds__(PCG_THREADS) void pcg_update_kernel(Real* __restrict__ x, Real* __restrict__ r,
                                                                 Real* __restrict__ z, const Real* __restrict__ p,
                                                                 const Real* __restrict__ Ap,
                                                                 const Real* __restrict__ dinv,
                                                                 double* __restrict__ part, int64_t n,
                                                                 const double* __restrict__ S) {
  __shared__ double sh[PCG_THREADS];
  if (pcg_done(S)) return;
  const int64_t i = blockIdx.x * static_cast<int64_t>(PCG_THREADS) + threadIdx.x;
  const Real al = static_cast<Real>(S[S_ALPHA]);
  double d = 0.0;
  if (i < n) {
    x[i] = fma(al, p[i], x[i]);
    const Real ri = fma(-al, Ap[i], r[i]);
    const Real zi = dinv[i] * ri;
    r[i] = ri;
    z[i] = zi;
    d = static_cast<double>(ri) * static_cast<double>(zi);
  }
  const double s = block_sum(d, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// p = z + beta p
template <typename Real>
__global__ __launch_bounds__(PCG_THREADS) void pcg_direction_kernel(Real* __restrict__ p, const Real* __restrict__ z,
                                                                    int64_t n, const double* __restrict__ S) {
  if (pcg_done(S)) return;
  const int64_t i = blockIdx.x * static_cast<int64_t>(PCG_THREADS) + threadIdx.x;
  if (i >= n) return;
  p[i] = fma(static_cast<Real>(S[S_BETA]), p[i], z[i]);
}

// Sum of the block partials (fixed order) and the scalar recurrences.
//   op 0: rz = rz0 = sum (done at once for a zero right-hand side)
//   op 1: alpha = rz / (p . Ap)
//   op 2: beta = rz_new / rz, rz = rz_new, done once rz_new <= tol^2 rz0
__global__ __launch_bounds__(PCG_THREADS) void pcg_scalar_kernel(const double* __restrict__ part, int nb,
                                                                 double* __restrict__ S, int op) {
  __shared__ double sh[PCG_THREADS];
  if (pcg_done(S)) return;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nb; i += PCG_THREADS) acc += part[i];
  const double v = block_sum(acc, sh);
  if (threadIdx.x != 0) return;
  if (op == 0) {
    S[S_RZ] = v;
    S[S_RZ0] = v;
    if (!(v > 0.0)) S[S_DONE] = 1.0;
  } else if (op == 1) {
    S[S_PAP] = v;
    S[S_ALPHA] = S[S_RZ] / v;
  } else {
    S[S_BETA] = v / S[S_RZ];
    S[S_RZ] = v;
    S[S_ITER] += 1.0;
    if (!(v > S[S_TOL2] * S[S_RZ0])) S[S_DONE] = 1.0;
  }
}

// After the fixed launch sequence: a solve that has not met its tolerance
// (nor broken down) sets ST_PCG_STALL in the workspace status word.
__global__ void pcg_check_kernel(const double* __restrict__ S, uint32_t* __restrict__ status) {
  if (threadIdx.x == 0 && !pcg_done(S)) atomicOr(status, ST_PCG_STALL);
}

__global__ void pcg_setup_kernel(double* __restrict__ S, double tol2) {
  if (threadIdx.x != 0) return;
  for (int i = 0; i < 8; ++i) S[i] = 0.0;
  S[S_TOL2] = tol2;
}

// u_out = a0 u_n + b0 (u_s - dt x), x = M^{-1} R (dinv != null: x = dinv * R, a
// diagonal mass of nm entries shared by every variable); a0 = 0: u_n is not read
template <typename Real>
__global__ __launch_bounds__(256) void stage_update_kernel(const Real* __restrict__ us, const Real* __restrict__ un,
                                                           const Real* __restrict__ x, const Real* __restrict__ dinv,
                                                           Real* __restrict__ uo, Real a0, Real b0, Real dt,
                                                           int64_t n, int64_t nm) {
  const int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= n) return;
  const Real xi = dinv ? x[i] * dinv[i % nm] : x[i];
  const Real base = (a0 != Real(0)) ? a0 * un[i] : Real(0);
  uo[i] = base + b0 * (us[i] - dt * xi);
}

// The whole PCG solve of a line (segments) in one workgroup per variable
// (workgroup v: variable v; every vector is [n_var][ndof]): the same
// iteration, tolerance and cap as the launch sequence above, with the phases
// separated by workgroup barriers instead of kernel launches (a 1D mesh has
// at most a few thousand DOFs, where the launch sequence costs ~3 us per
// launch and the arithmetic well under that).  The element mass is
// (h_e / 2) M_ref with M_ref = sum_q w_q l_i(x_q) l_j(x_q), formed in LDS from
// the tables of any degree.  Dot products: per-thread partials in a fixed
// stride order, then a fixed tree.
constexpr int SMALL_THREADS = 1024;

__device__ __forceinline__ double wg_sum(double v, double* sh) {
  __syncthreads();
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = SMALL_THREADS / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  return sh[0];
}

template <typename Real>
__global__ __launch_bounds__(SMALL_THREADS) void pcg_line_kernel(
    const Real* __restrict__ b, Real* __restrict__ x, Real* __restrict__ r, Real* __restrict__ z,
    Real* __restrict__ p, Real* __restrict__ Ap, Real* __restrict__ ycell, const Real* __restrict__ dinv,
    const double* __restrict__ tab, const double* __restrict__ hcell, const int32_t* __restrict__ cdof,
    const int32_t* __restrict__ dptr, const int32_t* __restrict__ dent, int deg, int64_t E, int64_t n, double tol2,
    int maxit, uint32_t* __restrict__ status) {
  __shared__ double sh[SMALL_THREADS];
  __shared__ double Mref[(HP_MAXP + 1) * (HP_MAXP + 1)];
  const int tid = threadIdx.x;
  {
    const int64_t off = static_cast<int64_t>(blockIdx.x) * n;   // this workgroup's variable
    b += off; x += off; r += off; z += off; p += off; Ap += off;
    ycell += static_cast<int64_t>(blockIdx.x) * E * (deg + 1);
  }
  const int n1 = deg + 1;
  const HPOff o = hp_off(deg);
  for (int w = tid; w < n1 * n1; w += SMALL_THREADS) {
    const int i = w / n1, j = w - i * n1;
    double s = 0.0;
    for (int q = 0; q < n1; ++q) s += tab[o.wq + q] * tab[o.DQ + i * n1 + q] * tab[o.DQ + j * n1 + q];
    Mref[w] = s;
  }
  double d = 0.0;
  for (int64_t i = tid; i < n; i += SMALL_THREADS) {
    const Real bi = b[i];
    const Real zi = dinv[i] * bi;
    x[i] = Real(0);
    r[i] = bi;
    z[i] = zi;
    p[i] = zi;
    d += static_cast<double>(bi) * static_cast<double>(zi);
  }
  double rz = wg_sum(d, sh);
  const double rz0 = rz;
  bool done = !(rz > 0.0);
  for (int it = 0; it < maxit && !done; ++it) {
    for (int64_t w = tid; w < E * n1; w += SMALL_THREADS) {
      const int64_t e = w / n1;
      const int i = static_cast<int>(w - e * n1);
      double y = 0.0;
      for (int j = 0; j < n1; ++j) y += Mref[i * n1 + j] * static_cast<double>(p[cdof[e * n1 + j]]);
      ycell[w] = static_cast<Real>(0.5 * hcell[e] * y);
    }
    __syncthreads();
    d = 0.0;
    for (int64_t I = tid; I < n; I += SMALL_THREADS) {
      Real s = Real(0);
      for (int k = dptr[I]; k < dptr[I + 1]; ++k) s += ycell[dent[k]];
      Ap[I] = s;
      d += static_cast<double>(p[I]) * static_cast<double>(s);
    }
    const double al = rz / wg_sum(d, sh);
    d = 0.0;
    for (int64_t i = tid; i < n; i += SMALL_THREADS) {
      x[i] = fma(static_cast<Real>(al), p[i], x[i]);
      const Real ri = fma(static_cast<Real>(-al), Ap[i], r[i]);
      const Real zi = dinv[i] * ri;
      r[i] = ri;
      z[i] = zi;
      d += static_cast<double>(ri) * static_cast<double>(zi);
    }
    const double rzn = wg_sum(d, sh);
    const double be = rzn / rz;
    rz = rzn;
    if (!(rzn > tol2 * rz0)) { done = true; break; }
    for (int64_t i = tid; i < n; i += SMALL_THREADS) p[i] = fma(static_cast<Real>(be), p[i], z[i]);
    __syncthreads();
  }
  if (tid == 0 && !done) atomicOr(status, ST_PCG_STALL);
}

static unsigned nbk(int64_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }

template <typename Real>
static void mass_cells(const cvw_mesh* m, const Real* x, Real* ycell, const double* S, hipStream_t s) {
  // CG quadrilaterals (float32); lines take pcg_line_kernel
  const dim3 g(nbk(m->E, 128)), b(128);
  if constexpr (std::is_same<Real, float>::value) {
    if (m->degree == 1)
      hipLaunchKernelGGL(cgq_mass_kernel<1>, g, b, 0, s, x, ycell, m->d_cell_dof, m->d_geo, m->d_cgt, m->E, S);
    else
      hipLaunchKernelGGL(cgq_mass_kernel<2>, g, b, 0, s, x, ycell, m->d_cell_dof, m->d_geo, m->d_cgt, m->E, S);
  }
}

size_t pcg_partials(int64_t n) { return nbk(n, PCG_THREADS); }

template <typename Real>
cvw_status cg_mass_solve(const cvw_mesh* m, const Real* b, Real* x, Real* r, Real* z, Real* p, Real* Ap,
                         Real* ycell, double* part, double* S, const Real* dinv, double tol, int maxit,
                         uint32_t* status, hipStream_t s, int nvar) {
  const int64_t n = m->ndof;
  if (m->cell == CVW_SEG) {            // a line: the whole solve in one workgroup per variable
    hipLaunchKernelGGL((pcg_line_kernel<Real>), dim3(nvar), dim3(SMALL_THREADS), 0, s, b, x, r, z, p, Ap, ycell, dinv,
                       m->d_hp, m->d_hcell, m->d_cell_dof, m->d_dof_ptr, m->d_dof_ent, m->degree, m->E, n,
                       tol * tol, maxit, status);
    return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
  }
  const int nb = static_cast<int>(nbk(n, PCG_THREADS));
  const dim3 g(nb), t(PCG_THREADS);
  hipLaunchKernelGGL(pcg_setup_kernel, dim3(1), dim3(64), 0, s, S, tol * tol);
  hipLaunchKernelGGL((pcg_init_kernel<Real>), g, t, 0, s, b, dinv, x, r, z, p, part, n);
  hipLaunchKernelGGL(pcg_scalar_kernel, dim3(1), t, 0, s, part, nb, S, 0);
  for (int it = 0; it < maxit; ++it) {
    mass_cells<Real>(m, p, ycell, S, s);
    hipLaunchKernelGGL((pcg_gather_dot_kernel<Real>), g, t, 0, s, ycell, p, Ap, part, m->d_dof_ptr, m->d_dof_ent,
                       n, S);
    hipLaunchKernelGGL(pcg_scalar_kernel, dim3(1), t, 0, s, part, nb, S, 1);
    hipLaunchKernelGGL((pcg_update_kernel<Real>), g, t, 0, s, x, r, z, p, Ap, dinv, part, n, S);
    hipLaunchKernelGGL(pcg_scalar_kernel, dim3(1), t, 0, s, part, nb, S, 2);
    hipLaunchKernelGGL((pcg_direction_kernel<Real>), g, t, 0, s, p, z, n, S);
  }
  hipLaunchKernelGGL(pcg_check_kernel, dim3(1), dim3(64), 0, s, S, status);
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

template <typename Real>
cvw_status stage_update(const Real* us, const Real* un, const Real* x, const Real* dinv, Real* uo, double a0,
                        double b0, double dt, int64_t n, hipStream_t s, int64_t nm) {
  hipLaunchKernelGGL((stage_update_kernel<Real>), dim3(nbk(n, 256)), dim3(256), 0, s, us, un, x, dinv, uo,
                     static_cast<Real>(a0), static_cast<Real>(b0), static_cast<Real>(dt), n, nm > 0 ? nm : n);
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

template cvw_status cg_mass_solve<float>(const cvw_mesh*, const float*, float*, float*, float*, float*, float*,
                                         float*, double*, double*, const float*, double, int, uint32_t*,
                                         hipStream_t, int);
template cvw_status cg_mass_solve<double>(const cvw_mesh*, const double*, double*, double*, double*, double*,
                                          double*, double*, double*, double*, const double*, double, int,
                                          uint32_t*, hipStream_t, int);
template cvw_status stage_update<float>(const float*, const float*, const float*, const float*, float*, double,
                                        double, double, int64_t, hipStream_t, int64_t);
template cvw_status stage_update<double>(const double*, const double*, const double*, const double*, double*,
                                         double, double, double, int64_t, hipStream_t, int64_t);

}  // namespace cvw
