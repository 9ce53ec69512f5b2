// DG on tetrahedra (P_1, P_2 at the equispaced lattice points; affine cells):
//
//  * tet_vertex_kernel -- eight lanes per mesh vertex: the Hermite data
//    D^k u^e(x_i), 1 <= |k| <= p, of every cell of the vertex patch (eq.
//    taylorsol) from reference derivatives of the basis at the reference
//    vertex and the chain rule with the cell's inverse Jacobian, the pointwise
//    smoothness indicators and Jiang-Shu weights, and the vertex candidate
//    (eq. taylorcand), Sec. 3.2.  Float64.
//  * tet_sensor_kernel -- one thread per cell: the cell-vertex WENO sensor
//    (eq. finalweno, eq. gamma) in float64 with the element semi-norms (eq.
//    snorm, h_e^{2|k|-3}) in closed form from the cell's volume and central
//    second moments (every polynomial involved has degree <= 2).
//  * tet_eval_kernel -- one thread per cell, float32: the viscosity (eq.
//    lostab), the shock-capturing weights (eqs. dissrateorig to alphaq), the
//    volume and interface terms of the DG residual and optionally the
//    Runge-Kutta stage update with the exact element mass; scalar laws and
//    the Euler equations (HLL at the faces; the sensor field and the SC
//    weights from the density).
//
// A face's points are Radon's symmetric rule; the neighbour's trace at the
// cell's own point g is the neighbour's basis at its rule point perm[s][g],
// s the permutation between the two cells' orders of the face's vertices
// (packed with the neighbour's id and face by the mesh build).
#include "cvw_device.h"
#include "cvw_cells3d.h"

namespace cvw {

constexpr int TET_THREADS = 64;
constexpr int TET_VLANES = 8;      // lanes per vertex in the vertex pass

// sum over the eight lanes of the own half row (quad butterflies, then the
// mirrored lane of the other quad); every lane receives bitwise the same value
__device__ __forceinline__ double oct_sumd(double x) {
#pragma clang fp contract(off)
  x = x + dppd<(1 | (0 << 2) | (3 << 4) | (2 << 6))>(x);
  x = x + dppd<(2 | (3 << 2) | (0 << 4) | (1 << 6))>(x);
  x = x + dppd<0x141>(x);
  return x;
}

template <int P>
struct TetShape {
  static constexpr int NLOC = (P + 1) * (P + 2) * (P + 3) / 6, NK = NLOC - 1, NQ = (P + 1) * (P + 1) * (P + 1);
};

struct TetGeo {
  double x0[3];
  double J[3][3];   // J[a][b] = d x_a / d xi_b
  double A[3][3];   // J^{-1}: A[b][a] = d xi_b / d x_a
  double det, h;
};

__device__ __forceinline__ TetGeo load_tetgeo(const double* __restrict__ g, int64_t e) {
  TetGeo G;
  const double* p = g + e * 16;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    G.x0[a] = p[a];
#pragma unroll
    for (int b = 0; b < 3; ++b) G.J[a][b] = p[3 + 3 * a + b];
  }
  G.h = p[12];
  const double (&J)[3][3] = G.J;
  const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1], c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2],
               c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
  G.det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
  const double inv = 1.0 / G.det;
  G.A[0][0] = c00 * inv;
  G.A[1][0] = c01 * inv;
  G.A[2][0] = c02 * inv;
  G.A[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * inv;
  G.A[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * inv;
  G.A[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * inv;
  G.A[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * inv;
  G.A[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * inv;
  G.A[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * inv;
  return G;
}

// physical derivatives (multi-index order (1,0,0),(0,1,0),(0,0,1),(2,0,0),
// (1,1,0),(1,0,1),(0,2,0),(0,1,1),(0,0,2)) from reference derivatives in the
// same order: d/dx_a = sum_b A[b][a] d/dxi_b
template <int P>
__device__ __forceinline__ void tet_phys(const double (&A)[3][3], const double* R, double* D) {
#pragma unroll
  for (int a = 0; a < 3; ++a) D[a] = A[0][a] * R[0] + A[1][a] * R[1] + A[2][a] * R[2];
  if constexpr (P >= 2) {
    double H[3][3];
    H[0][0] = R[3]; H[0][1] = H[1][0] = R[4]; H[0][2] = H[2][0] = R[5];
    H[1][1] = R[6]; H[1][2] = H[2][1] = R[7]; H[2][2] = R[8];
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ic[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      double s = 0.0;
#pragma unroll
      for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int d = 0; d < 3; ++d) s = fma(A[b][ia[t]] * A[d][ic[t]], H[b][d], s);
      D[3 + t] = s;
    }
  }
}

// first derivatives at the offset dx of a Taylor polynomial t about its point (P = 2: plus
// the constant second derivatives, already in t[3..8])
template <int P>
__device__ __forceinline__ void taylor_first(const double* t, const double (&dx)[3], double (&D)[3]) {
  D[0] = t[0];
  D[1] = t[1];
  D[2] = t[2];
  if constexpr (P >= 2) {
    D[0] += t[3] * dx[0] + t[4] * dx[1] + t[5] * dx[2];
    D[1] += t[4] * dx[0] + t[6] * dx[1] + t[7] * dx[2];
    D[2] += t[5] * dx[0] + t[7] * dx[1] + t[8] * dx[2];
  }
}

// ---------------------------------------------------------------------------
// vertex pass
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void tet_vertex_kernel(const float* __restrict__ u, float* __restrict__ cand,
                                                         const int32_t* __restrict__ vptr,
                                                         const int32_t* __restrict__ vent,
                                                         const double* __restrict__ geot,
                                                         const TetTables* __restrict__ tab, int64_t Nv,
                                                         MethodScalars ms) {
  using S = TetShape<P>;
  constexpr int NLOC = S::NLOC, NK = S::NK;
  __shared__ double sTV[4][NK][NLOC];
  for (int i = threadIdx.x; i < 4 * NK * NLOC; i += blockDim.x) {
    const int l = i / (NK * NLOC), r = i % (NK * NLOC);
    sTV[l][r / NLOC][r % NLOC] = tab->TV[l][r / NLOC][r % NLOC];
  }
  __syncthreads();
  // TET_VLANES lanes per vertex, each taking every TET_VLANES-th cell of the patch
  const int64_t v = (static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x) / TET_VLANES;
  const int sub = threadIdx.x % TET_VLANES;
  const bool on = v < Nv;
  double acc[NK], wsum = 0.0;
#pragma unroll
  for (int k = 0; k < NK; ++k) acc[k] = 0.0;
  const int32_t i0 = on ? vptr[v] + sub : 0, i1 = on ? vptr[v + 1] : 0;
  for (int32_t i = i0; i < i1; i += TET_VLANES) {
    const int32_t ent = vent[i];
    const int64_t ce = ent >> 2;
    const int lv = ent & 3;
    const TetGeo G = load_tetgeo(geot, ce);
    const float* uc = u + ce * NLOC;
    const double u0 = static_cast<double>(uc[0]);
    double R[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) R[k] = 0.0;
#pragma unroll
    for (int j = 1; j < NLOC; ++j) {
      const double dj = static_cast<double>(uc[j]) - u0;
#pragma unroll
      for (int k = 0; k < NK; ++k) R[k] = fma(sTV[lv][k][j], dj, R[k]);
    }
    double D[NK];
    tet_phys<P>(G.A, R, D);
    // pointwise semi-norm with h_e^{2|k|} of this cell
    const double h2 = G.h * G.h;
    double b2 = 0.0;
#pragma unroll
    for (int k = 0; k < NK; ++k) b2 = fma((k < 3 ? h2 : h2 * h2) * D[k], D[k], b2);
    double beta = sqrt(b2);
    double w;
    if (ms.fast_exp) {
      const double t = ms.eps_vd + beta;
      w = 1.0 / (t * t);
    } else {
      beta = pow(beta, static_cast<double>(ms.q_beta));
      w = pow(ms.eps_vd + beta, -static_cast<double>(ms.r));
    }
#pragma unroll
    for (int k = 0; k < NK; ++k) acc[k] = fma(w, D[k], acc[k]);
    wsum += w;
  }
  // sums over the vertex's lanes (all lanes of the wavefront take part)
#pragma unroll
  for (int k = 0; k < NK; ++k) acc[k] = oct_sumd(acc[k]);
  wsum = oct_sumd(wsum);
  if (!on || sub != 0) return;
  const double iw = 1.0 / wsum;
#pragma unroll
  for (int k = 0; k < NK; ++k) cand[v * NK + k] = static_cast<float>(acc[k] * iw);
}

// ---------------------------------------------------------------------------
// cell pass
// ---------------------------------------------------------------------------
template <int FLUX>
__device__ __forceinline__ float tet_fn(const MethodScalars& ms, float u, const float (&n)[3]) {
  const float vn = ms.fp[0] * n[0] + ms.fp[1] * n[1] + ms.fp[2] * n[2];
  if constexpr (FLUX == CVW_BURGERS) return 0.5f * u * u * vn;
  else return vn * u;
}

// Element semi-norm (eq. snorm, weights h_e^{2|k|-3}) of a polynomial of
// degree <= 2 on an affine cell, in closed form: its gradient is affine,
// g + H (x - x_c) with g the gradient at the centroid x_c and H the constant
// Hessian (xx, xy, xz, yy, yz, zz), so that
//   int_K |grad p|^2 = vol |g|^2 + tr(M H H),  M = int_K (x - x_c)(x - x_c)^T,
//   int_K |D^k p|^2 = vol H_k^2 for |k| = 2.
template <int P>
__device__ __forceinline__ double tet_snorm(const double (&g)[3], const double (&H)[6], const double (&M)[6], double vol,
                                            double hw1, double hw2) {
  double s1 = vol * (g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  if constexpr (P >= 2) {
    const double Hf[3][3] = {{H[0], H[1], H[2]}, {H[1], H[3], H[4]}, {H[2], H[4], H[5]}};
    const double Mf[3][3] = {{M[0], M[1], M[2]}, {M[1], M[3], M[4]}, {M[2], M[4], M[5]}};
    // tr(M H H) = sum_{a,c} (M H)_{ac} H_{ca}
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double mh = Mf[a][0] * Hf[0][c] + Mf[a][1] * Hf[1][c] + Mf[a][2] * Hf[2][c];
        s1 = fma(mh, Hf[c][a], s1);
      }
    double s2 = 0.0;
#pragma unroll
    for (int t = 0; t < 6; ++t) s2 = fma(H[t], H[t], s2);
    return fma(hw1, s1, hw2 * vol * s2);
  } else {
    return hw1 * s1;
  }
}

// Sensor pass: one thread per cell, float64 (the weights, square roots and
// the ratio of gamma_e in float32).  u_h, the four vertex candidates (Taylor
// polynomials about the vertices, eq. taylorcand) and u_h - u_h^{e,*} are
// polynomials of degree <= p, each semi-norm the closed form above.
template <int P>
__global__ __launch_bounds__(TET_THREADS) void tet_sensor_kernel(const float* __restrict__ u, float* __restrict__ gamma,
                                                                 const float* __restrict__ cand,
                                                                 const int32_t* __restrict__ cell_vtx,
                                                                 const double* __restrict__ geot,
                                                                 const TetTables* __restrict__ tab, int64_t E,
                                                                 MethodScalars ms) {
  using S = TetShape<P>;
  constexpr int NLOC = S::NLOC, NK = S::NK;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * TET_THREADS + threadIdx.x;
  if (e >= E) return;
  const int4 vid = *reinterpret_cast<const int4*>(cell_vtx + e * 4);
  const TetGeo G = load_tetgeo(geot, e);
  float uv[NLOC];
#pragma unroll
  for (int j = 0; j < NLOC; ++j) uv[j] = u[e * NLOC + j];
  const double vol = G.det / 6.0;
  const double hw1 = 1.0 / G.h, hw2 = G.h;          // h_e^{2|k|-3}: |k| = 1, 2
  // centroid offset from vertex 0 and the central second moments
  // M = vol / 20 sum_i y_i y_i^T (y_i the vertices about the centroid)
  double cc[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) cc[a] = 0.25 * (G.J[a][0] + G.J[a][1] + G.J[a][2]);
  double M[6];
  {
    const int ia[6] = {0, 0, 0, 1, 1, 2}, ib[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
    for (int t = 0; t < 6; ++t) {
      const int a = ia[t], b = ib[t];
      const double s = G.J[a][0] * G.J[b][0] + G.J[a][1] * G.J[b][1] + G.J[a][2] * G.J[b][2] - 4.0 * cc[a] * cc[b];
      M[t] = vol / 20.0 * s;
    }
  }
  // u_h: the gradient at the centroid and the Hessian, from the nodal values
  // less the first one
  double du[NLOC];
  const double u00 = static_cast<double>(uv[0]);
#pragma unroll
  for (int j = 0; j < NLOC; ++j) du[j] = static_cast<double>(uv[j]) - u00;
  double R[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) R[k] = 0.0;
#pragma unroll
  for (int j = 1; j < NLOC; ++j) {
#pragma unroll
    for (int b = 0; b < 3; ++b) R[b] = fma(tab->Gc[b][j], du[j], R[b]);
    if constexpr (P >= 2) {
#pragma unroll
      for (int t = 0; t < 6; ++t) R[3 + t] = fma(tab->H2[t][j], du[j], R[3 + t]);
    }
  }
  double D[NK];
  tet_phys<P>(G.A, R, D);
  double gu[3] = {D[0], D[1], D[2]}, Hu[6] = {0, 0, 0, 0, 0, 0};
  if constexpr (P >= 2) {
#pragma unroll
    for (int t = 0; t < 6; ++t) Hu[t] = D[3 + t];
  }
  const double n02 = tet_snorm<P>(gu, Hu, M, vol, hw1, hw2);
  // the candidates: Taylor data about vertex l; gradient at the centroid
  // t_grad + H (x_c - x_l)
  double gl[4][3], Hl[4][6], b2[4];
  const int32_t vv[4] = {vid.x, vid.y, vid.z, vid.w};
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const float* cv = cand + static_cast<int64_t>(vv[l]) * NK;
    double t[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) t[k] = static_cast<double>(cv[k]);
    double dx[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) dx[a] = l == 0 ? cc[a] : cc[a] - G.J[a][l - 1];
#pragma unroll
    for (int a = 0; a < 3; ++a) gl[l][a] = t[a];
#pragma unroll
    for (int q = 0; q < 6; ++q) Hl[l][q] = 0.0;
    if constexpr (P >= 2) {
#pragma unroll
      for (int q = 0; q < 6; ++q) Hl[l][q] = t[3 + q];
      gl[l][0] += t[3] * dx[0] + t[4] * dx[1] + t[5] * dx[2];
      gl[l][1] += t[4] * dx[0] + t[6] * dx[1] + t[7] * dx[2];
      gl[l][2] += t[5] * dx[0] + t[7] * dx[1] + t[8] * dx[2];
    }
    b2[l] = tet_snorm<P>(gl[l], Hl[l], M, vol, hw1, hw2);
  }
  // weights of the cell candidate and the four vertex candidates
  const float n0 = fsqrt(static_cast<float>(fmax(n02, 0.0)));
  double om[5];
  {
    float wf[5], wsum = 0.0f;
#pragma unroll
    for (int l = 0; l < 5; ++l) {
      const float b = l == 0 ? n0 : fsqrt(static_cast<float>(fmax(b2[l - 1], 0.0)));
      const float lin = l == 0 ? 1.0f - 4.0f * ms.lin_w : ms.lin_w;
      if (ms.fast_exp) {
        const float tt = ms.eps_c + b;
        wf[l] = lin / (tt * tt);
      } else {
        wf[l] = lin * powf(ms.eps_c + powf(b, ms.q_beta), -ms.r);
      }
      wsum += wf[l];
    }
#pragma unroll
    for (int l = 0; l < 5; ++l) om[l] = static_cast<double>(wf[l] / wsum);
  }
  double osum = 0.0;
#pragma unroll
  for (int l = 1; l < 5; ++l) osum += om[l];
  // u_h - u_h^{e,*} = sum_{l >= 1} omega_l (u_h - s_l)
  double gd[3], Hd[6];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double v = osum * gu[a];
#pragma unroll
    for (int l = 0; l < 4; ++l) v = fma(-om[l + 1], gl[l][a], v);
    gd[a] = v;
  }
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    double v = osum * Hu[q];
#pragma unroll
    for (int l = 0; l < 4; ++l) v = fma(-om[l + 1], Hl[l][q], v);
    Hd[q] = v;
  }
  const double d2 = tet_snorm<P>(gd, Hd, M, vol, hw1, hw2);
  float gam = 1.0f;
  if (n02 > 0.0) {
    float ratio = fminf(1.0f, fsqrt(static_cast<float>(fmax(d2, 0.0))) / n0);
    if (!ms.fast_exp) ratio = powf(ratio, ms.q_sensor);
    gam = 1.0f - ratio;
  }
  gamma[e] = gam;
}

// Variables per node (the Euler equations: rho, m_x, m_y, m_z, E)
template <int FLUX>
struct TetNV {
  static constexpr int value = FLUX == CVW_EULER ? 5 : 1;
};

// Euler: velocity and pressure of a state
__device__ __forceinline__ float tet_prim(const MethodScalars& ms, const float* u, float (&v)[3]) {
  const float inv = frcp(u[0]);
  v[0] = u[1] * inv;
  v[1] = u[2] * inv;
  v[2] = u[3] * inv;
  return (ms.fp[0] - 1.0f) * (u[4] - 0.5f * u[0] * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]));
}

// HLL with Davis wave-speed estimates for the Euler equations, normal n
__device__ __forceinline__ void tet_hll(const MethodScalars& ms, const float* um, const float* up, const float (&n)[3],
                                        float* fs) {
  const float g = ms.fp[0];
  float vm3[3], vp3[3];
  const float pm = tet_prim(ms, um, vm3), pp = tet_prim(ms, up, vp3);
  const float vm = vm3[0] * n[0] + vm3[1] * n[1] + vm3[2] * n[2];
  const float vp = vp3[0] * n[0] + vp3[1] * n[1] + vp3[2] * n[2];
  const float cm = fsqrt(fmaxf(g * pm * frcp(um[0]), 0.0f)), cp = fsqrt(fmaxf(g * pp * frcp(up[0]), 0.0f));
  const float SL = fminf(vm - cm, vp - cp);
  const float SR = fmaxf(vm + cm, vp + cp);
  float Fm[5], Fp[5];
  Fm[0] = um[0] * vm;
  Fp[0] = up[0] * vp;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    Fm[1 + a] = um[1 + a] * vm + pm * n[a];
    Fp[1 + a] = up[1 + a] * vp + pp * n[a];
  }
  Fm[4] = (um[4] + pm) * vm;
  Fp[4] = (up[4] + pp) * vp;
  const float inv = frcp(SR - SL);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const float mid = (SR * Fm[v] - SL * Fp[v] + SL * SR * (up[v] - um[v])) * inv;
    fs[v] = (SL >= 0.0f) ? Fm[v] : ((SR <= 0.0f) ? Fp[v] : mid);
  }
}

template <int P, int FLUX>
__global__ __launch_bounds__(TET_THREADS) void tet_eval_kernel(
    const float* __restrict__ u, const float* __restrict__ u0, float* __restrict__ out, float* __restrict__ gamma_out,
    float* __restrict__ alpha_out, const float* __restrict__ gamma_in, const int32_t* __restrict__ nbrt, const double* __restrict__ geot, const TetTables* __restrict__ tab, int64_t E,
    MethodScalars ms, int mode, float dt, float a0, float b0, uint32_t* __restrict__ status) {
  using S = TetShape<P>;
  constexpr int NLOC = S::NLOC, NK = S::NK, NQ = S::NQ, NV = TetNV<FLUX>::value;
  const int tid = threadIdx.x;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * TET_THREADS + tid;
  if (e >= E) return;
  const TetGeo G = load_tetgeo(geot, e);
  // variable v of cell e at (v E + e) NLOC
  float uv[NV][NLOC];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int j = 0; j < NLOC; ++j) uv[v][j] = u[(v * E + e) * NLOC + j];
  const double h2 = G.h * G.h;

  // ---- gamma_e: from the sensor pass, or the fixed value
  const float gam = ms.sensor_kind != CVW_SENSOR_FIXED ? gamma_in[e] : ms.fixed_gamma;

  // ---- residual (float32)
  float A[3][3];
#pragma unroll
  for (int b = 0; b < 3; ++b)
#pragma unroll
    for (int a = 0; a < 3; ++a) A[b][a] = static_cast<float>(G.A[b][a]);
  const float fdet = static_cast<float>(G.det);
  // second derivatives of the sensor field (P = 2; constant), for alpha~
  float hs2 = 0.0f;
  if constexpr (P >= 2) {
    double R[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) R[k] = 0.0;
#pragma unroll
    for (int t = 0; t < 6; ++t)
#pragma unroll
      for (int j = 0; j < NLOC; ++j) R[3 + t] = fma(tab->H2[t][j], static_cast<double>(uv[0][j]), R[3 + t]);
    double D[NK];
    tet_phys<P>(G.A, R, D);
#pragma unroll
    for (int t = 0; t < 6; ++t) hs2 += static_cast<float>(D[3 + t] * D[3 + t]);
  }
  float lam = ms.lam_g;
  if (!(lam > 0.0f)) {
    const float vn = fsqrt(ms.fp[0] * ms.fp[0] + ms.fp[1] * ms.fp[1] + ms.fp[2] * ms.fp[2]);
    lam = 0.0f;
    for (int q = 0; q < NQ; ++q) {
      float uq[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        uq[v] = 0.0f;
#pragma unroll
        for (int j = 0; j < NLOC; ++j) uq[v] = fmaf(tab->Bs[q][j], uv[v][j], uq[v]);
      }
      float sp;
      if constexpr (FLUX == CVW_EULER) {
        float vel[3];
        const float pq = tet_prim(ms, uq, vel);
        sp = fsqrt(vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2]) + fsqrt(fmaxf(ms.fp[0] * pq * frcp(uq[0]), 0.0f));
      } else {
        sp = FLUX == CVW_BURGERS ? fabsf(uq[0]) * vn : vn;
      }
      lam = fmaxf(lam, sp);
    }
  }
  const float nu = lam * static_cast<float>(G.h) / (2.0f * P);
  // SC weights (sensor field): S = sum W f, T = sum W alpha~ f over the volume points
  const bool sc_active = ms.sc_on && gam < ms.c_gamma;
  float Sv = 0.0f, Tv = 0.0f;
  const float fh2 = static_cast<float>(h2);
  if (sc_active) {
    for (int q = 0; q < NQ; ++q) {
      float gr[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int j = 0; j < NLOC; ++j)
#pragma unroll
        for (int b = 0; b < 3; ++b) gr[b] = fmaf(tab->Gs[b][q][j], uv[0][j], gr[b]);
      float g2 = 0.0f;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float d = A[0][a] * gr[0] + A[1][a] * gr[1] + A[2][a] * gr[2];
        g2 = fmaf(d, d, g2);
      }
      const float at = fsqrt(fh2 * g2 + fh2 * fh2 * hs2);
      const float W = tab->wqs[q] * fdet;
      const float f = (1.0f - gam) * g2;
      Sv = fmaf(W, f, Sv);
      Tv = fmaf(W * at, f, Tv);
    }
  }
  const bool use_alpha = sc_active && Sv > 0.0f && Tv > 0.0f;
  const float ratioST = use_alpha ? Sv / Tv : 0.0f;
  float r[NV][NLOC];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int j = 0; j < NLOC; ++j) r[v][j] = 0.0f;
  for (int q = 0; q < NQ; ++q) {
    float uq[NV], gp[NV][3];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      float gr[3] = {0.0f, 0.0f, 0.0f};
      uq[v] = 0.0f;
#pragma unroll
      for (int j = 0; j < NLOC; ++j) {
        uq[v] = fmaf(tab->Bs[q][j], uv[v][j], uq[v]);
#pragma unroll
        for (int b = 0; b < 3; ++b) gr[b] = fmaf(tab->Gs[b][q][j], uv[v][j], gr[b]);
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) gp[v][a] = A[0][a] * gr[0] + A[1][a] * gr[1] + A[2][a] * gr[2];
    }
    float alpha = 1.0f;
    if (use_alpha) {
      const float g2 = gp[0][0] * gp[0][0] + gp[0][1] * gp[0][1] + gp[0][2] * gp[0][2];
      alpha = fsqrt(fh2 * g2 + fh2 * fh2 * hs2) * ratioST;
    }
    const float W = tab->wqs[q] * fdet;
    const float gs = nu * alpha * (1.0f - gam);
    if (mode == MODE_SENSOR) {
      if (alpha_out) alpha_out[e * NQ + q] = alpha;
      continue;
    }
    float vel[3] = {0.0f, 0.0f, 0.0f}, pres = 0.0f;
    if constexpr (FLUX == CVW_EULER) pres = tet_prim(ms, uq, vel);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      float V[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        float fa;
        if constexpr (FLUX == CVW_EULER)   // f_a of variable v: m_a, m_c v_a + p delta_ca, (E + p) v_a
          fa = v == 0 ? uq[1 + a] : (v < 4 ? uq[v] * vel[a] + (v - 1 == a ? pres : 0.0f) : (uq[4] + pres) * vel[a]);
        else
          fa = FLUX == CVW_BURGERS ? 0.5f * uq[0] * uq[0] * ms.fp[a] : ms.fp[a] * uq[0];
        V[a] = W * (gs * gp[v][a] - fa);
      }
      float Vr[3];
#pragma unroll
      for (int b = 0; b < 3; ++b) Vr[b] = A[b][0] * V[0] + A[b][1] * V[1] + A[b][2] * V[2];
#pragma unroll
      for (int j = 0; j < NLOC; ++j)
#pragma unroll
        for (int b = 0; b < 3; ++b) r[v][j] = fmaf(tab->Gs[b][q][j], Vr[b], r[v][j]);
    }
  }
  if (mode == MODE_SENSOR) {
    if (gamma_out) gamma_out[e] = gam;
    return;
  }

  // ---- interface terms (face f opposite vertex f)
  float xvf[4][3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    xvf[0][a] = 0.0f;
#pragma unroll
    for (int l = 1; l < 4; ++l) xvf[l][a] = static_cast<float>(G.J[a][l - 1]);   // relative to vertex 0
  }
#pragma unroll(NV == 1 ? 4 : 1)
  for (int f = 0; f < 4; ++f) {
    const int32_t code = nbrt[e * 4 + f];
    const int64_t e2 = code >> 5;
    const int f2 = (code >> 3) & 3, sg = code & 7;
    float va[3], vb[3], vc[3], vo[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {     // the face's vertices and the opposite one (a select: f may be a loop variable)
      float x0 = xvf[0][a], x1 = xvf[1][a], x2 = xvf[2][a], x3 = xvf[3][a];
      va[a] = f == 0 ? x1 : x0;
      vb[a] = f <= 1 ? x2 : x1;
      vc[a] = f <= 2 ? x3 : x2;
      vo[a] = f == 0 ? x0 : (f == 1 ? x1 : (f == 2 ? x2 : x3));
    }
    const float t1[3] = {vb[0] - va[0], vb[1] - va[1], vb[2] - va[2]};
    const float t2[3] = {vc[0] - va[0], vc[1] - va[1], vc[2] - va[2]};
    float n[3] = {t1[1] * t2[2] - t1[2] * t2[1], t1[2] * t2[0] - t1[0] * t2[2], t1[0] * t2[1] - t1[1] * t2[0]};
    const float jf = fsqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
    const float ij = 1.0f / jf;
    const float side = n[0] * (vo[0] - va[0]) + n[1] * (vo[1] - va[1]) + n[2] * (vo[2] - va[2]);
    const float sgn = side > 0.0f ? -ij : ij;          // outward: away from the opposite vertex
#pragma unroll
    for (int a = 0; a < 3; ++a) n[a] *= sgn;
    float un[NV][NLOC];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int j = 0; j < NLOC; ++j) un[v][j] = u[(v * E + e2) * NLOC + j];
    float lfv = 0.0f;
    if constexpr (FLUX != CVW_BURGERS) lfv = fabsf(ms.fp[0] * n[0] + ms.fp[1] * n[1] + ms.fp[2] * n[2]);
    const float bn = fabsf(ms.fp[0] * n[0] + ms.fp[1] * n[1] + ms.fp[2] * n[2]);
#pragma unroll
    for (int g = 0; g < TET_NFP; ++g) {
      const int g2 = tab->perm[sg][g];
      float um[NV], up[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        um[v] = 0.0f;
        up[v] = 0.0f;
#pragma unroll
        for (int j = 0; j < NLOC; ++j) {
          um[v] = fmaf(tab->Bf[f][g][j], uv[v][j], um[v]);
          up[v] = fmaf(tab->Bf[f2][g2][j], un[v][j], up[v]);
        }
      }
      float fs[NV];
      if constexpr (FLUX == CVW_EULER) {
        tet_hll(ms, um, up, n, fs);
      } else {
        float lf = ms.lam_g;
        if (!(lf > 0.0f)) lf = FLUX == CVW_BURGERS ? fmaxf(fabsf(um[0]), fabsf(up[0])) * bn : lfv;
        fs[0] = 0.5f * (tet_fn<FLUX>(ms, um[0], n) + tet_fn<FLUX>(ms, up[0], n)) - 0.5f * lf * (up[0] - um[0]);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const float w = tab->wf[g] * jf * fs[v];
#pragma unroll
        for (int j = 0; j < NLOC; ++j) r[v][j] = fmaf(tab->Bf[f][g][j], w, r[v][j]);
      }
    }
  }

  // ---- output
  bool nonfinite = false;
  if (mode == MODE_RESIDUAL) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int j = 0; j < NLOC; ++j) {
        nonfinite = nonfinite || !isfinite(r[v][j]);
        out[(v * E + e) * NLOC + j] = r[v][j];
      }
  } else {
    // u_out = a0 u_n + b0 (u - dt M_e^{-1} r), M_e = det J M_ref
    const float scl = dt / fdet;
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int j = 0; j < NLOC; ++j) {
        float x = 0.0f;
#pragma unroll
        for (int i = 0; i < NLOC; ++i) x = fmaf(tab->Minv[j][i], r[v][i], x);
        const int64_t idx = (v * E + e) * NLOC + j;
        const float base = (a0 != 0.0f) ? a0 * u0[idx] : 0.0f;
        const float o = base + b0 * (uv[v][j] - scl * x);
        nonfinite = nonfinite || !isfinite(o);
        out[idx] = o;
      }
  }
  if (gamma_out) gamma_out[e] = gam;
  if (nonfinite) atomicOr(status, ST_NONFINITE);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
cvw_status tet_candidates(const cvw_mesh* m, const cvw_params* prm, const float* u, float* cand, hipStream_t s) {
  const MethodScalars ms = make_scalars(prm);
  const dim3 g(static_cast<unsigned>((m->Nv * TET_VLANES + 255) / 256)), b(256);
  switch (m->degree) {
    case 1: hipLaunchKernelGGL(tet_vertex_kernel<1>, g, b, 0, s, u, cand, m->d_vtx_ptr, m->d_vtx_ent, m->d_geoth, m->d_tett, m->Nv, ms); break;
    case 2: hipLaunchKernelGGL(tet_vertex_kernel<2>, g, b, 0, s, u, cand, m->d_vtx_ptr, m->d_vtx_ent, m->d_geoth, m->d_tett, m->Nv, ms); break;
    default: set_error("tetrahedra: degree 1 or 2"); return CVW_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

template <int P, int FLUX>
static void launch_tet_eval(const cvw_mesh* m, const MethodScalars& ms, int mode, const float* u, const float* u0,
                            float* out, float* gamma, float* alpha, const float* cand, float* gbuf, uint32_t* status,
                            float dt, float a0, float b0, hipStream_t s) {
  const dim3 g(static_cast<unsigned>((m->E + TET_THREADS - 1) / TET_THREADS)), b(TET_THREADS);
  // the sensor pass writes gamma_e into the caller's array when there is one, else into the scratch
  float* gs = gamma ? gamma : gbuf;
  const bool plain = ms.sensor_kind != CVW_SENSOR_FIXED;
  if (plain)
    hipLaunchKernelGGL((tet_sensor_kernel<P>), g, b, 0, s, u, gs, cand, m->d_cell_vtx, m->d_geoth, m->d_tett, m->E, ms);
  float* gout = (plain && gamma) ? nullptr : gamma;
  hipLaunchKernelGGL((tet_eval_kernel<P, FLUX>), g, b, 0, s, u, u0, out, gout, alpha, gs, m->d_nbrt, m->d_geoth,
                     m->d_tett, m->E, ms, mode, dt, a0, b0, status);
}

cvw_status tet_eval(const cvw_mesh* m, const cvw_params* prm, int mode, const float* u, const float* u0, float* out,
                    float* gamma, float* alpha, const float* cand, float* gbuf, uint32_t* status, float dt, float a0,
                    float b0, hipStream_t s) {
  const MethodScalars ms = make_scalars(prm);
  const bool burgers = prm->flux == CVW_BURGERS;
  const bool euler = prm->flux == CVW_EULER;
  switch (m->degree) {
    case 1:
      if (burgers) launch_tet_eval<1, CVW_BURGERS>(m, ms, mode, u, u0, out, gamma, alpha, cand, gbuf, status, dt, a0, b0, s);
      else if (euler) launch_tet_eval<1, CVW_EULER>(m, ms, mode, u, u0, out, gamma, alpha, cand, gbuf, status, dt, a0, b0, s);
      else launch_tet_eval<1, CVW_ADVECT_CONST>(m, ms, mode, u, u0, out, gamma, alpha, cand, gbuf, status, dt, a0, b0, s);
      break;
    case 2:
      if (burgers) launch_tet_eval<2, CVW_BURGERS>(m, ms, mode, u, u0, out, gamma, alpha, cand, gbuf, status, dt, a0, b0, s);
      else if (euler) launch_tet_eval<2, CVW_EULER>(m, ms, mode, u, u0, out, gamma, alpha, cand, gbuf, status, dt, a0, b0, s);
      else launch_tet_eval<2, CVW_ADVECT_CONST>(m, ms, mode, u, u0, out, gamma, alpha, cand, gbuf, status, dt, a0, b0, s);
      break;
    default: set_error("tetrahedra: degree 1 or 2"); return CVW_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

}  // namespace cvw
