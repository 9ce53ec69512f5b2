// DG on affine triangles (P_1..P_3, equispaced Lagrange nodes, Stroud rule):
//
//  * tri_vertex_kernel -- one thread per mesh vertex: Hermite data D^k u^e(x_i),
//    1 <= |k| <= p, of every cell of the vertex patch (eq. taylorsol), the
//    pointwise smoothness indicators and Jiang-Shu weights, and the vertex
//    candidate (eq. taylorcand), Sec. 3.2.  Float64 (derivatives of order 3 of
//    smooth data cancel strongly).
//  * tri_eval_kernel -- one thread per cell: the cell-vertex WENO sensor
//    (eq. finalweno, eq. gamma) in float64, the viscosity (eq. lostab), the
//    shock-capturing weights (eqs. dissrateorig to alphaq), the volume and
//    interface terms of the residual (Sec. 2.1) in float32, and optionally the
//    exact element mass inverse with a Runge-Kutta stage update.
//
// The sensor works on Taylor coefficients: the cell polynomial and the three
// vertex candidates (Taylor polynomials about their vertices) are all written
// as D^m v(x_0), |m| >= 1, about the cell's vertex 0, and each element
// semi-norm (eq. snorm) is a quadratic form in them whose entries are the
// cell's moments about x_0 up to degree 2p - 2, taken once per cell with the
// Stroud rule (exact for those degrees).  Reference tables are read with indices
// that are uniform across a wavefront (scalar loads), except the neighbour-
// face tables, which live in LDS.
#include "cvw_device.h"
#include "cvw_limit.h"

namespace cvw {

__host__ __device__ constexpr int kbase(int n) { return n * (n + 1) / 2 - 1; }   // index of (n, 0)

// D^k_x of a function from its reference derivatives of the same order:
// d/dx = A00 d/dxi + A10 d/deta, d/dy = A01 d/dxi + A11 d/deta (A = J^{-1}).
// R[kbase(n) + b] = d_xi^{n-b} d_eta^b u; out in the same multi-index order.
template <int P>
__device__ __forceinline__ void phys_from_ref(const double A[2][2], const double* R, double* out) {
#pragma unroll
  for (int n = 1; n <= P; ++n)
#pragma unroll
    for (int j = 0; j <= n; ++j) {
      double c[P + 1];
#pragma unroll
      for (int b = 0; b <= P; ++b) c[b] = (b == 0) ? 1.0 : 0.0;
#pragma unroll
      for (int t = 0; t < n; ++t) {
        const int col = (t < n - j) ? 0 : 1;
        const double c0 = A[0][col], c1 = A[1][col];
#pragma unroll
        for (int b = P; b >= 1; --b) c[b] = c[b] * c0 + c[b - 1] * c1;
        c[0] *= c0;
      }
      double s = 0.0;
#pragma unroll
      for (int b = 0; b <= n; ++b) s = fma(c[b], R[kbase(n) + b], s);
      out[kbase(n) + j] = s;
    }
}

// D^m v(x_0 + d) for every 1 <= |m| <= P from t[k] = D^k v(x_0)
template <int P>
__device__ __forceinline__ void taylor_eval(const double* t, double dx, double dy, double* D) {
  double px[P], py[P];
  px[0] = 1.0;
  py[0] = 1.0;
#pragma unroll
  for (int a = 1; a < P; ++a) {
    px[a] = px[a - 1] * dx / a;
    py[a] = py[a - 1] * dy / a;
  }
#pragma unroll
  for (int n = 1; n <= P; ++n)
#pragma unroll
    for (int j = 0; j <= n; ++j) {
      const int mx = n - j, my = j;
      double s = 0.0;
#pragma unroll
      for (int n2 = P; n2 >= n; --n2)
#pragma unroll
        for (int j2 = 0; j2 <= n2; ++j2) {
          const int kx = n2 - j2, ky = j2;
          if (kx >= mx && ky >= my) s = fma(t[kbase(n2) + j2], px[kx - mx] * py[ky - my], s);
        }
      D[kbase(n) + j] = s;
    }
}

struct TriGeo {
  double x0, y0;
  double J[2][2];   // J[a][b] = d x_a / d xi_b
  double A[2][2];   // J^{-1}
  double det, h;
};

__device__ __forceinline__ TriGeo load_trigeo(const double* __restrict__ g, int64_t e) {
  TriGeo G;
  const double* p = g + e * 8;
  G.x0 = p[0];
  G.y0 = p[1];
  G.J[0][0] = p[2];
  G.J[1][0] = p[3];
  G.J[0][1] = p[4];
  G.J[1][1] = p[5];
  G.h = p[6];
  G.det = G.J[0][0] * G.J[1][1] - G.J[0][1] * G.J[1][0];
  const double inv = 1.0 / G.det;
  G.A[0][0] = G.J[1][1] * inv;
  G.A[0][1] = -G.J[0][1] * inv;
  G.A[1][0] = -G.J[1][0] * inv;
  G.A[1][1] = G.J[0][0] * inv;
  return G;
}

// weights h^{2|k| - 2} of eq. (snorm) in two dimensions, per order n = 1..P
template <int P>
__device__ __forceinline__ void order_weights(double h, double* hw) {
  hw[0] = 1.0;
#pragma unroll
  for (int n = 1; n < P; ++n) hw[n] = hw[n - 1] * h * h;
}

template <int P>
__device__ __forceinline__ double weighted_sq(const double* D, const double* hw) {
  double s = 0.0;
#pragma unroll
  for (int n = 1; n <= P; ++n)
#pragma unroll
    for (int j = 0; j <= n; ++j) s = fma(hw[n - 1] * D[kbase(n) + j], D[kbase(n) + j], s);
  return s;
}

// Moments of the cell about x_0 (vertex 0): mu[midx(ax, ay)] = int_T (x - x0)^ax
// (y - y0)^ay dx, ax + ay <= 2P - 2, from the Stroud rule (exact for them).
__host__ __device__ constexpr int midx(int ax, int ay) { return (ax + ay) * (ax + ay + 1) / 2 + ay; }
template <int P> constexpr int NMOM = (2 * P - 1) * (2 * P) / 2;

template <int P>
__device__ __forceinline__ void mom_add(double w, double dx, double dy, double* mu) {
  double px[2 * P - 1], py[2 * P - 1];
  px[0] = w;
  py[0] = 1.0;
#pragma unroll
  for (int a = 1; a < 2 * P - 1; ++a) {
    px[a] = px[a - 1] * dx;
    py[a] = py[a - 1] * dy;
  }
#pragma unroll
  for (int n = 0; n <= 2 * P - 2; ++n)
#pragma unroll
    for (int ay = 0; ay <= n; ++ay) mu[midx(n - ay, ay)] = fma(px[n - ay], py[ay], mu[midx(n - ay, ay)]);
}

template <int P>
__device__ __forceinline__ void cell_moments(const TriGeo& G, const TriTables* __restrict__ tab, double* mu) {
  constexpr int NQ = (P + 1) * (P + 1);
#pragma unroll
  for (int i = 0; i < NMOM<P>; ++i) mu[i] = 0.0;
  const double adet = fabs(G.det);
#pragma unroll 1
  for (int q = 0; q < NQ; ++q) {
    const double xi = tab->xqd[q], eta = tab->yqd[q];
    mom_add<P>(tab->wqd[q] * adet, G.J[0][0] * xi + G.J[0][1] * eta, G.J[1][0] * xi + G.J[1][1] * eta, mu);
  }
}

// ||v||_e^2 of eq. (snorm), sum_m h^{2|m|-2} int_T |D^m v|^2, for v given by its
// Taylor coefficients t at x_0: with D^m v(x) = sum_{k >= m} t_k (x - x0)^{k-m} / (k-m)!
// every integral is a combination of the moments mu
template <int P>
__device__ __forceinline__ double seminorm_mom(const double* t, const double* mu, const double* hw) {
  constexpr double ifct[4] = {1.0, 1.0, 0.5, 1.0 / 6.0};
  double s = 0.0;
#pragma unroll
  for (int n = 1; n <= P; ++n)
#pragma unroll
    for (int j = 0; j <= n; ++j) {
      const int mx = n - j, my = j;
      double sm = 0.0;
#pragma unroll
      for (int n2 = n; n2 <= P; ++n2)
#pragma unroll
        for (int j2 = 0; j2 <= n2; ++j2) {
          const int kx = n2 - j2, ky = j2;
          if (kx < mx || ky < my) continue;
          double inner = 0.0;
#pragma unroll
          for (int n3 = n; n3 <= P; ++n3)
#pragma unroll
            for (int j3 = 0; j3 <= n3; ++j3) {
              const int lx = n3 - j3, ly = j3;
              if (lx < mx || ly < my) continue;
              inner = fma(t[kbase(n3) + j3] * (ifct[lx - mx] * ifct[ly - my]),
                          mu[midx(kx - mx + lx - mx, ky - my + ly - my)], inner);
            }
          sm = fma(t[kbase(n2) + j2] * (ifct[kx - mx] * ifct[ky - my]), inner, sm);
        }
      s = fma(hw[n - 1], sm, s);
    }
  return s;
}

// Taylor coefficients at x_0 of the vertex candidate of local vertex l
// (a Taylor polynomial about x_l with coefficients c), constant term dropped
template <int P>
__device__ __forceinline__ void candidate_at_x0(const float* __restrict__ cand, int32_t vtx, int l, const TriGeo& G,
                                                double* s) {
  constexpr int NK = (P + 1) * (P + 2) / 2 - 1;
  double c[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) c[k] = static_cast<double>(cand[static_cast<int64_t>(vtx) * NK + k]);
  double dx = 0.0, dy = 0.0;      // x_0 - x_l
  if (l == 1) { dx = -G.J[0][0]; dy = -G.J[1][0]; }
  if (l == 2) { dx = -G.J[0][1]; dy = -G.J[1][1]; }
  taylor_eval<P>(c, dx, dy, s);
}

// value at x_0 + d of the polynomial with D^k = t[k] at x_0 (1 <= |k| <= P)
// and value 0 at x_0
template <int P>
__device__ __forceinline__ double taylor_value0(const double* t, double dx, double dy) {
  constexpr double fct[4] = {1.0, 1.0, 2.0, 6.0};
  double s = 0.0;
#pragma unroll
  for (int n = 1; n <= P; ++n)
#pragma unroll
    for (int j = 0; j <= n; ++j) {
      double m = t[kbase(n) + j] / (fct[n - j] * fct[j]);
#pragma unroll
      for (int i = 0; i < n - j; ++i) m *= dx;
#pragma unroll
      for (int i = 0; i < j; ++i) m *= dy;
      s += m;
    }
  return s;
}

// HWENO limiter (Sec. 3; candidates with corrected cell averages, Sec. 3.2),
// one thread per (listed cell, variable), float64:
//   u* = w_0 u_h^e + (1 - w_0) mean(u_h^e) + V - mean(V),
//   V(x) = sum_k cb_k (x - x_0)^k / k!,  cb = sum_{l>=1} w_l D^k u_{h,l}(x_0),
// the candidates and the weights exactly as in the sensor.  Nodes: (i/P, j/P)
// on the reference triangle, j outer.
template <int P, int NV>
__global__ __launch_bounds__(256) void tri_limit_kernel(const float* __restrict__ u, float* __restrict__ out,
                                                        const float* __restrict__ cand,
                                                        const uint32_t* __restrict__ count,
                                                        const int32_t* __restrict__ list,
                                                        const int32_t* __restrict__ cell_vtx,
                                                        const double* __restrict__ geot,
                                                        const TriTables* __restrict__ tab, int64_t E, int64_t Nv,
                                                        MethodScalars ms) {
  constexpr int NLOC = (P + 1) * (P + 2) / 2, NK = NLOC - 1, NQ = (P + 1) * (P + 1);
  const int64_t gid = blockIdx.x * 256LL + threadIdx.x;
  const int64_t k = gid / NV;
  const int v = static_cast<int>(gid % NV);
  if (k >= (list ? static_cast<int64_t>(*count) : E)) return;
  const int64_t e = list ? list[k] : k;
  const float* ue = u + (static_cast<int64_t>(v) * E + e) * NLOC;
  double uv[NLOC];
#pragma unroll
  for (int j = 0; j < NLOC; ++j) uv[j] = ue[j];
  const TriGeo G = load_trigeo(geot, e);
  double hw[P];
  order_weights<P>(G.h, hw);
  // own Taylor coefficients at x_0 and element semi-norm
  double a[NK];
  {
    double R[NK];
#pragma unroll
    for (int m = 0; m < NK; ++m) {
      double s = 0.0;
#pragma unroll
      for (int j = 1; j < NLOC; ++j) s = fma(tab->TV[0][m][j], uv[j] - uv[0], s);
      R[m] = s;
    }
    phys_from_ref<P>(G.A, R, a);
  }
  double mom[NMOM<P>];
  cell_moments<P>(G, tab, mom);
  const double n2 = seminorm_mom<P>(a, mom, hw);
  // weights of the cell candidate and the three vertex candidates
  const float* cv = cand + static_cast<int64_t>(v) * Nv * NK;
  const double qb = static_cast<double>(ms.q_beta), rr = static_cast<double>(ms.r);
  auto wfun = [&](double lin, double b2) {
    const double beta = ms.fast_exp ? sqrt(b2) : pow(sqrt(b2), qb);
    const double den = ms.eps_cd + beta;
    return ms.fast_exp ? lin / (den * den) : lin * pow(den, -rr);
  };
  int32_t vtx[3];
#pragma unroll
  for (int l = 0; l < 3; ++l) vtx[l] = cell_vtx[e * 3 + l];
  double wt[4];
  wt[0] = wfun(1.0 - 3.0 * ms.lin_wd, n2);
  double tot = wt[0];
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    double s[NK];
    candidate_at_x0<P>(cv, vtx[l], l, G, s);
    wt[l + 1] = wfun(ms.lin_wd, seminorm_mom<P>(s, mom, hw));
    tot += wt[l + 1];
  }
  double cb[NK], wrest = 0.0;
#pragma unroll
  for (int t = 0; t < NK; ++t) cb[t] = 0.0;
#pragma unroll
  for (int l = 0; l < 3; ++l) {
    double s[NK];
    candidate_at_x0<P>(cv, vtx[l], l, G, s);
    const double om = wt[l + 1] / tot;
    wrest += om;
#pragma unroll
    for (int t = 0; t < NK; ++t) cb[t] = fma(om, s[t], cb[t]);
  }
  // cell means of u_h^e and of V on the volume rule (weights sum to 1/2)
  double mu = 0.0, mv = 0.0;
#pragma unroll 1
  for (int q = 0; q < NQ; ++q) {
    const double xi = tab->xqd[q], eta = tab->yqd[q];
    double uq = 0.0;
#pragma unroll
    for (int j = 0; j < NLOC; ++j) uq = fma(static_cast<double>(tab->B[q][j]), uv[j], uq);
    mu = fma(tab->wqd[q], uq, mu);
    mv = fma(tab->wqd[q], taylor_value0<P>(cb, G.J[0][0] * xi + G.J[0][1] * eta, G.J[1][0] * xi + G.J[1][1] * eta), mv);
  }
  mu *= 2.0;
  mv *= 2.0;
  const double om0 = wt[0] / tot;
  float* oe = out + (static_cast<int64_t>(v) * E + e) * NLOC;
  int node = 0;
#pragma unroll
  for (int jj = 0; jj <= P; ++jj)
#pragma unroll
    for (int ii = 0; ii <= P - jj; ++ii) {
      const double xi = static_cast<double>(ii) / P, eta = static_cast<double>(jj) / P;
      const double V = taylor_value0<P>(cb, G.J[0][0] * xi + G.J[0][1] * eta, G.J[1][0] * xi + G.J[1][1] * eta);
      oe[node] = static_cast<float>(om0 * uv[node] + wrest * mu + V - mv);
      ++node;
    }
}

// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void tri_vertex_kernel(const float* __restrict__ u, float* __restrict__ cand,
                                                         const int32_t* __restrict__ vptr,
                                                         const int32_t* __restrict__ vent,
                                                         const float4* __restrict__ geov,
                                                         const TriTables* __restrict__ tab, int64_t Nv,
                                                         MethodScalars ms) {
  constexpr int NLOC = (P + 1) * (P + 2) / 2, NK = NLOC - 1;
  // XCD-aware order: each XCD walks a contiguous range of vertices, so the
  // cells shared by neighbouring vertex rows are read again from its own L2
  const int64_t i = xcd_block(blockIdx.x, gridDim.x) * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (i >= Nv) return;
  double num[NK], den = 0.0;
#pragma unroll
  for (int k = 0; k < NK; ++k) num[k] = 0.0;
  for (int it = vptr[i]; it < vptr[i + 1]; ++it) {
    const int ent = vent[it];
    const int64_t e = ent >> 2;
    const int lv = ent & 3;
    const float4 ga = geov[2 * e], gb = geov[2 * e + 1];   // A (row major), h_e
    const double A[2][2] = {{static_cast<double>(ga.x), static_cast<double>(ga.y)},
                            {static_cast<double>(ga.z), static_cast<double>(ga.w)}};
    const double h = static_cast<double>(gb.x);
    double uc[NLOC];
    const float* ue = u + e * NLOC;
    const double u0 = static_cast<double>(ue[0]);
#pragma unroll
    for (int j = 0; j < NLOC; ++j) uc[j] = static_cast<double>(ue[j]) - u0;
    double R[NK], H[NK];
#pragma unroll
    for (int m = 0; m < NK; ++m) {
      double s = 0.0;
#pragma unroll
      for (int j = 1; j < NLOC; ++j) s = fma(tab->TV[lv][m][j], uc[j], s);
      R[m] = s;
    }
    phys_from_ref<P>(A, R, H);
    // eq. (pointsnorm) with h of the cell whose polynomial is measured
    double hw[P];
    order_weights<P>(h, hw);
    const double beta0 = h * sqrt(weighted_sq<P>(H, hw));
    const double beta = ms.fast_exp ? beta0 : pow(beta0, static_cast<double>(ms.q_beta));
    const double wt = ms.fast_exp ? 1.0 / ((ms.eps_vd + beta) * (ms.eps_vd + beta))
                                  : pow(ms.eps_vd + beta, -static_cast<double>(ms.r));
    den += wt;
#pragma unroll
    for (int k = 0; k < NK; ++k) num[k] = fma(wt, H[k], num[k]);
  }
  const double inv = 1.0 / den;
#pragma unroll
  for (int k = 0; k < NK; ++k) cand[i * NK + k] = static_cast<float>(num[k] * inv);
}

// ---------------------------------------------------------------------------
constexpr int TRI_EVAL_THREADS = 128;

// OPEN: the mesh has boundary faces (negative neighbour codes)
template <int P, int FLUX, bool OPEN>
__global__ __launch_bounds__(TRI_EVAL_THREADS) void tri_eval_kernel(const float* __restrict__ u, const float* __restrict__ u0,
                                                       float* __restrict__ out, float* __restrict__ gamma_out,
                                                       float* __restrict__ alpha_out, const float* __restrict__ cand,
                                                       const int32_t* __restrict__ cell_vtx,
                                                       const int32_t* __restrict__ nbrf,
                                                       const double* __restrict__ geot,
                                                       const TriTables* __restrict__ tab, int64_t E,
                                                       MethodScalars ms, int mode, float dt, float a0, float b0,
                                                       uint32_t* __restrict__ status) {
  constexpr int NLOC = (P + 1) * (P + 2) / 2, NK = NLOC - 1, NQ = (P + 1) * (P + 1), NG = P + 1;
  constexpr int NV = NVar<FLUX>::value;
  __shared__ float sBf[3][NG][NLOC];
  // per-thread pointwise semi-norm at the volume points (where SC is active)
  __shared__ float s_at[NQ][TRI_EVAL_THREADS];
  const int tid = threadIdx.x;
  for (int t = threadIdx.x; t < 3 * NG * NLOC; t += blockDim.x) {
    const int f = t / (NG * NLOC), g = (t / NLOC) % NG, j = t % NLOC;
    sBf[f][g][j] = tab->Bf[f][g][j];
  }
  __syncthreads();
  // XCD-aware order (the neighbours across the next row of squares then share an L2)
  const int64_t e = xcd_block(blockIdx.x, gridDim.x) * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (e >= E) return;
  const int64_t stride = E * NLOC;
  float uv[NV][NLOC];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int j = 0; j < NLOC; ++j) uv[v][j] = u[v * stride + e * NLOC + j];
  const TriGeo G = load_trigeo(geot, e);
  const double adet = fabs(G.det);
  double hw[P];
  order_weights<P>(G.h, hw);

  // ---- sensor field derivatives at the volume points (float64) ----
  const bool plain = ms.sensor_kind == CVW_SENSOR_PLAIN;
  double a[NK];
  {
    double R[NK];
    const double s0 = static_cast<double>(uv[0][0]);
#pragma unroll
    for (int m = 0; m < NK; ++m) {
      double s = 0.0;
#pragma unroll
      for (int j = 1; j < NLOC; ++j) s = fma(tab->TV[0][m][j], static_cast<double>(uv[0][j]) - s0, s);
      R[m] = s;
    }
    phys_from_ref<P>(G.A, R, a);
  }
  // ---- sensor gamma_e (float64) ----
  double gam = ms.fixed_gammad;
  if (plain) {
    double mu[NMOM<P>];
    cell_moments<P>(G, tab, mu);
    const double n0 = sqrt(seminorm_mom<P>(a, mu, hw));
    const double qb = static_cast<double>(ms.q_beta), rr = static_cast<double>(ms.r);
    double beta[4];
    beta[0] = ms.fast_exp ? n0 : pow(n0, qb);
    int32_t vtx[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) vtx[l] = cell_vtx[e * 3 + l];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      double s[NK];
      candidate_at_x0<P>(cand, vtx[l], l, G, s);
      const double nl = sqrt(seminorm_mom<P>(s, mu, hw));
      beta[l + 1] = ms.fast_exp ? nl : pow(nl, qb);
    }
    double wt[4], tot = 0.0;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const double lin = (l == 0) ? 1.0 - 3.0 * ms.lin_wd : ms.lin_wd;
      const double b = ms.eps_cd + beta[l];
      wt[l] = ms.fast_exp ? lin / (b * b) : lin * pow(b, -rr);
      tot += wt[l];
    }
    double diff[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) diff[k] = 0.0;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
      double s[NK];
      candidate_at_x0<P>(cand, vtx[l], l, G, s);
      const double om = wt[l + 1] / tot;
#pragma unroll
      for (int k = 0; k < NK; ++k) diff[k] = fma(om, a[k] - s[k], diff[k]);
    }
    const double d = sqrt(seminorm_mom<P>(diff, mu, hw));
    if (n0 > 0.0) {
      const double ratio = fmin(1.0, d / n0);
      gam = 1.0 - (ms.q_sensor == 1.0f ? ratio : pow(ratio, static_cast<double>(ms.q_sensor)));
    } else {
      gam = 1.0;
    }
  }
  const float gf = static_cast<float>(gam);

  // ---- float32 geometry, wave speed, viscosity ----
  const float J00 = static_cast<float>(G.J[0][0]), J01 = static_cast<float>(G.J[0][1]);
  const float J10 = static_cast<float>(G.J[1][0]), J11 = static_cast<float>(G.J[1][1]);
  const float A00 = static_cast<float>(G.A[0][0]), A01 = static_cast<float>(G.A[0][1]);
  const float A10 = static_cast<float>(G.A[1][0]), A11 = static_cast<float>(G.A[1][1]);
  const float X0 = static_cast<float>(G.x0), Y0 = static_cast<float>(G.y0);
  const float fdet = static_cast<float>(adet);
  float lam = ms.lam_g;
  if (!(ms.lam_g > 0.0f)) {
    lam = 0.0f;
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
      float uq[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        float s = 0.0f;
#pragma unroll
        for (int j = 0; j < NLOC; ++j) s = fmaf(tab->B[q][j], uv[v][j], s);
        uq[v] = s;
      }
      const float px = X0 + J00 * tab->xq[q] + J01 * tab->yq[q];
      const float py = Y0 + J10 * tab->xq[q] + J11 * tab->yq[q];
      lam = fmaxf(lam, wave_speed<FLUX>(ms, uq, px, py));
    }
  }
  const float nu = lam * static_cast<float>(G.h) / (2.0f * P);

  // ---- shock-capturing weights (eq. alphaq), from the sensor field: the
  // derivatives at the volume points (float64) only in cells where they can
  // be active (a wave whose cells all have gamma_e >= C_gamma skips them) ----
  bool sc_active = false;
  float ratio = 1.0f;
  if (ms.sc_on && gam < ms.c_gammad) {
    float S = 0.0f, T = 0.0f;
#pragma unroll 1
    for (int q = 0; q < NQ; ++q) {
      const double xi = tab->xqd[q], eta = tab->yqd[q];
      double D[NK];
      taylor_eval<P>(a, G.J[0][0] * xi + G.J[0][1] * eta, G.J[1][0] * xi + G.J[1][1] * eta, D);
      const float at = static_cast<float>(G.h * sqrt(weighted_sq<P>(D, hw)));   // eq. (pointsnorm) at x_q
      s_at[q][tid] = at;
      const float f = (1.0f - gf) * static_cast<float>(D[0] * D[0] + D[1] * D[1]);
      const float W = tab->wq[q] * fdet;
      S = fmaf(W, f, S);
      T = fmaf(W * at, f, T);
    }
    sc_active = S > 0.0f && T > 0.0f;
    if (sc_active) ratio = S / T;
  }

  if (mode == MODE_SENSOR) {
    gamma_out[e] = gf;
    if (alpha_out)
      for (int q = 0; q < NQ; ++q) alpha_out[e * NQ + q] = sc_active ? s_at[q][tid] * ratio : 1.0f;
    return;
  }

  // ---- volume terms ----
  float r[NV][NLOC];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int j = 0; j < NLOC; ++j) r[v][j] = 0.0f;
  const float cbase = nu * (1.0f - gf);
#pragma unroll 1
  for (int q = 0; q < NQ; ++q) {
    float uq[NV], ux[NV], uy[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      float s = 0.0f, gx = 0.0f, gy = 0.0f;
#pragma unroll
      for (int j = 0; j < NLOC; ++j) {
        s = fmaf(tab->B[q][j], uv[v][j], s);
        gx = fmaf(tab->Gx[q][j], uv[v][j], gx);
        gy = fmaf(tab->Gy[q][j], uv[v][j], gy);
      }
      uq[v] = s;
      ux[v] = A00 * gx + A10 * gy;
      uy[v] = A01 * gx + A11 * gy;
    }
    const float px = X0 + J00 * tab->xq[q] + J01 * tab->yq[q];
    const float py = Y0 + J10 * tab->xq[q] + J11 * tab->yq[q];
    float fx[NV], fy[NV];
    phys_flux<FLUX>(ms, uq, px, py, fx, fy);
    const float cst = cbase * (sc_active ? s_at[q][tid] * ratio : 1.0f);
    const float W = tab->wq[q] * fdet;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const float Gx = -fx[v] + cst * ux[v], Gy = -fy[v] + cst * uy[v];
      // grad phi_j . G = grad_ref phi_j . (A G)
      const float Hx = W * (A00 * Gx + A01 * Gy), Hy = W * (A10 * Gx + A11 * Gy);
#pragma unroll
      for (int j = 0; j < NLOC; ++j) r[v][j] = fmaf(tab->Gx[q][j], Hx, fmaf(tab->Gy[q][j], Hy, r[v][j]));
    }
  }

  // ---- interface terms: own faces, the neighbour's trace at the reversed points ----
#pragma unroll
  for (int f = 0; f < 3; ++f) {
    const int nb = nbrf[e * 3 + f];
    const bool bnd = OPEN && nb < 0;                   // boundary face: exterior state from its data
    const int64_t en = bnd ? 0 : (nb >> 2);
    const int fn = bnd ? 0 : (nb & 3);
    float un[NV][NLOC];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int j = 0; j < NLOC; ++j) un[v][j] = bnd ? 0.0f : u[v * stride + en * NLOC + j];
    // edge from vertex f to vertex f+1 (vertex 0 at the origin of the map)
    const float ax = (f == 0) ? 0.0f : (f == 1 ? J00 : J01), ay = (f == 0) ? 0.0f : (f == 1 ? J10 : J11);
    const float bx = (f == 0) ? J00 : (f == 1 ? J01 : 0.0f), by = (f == 0) ? J10 : (f == 1 ? J11 : 0.0f);
    const float tx = bx - ax, ty = by - ay;
    const float len = sqrtf(tx * tx + ty * ty);
    const float nx = ty / len, ny = -tx / len;
    const float jf = 0.5f * len;
#pragma unroll
    for (int g = 0; g < NG; ++g) {
      float um[NV], up[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        float sm = 0.0f, sp = 0.0f;
#pragma unroll
        for (int j = 0; j < NLOC; ++j) {
          sm = fmaf(tab->Bf[f][g][j], uv[v][j], sm);
          sp = fmaf(sBf[fn][NG - 1 - g][j], un[v][j], sp);
        }
        um[v] = sm;
        up[v] = sp;
      }
      if (bnd) ghost_state<FLUX>(ms, nb, um, nx, ny, up);
      const float px = X0 + J00 * tab->xf[f][g] + J01 * tab->yf[f][g];
      const float py = Y0 + J10 * tab->xf[f][g] + J11 * tab->yf[f][g];
      float fs[NV];
      num_flux<FLUX>(ms, um, up, nx, ny, px, py, fs);
      const float w = tab->wf[g] * jf;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const float wf = w * fs[v];
#pragma unroll
        for (int j = 0; j < NLOC; ++j) r[v][j] = fmaf(tab->Bf[f][g][j], wf, r[v][j]);
      }
    }
  }

  bool bad = false;
#pragma unroll
  for (int j = 0; j < NLOC; ++j) {
    float nodal[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) nodal[v] = uv[v][j];
    if (!state_admissible<FLUX>(ms, nodal)) bad = true;
  }
  if (bad) atomicOr(status, ST_NONPOSITIVE);
  bool nonfinite = false;
  if (mode == MODE_RESIDUAL) {
    if (gamma_out) gamma_out[e] = gf;
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int j = 0; j < NLOC; ++j) {
        nonfinite = nonfinite || !isfinite(r[v][j]);
        out[v * stride + e * NLOC + j] = r[v][j];
      }
  } else {
    // u_out = a0 u_n + b0 (u - dt M_e^{-1} r), M_e = |det J| M_ref
    const float sc = dt / fdet;
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int j = 0; j < NLOC; ++j) {
        float x = 0.0f;
#pragma unroll
        for (int i = 0; i < NLOC; ++i) x = fmaf(tab->Minv[j][i], r[v][i], x);
        const int64_t idx = v * stride + e * NLOC + j;
        const float base = (a0 != 0.0f) ? a0 * u0[idx] : 0.0f;
        const float o = base + b0 * (uv[v][j] - sc * x);
        nonfinite = nonfinite || !isfinite(o);
        out[idx] = o;
      }
  }
  if (nonfinite) atomicOr(status, ST_NONFINITE);
}

// ---------------------------------------------------------------------------
// float64 totals sum_e int_{K_e} u_h = sum_e |det J_e| sum_j m_j u_j, fixed-order
// reductions (grid-stride thread partials, block tree, then one block)
constexpr int TRI_TOT_BLOCKS = 512;

template <int NLOC>
__global__ __launch_bounds__(256) void tri_totals_partial(const float* __restrict__ u,
                                                          const double* __restrict__ geot,
                                                          const TriTables* __restrict__ tab,
                                                          double* __restrict__ part, int64_t E) {
  __shared__ double sh[256];
  const int v = blockIdx.y;
  double acc = 0.0;
  for (int64_t e = blockIdx.x * 256 + threadIdx.x; e < E; e += static_cast<int64_t>(TRI_TOT_BLOCKS) * 256) {
    const double* g = geot + e * 8;
    const double det = fabs(g[2] * g[5] - g[4] * g[3]);
    double s = 0.0;
    for (int j = 0; j < NLOC; ++j)
      s += static_cast<double>(tab->mvec[j]) * static_cast<double>(u[(v * E + e) * NLOC + j]);
    acc += det * s;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[v * TRI_TOT_BLOCKS + blockIdx.x] = sh[0];
}

__global__ __launch_bounds__(256) void tri_totals_final(const double* __restrict__ part, double* __restrict__ out) {
  __shared__ double sh[256];
  const int v = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < TRI_TOT_BLOCKS; i += 256) acc += part[v * TRI_TOT_BLOCKS + i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[v] = sh[0];
}

// ---------------------------------------------------------------------------
static unsigned nblk(int64_t n, int t) { return static_cast<unsigned>((n + t - 1) / t); }
// block count rounded up to a multiple of 8 (the XCD-aware kernels; the extra blocks exit)
static unsigned nblk8(int64_t n, int t) { return (nblk(n, t) + 7u) / 8u * 8u; }

cvw_status tri_candidates(const cvw_mesh* m, const cvw_params* prm, const float* u, float* cand, hipStream_t s) {
  const MethodScalars ms = make_scalars(prm);
  const dim3 g(nblk8(m->Nv, 256)), b(256);
  switch (m->degree) {
    case 1: hipLaunchKernelGGL(tri_vertex_kernel<1>, g, b, 0, s, u, cand, m->d_vtx_ptr, m->d_vtx_ent, reinterpret_cast<const float4*>(m->d_geov), m->d_trit, m->Nv, ms); break;
    case 2: hipLaunchKernelGGL(tri_vertex_kernel<2>, g, b, 0, s, u, cand, m->d_vtx_ptr, m->d_vtx_ent, reinterpret_cast<const float4*>(m->d_geov), m->d_trit, m->Nv, ms); break;
    case 3: hipLaunchKernelGGL(tri_vertex_kernel<3>, g, b, 0, s, u, cand, m->d_vtx_ptr, m->d_vtx_ent, reinterpret_cast<const float4*>(m->d_geov), m->d_trit, m->Nv, ms); break;
    default: set_error("degree not supported on the GPU path"); return CVW_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

template <int P, int FLUX>
static void launch_eval(const cvw_mesh* m, const MethodScalars& ms, int mode, const float* u, const float* u0,
                        float* out, float* gamma, float* alpha, const float* cand, uint32_t* status, float dt,
                        float a0, float b0, hipStream_t s) {
  auto kern = m->closed ? tri_eval_kernel<P, FLUX, false> : tri_eval_kernel<P, FLUX, true>;
  hipLaunchKernelGGL(kern, dim3(nblk8(m->E, TRI_EVAL_THREADS)), dim3(TRI_EVAL_THREADS), 0, s, u, u0, out, gamma, alpha,
                     cand, m->d_cell_vtx, m->d_nbrf, m->d_geot, m->d_trit, m->E, ms, mode, dt, a0, b0, status);
}

template <int P>
static cvw_status eval_flux(const cvw_mesh* m, const MethodScalars& ms, int flux, int mode, const float* u,
                            const float* u0, float* out, float* gamma, float* alpha, const float* cand,
                            uint32_t* status, float dt, float a0, float b0, hipStream_t s) {
  switch (flux) {
    case CVW_ADVECT_CONST: launch_eval<P, CVW_ADVECT_CONST>(m, ms, mode, u, u0, out, gamma, alpha, cand, status, dt, a0, b0, s); break;
    case CVW_ADVECT_ROT: launch_eval<P, CVW_ADVECT_ROT>(m, ms, mode, u, u0, out, gamma, alpha, cand, status, dt, a0, b0, s); break;
    case CVW_BURGERS: launch_eval<P, CVW_BURGERS>(m, ms, mode, u, u0, out, gamma, alpha, cand, status, dt, a0, b0, s); break;
    case CVW_KPP: launch_eval<P, CVW_KPP>(m, ms, mode, u, u0, out, gamma, alpha, cand, status, dt, a0, b0, s); break;
    case CVW_EULER: launch_eval<P, CVW_EULER>(m, ms, mode, u, u0, out, gamma, alpha, cand, status, dt, a0, b0, s); break;
    default: set_error("unknown flux"); return CVW_EINVAL;
  }
  return CVW_OK;
}

cvw_status tri_eval(const cvw_mesh* m, const cvw_params* prm, int mode, const float* u, const float* u0, float* out,
                    float* gamma, float* alpha, const float* cand, uint32_t* status, float dt, float a0, float b0,
                    hipStream_t s) {
  const MethodScalars ms = make_scalars(prm);
  cvw_status st;
  switch (m->degree) {
    case 1: st = eval_flux<1>(m, ms, prm->flux, mode, u, u0, out, gamma, alpha, cand, status, dt, a0, b0, s); break;
    case 2: st = eval_flux<2>(m, ms, prm->flux, mode, u, u0, out, gamma, alpha, cand, status, dt, a0, b0, s); break;
    case 3: st = eval_flux<3>(m, ms, prm->flux, mode, u, u0, out, gamma, alpha, cand, status, dt, a0, b0, s); break;
    default: set_error("degree not supported on the GPU path"); return CVW_EUNSUPPORTED;
  }
  if (st != CVW_OK) return st;
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

cvw_status tri_limit(const cvw_mesh* m, const cvw_params* prm, const float* u, float* out, const float* cand,
                     const uint32_t* count, const int32_t* list, hipStream_t s) {
  const MethodScalars ms = make_scalars(prm);
  const int nv = prm->flux == CVW_EULER ? 4 : 1;
  const dim3 g(nblk(m->E * nv, 256)), b(256);
#define CVW_TRI_LIMIT(P)                                                                                            \
  if (nv == 4)                                                                                                      \
    hipLaunchKernelGGL((tri_limit_kernel<P, 4>), g, b, 0, s, u, out, cand, count, list, m->d_cell_vtx, m->d_geot,   \
                       m->d_trit, m->E, m->Nv, ms);                                                                 \
  else                                                                                                              \
    hipLaunchKernelGGL((tri_limit_kernel<P, 1>), g, b, 0, s, u, out, cand, count, list, m->d_cell_vtx, m->d_geot,   \
                       m->d_trit, m->E, m->Nv, ms);
  switch (m->degree) {
    case 1: CVW_TRI_LIMIT(1) break;
    case 2: CVW_TRI_LIMIT(2) break;
    case 3: CVW_TRI_LIMIT(3) break;
    default: set_error("degree not supported on the GPU path"); return CVW_EUNSUPPORTED;
  }
#undef CVW_TRI_LIMIT
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

cvw_status tri_totals(const cvw_mesh* m, int nvar, const float* u, double* partial, double* out_dev, hipStream_t s) {
  const dim3 g(TRI_TOT_BLOCKS, nvar), b(256);
  switch (m->degree) {
    case 1: hipLaunchKernelGGL(tri_totals_partial<3>, g, b, 0, s, u, m->d_geot, m->d_trit, partial, m->E); break;
    case 2: hipLaunchKernelGGL(tri_totals_partial<6>, g, b, 0, s, u, m->d_geot, m->d_trit, partial, m->E); break;
    case 3: hipLaunchKernelGGL(tri_totals_partial<10>, g, b, 0, s, u, m->d_geot, m->d_trit, partial, m->E); break;
    default: set_error("degree not supported on the GPU path"); return CVW_EUNSUPPORTED;
  }
  hipLaunchKernelGGL(tri_totals_final, dim3(nvar), dim3(256), 0, s, partial, out_dev);
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

}  // namespace cvw
