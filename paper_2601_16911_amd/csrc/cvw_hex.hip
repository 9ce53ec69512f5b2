// DG on hexahedra (Q_1, Q_2 on congruent axis-aligned boxes, Gauss nodes):
//
//  * hex_vertex_kernel -- one thread per mesh vertex: the Hermite data
//    D^k u^e(x_i), 1 <= |k| <= p, of each of the eight cells of the vertex
//    patch (eq. taylorsol) by one-dimensional passes with the derivatives of
//    the Lagrange basis at the cell ends, the pointwise smoothness indicators
//    and Jiang-Shu weights, and the vertex candidate (eq. taylorcand), Sec.
//    3.2.  Float64.
//  * hex_sensor_kernel -- one thread per cell: the cell-vertex WENO sensor
//    (eq. finalweno, eq. gamma).
//  * hex_eval_kernel -- a team of lanes per cell, one lane per node (8 lanes
//    for Q_1, 27 of 32 for Q_2): the viscosity (eq. lostab), the
//    shock-capturing weights (eqs. dissrateorig to alphaq), the volume and
//    interface terms of the DG residual in float32, and optionally the
//    Runge-Kutta stage update with the exact (diagonal, Gauss-collocated)
//    element mass; scalar laws and the Euler equations (HLL at the faces,
//    the sensor field and the SC weights from the density).
//
// The sensor works in the monomials xi^A of the cell's reference coordinates
// about its centre: the cell polynomial (its nodal values less the first one,
// so that constant data gives exact zeros) and the eight vertex candidates
// (Taylor polynomials about the corners, re-expanded about the centre) are
// coefficient vectors, and every element semi-norm of eq. snorm is the
// quadratic form of one Gram matrix of the monomials (exact integrals, built
// on the host for the mesh's box; nonzero only between monomials whose
// exponents have equal parity in every direction).  The cell pass's team
// exchanges nodal values and quadrature terms through LDS and reduces with
// cross-lane shuffles; idle lanes of a Q_2 team carry zeros.
#include "cvw_device.h"
#include "cvw_cells3d.h"

namespace cvw {

template <int P>
struct HexShape {
  static constexpr int N1 = P + 1, NL = N1 * N1 * N1, NK = (P + 1) * (P + 2) * (P + 3) / 6 - 1;
  static constexpr int TEAM = NL <= 8 ? 8 : 32;      // lanes per cell, a power of two within a wavefront
  static constexpr int CPB = 256 / TEAM;             // cells per block of 256 threads
};

// Team reductions: the butterfly of the row reductions (quad pairs, the
// mirrored lane of the other quad, of the other half row) over 8 or 16 lanes,
// then the other row of a 32-lane team; every lane of the team receives
// bitwise the same value.
template <int TEAM>
__device__ __forceinline__ float team_sumf(float x) {
#pragma clang fp contract(off)
  x = x + dpp<(1 | (0 << 2) | (3 << 4) | (2 << 6))>(x);
  x = x + dpp<(2 | (3 << 2) | (0 << 4) | (1 << 6))>(x);
  x = x + dpp<0x141>(x);
  if constexpr (TEAM >= 16) x = x + dpp<0x140>(x);
  if constexpr (TEAM >= 32) x = x + __shfl_xor(x, 16);
  return x;
}
template <int TEAM>
__device__ __forceinline__ float team_maxf(float x) {
  x = fmaxf(x, dpp<(1 | (0 << 2) | (3 << 4) | (2 << 6))>(x));
  x = fmaxf(x, dpp<(2 | (3 << 2) | (0 << 4) | (1 << 6))>(x));
  x = fmaxf(x, dpp<0x141>(x));
  if constexpr (TEAM >= 16) x = fmaxf(x, dpp<0x140>(x));
  if constexpr (TEAM >= 32) x = fmaxf(x, __shfl_xor(x, 16));
  return x;
}

// A team lives inside one wavefront and its LDS slots are its own: an
// exchange needs only the wavefront's LDS operations kept in program order
// (they complete in issue order), not a workgroup barrier.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// scalar fluxes in 3D: f_d(u) = v_d u (constant advection) or u^2 / 2 b_d (Burgers)
template <int FLUX>
__device__ __forceinline__ float hex_flux(const MethodScalars& ms, float u, int d) {
  if constexpr (FLUX == CVW_BURGERS) return 0.5f * u * u * ms.fp[d];
  else return ms.fp[d] * u;
}
template <int FLUX>
__device__ __forceinline__ float hex_speed(const MethodScalars& ms, float u) {
  const float vn = fsqrt(ms.fp[0] * ms.fp[0] + ms.fp[1] * ms.fp[1] + ms.fp[2] * ms.fp[2]);
  if constexpr (FLUX == CVW_BURGERS) return fabsf(u) * vn;
  else return vn;
}

// Variables per node: one for the scalar laws, (rho, m_x, m_y, m_z, E) for
// the Euler equations (gas gamma = fp[0])
template <int FLUX>
struct HexNV {
  static constexpr int value = FLUX == CVW_EULER ? 5 : 1;
};

// local maximum wave speed (Euler: |v| + c)
template <int FLUX>
__device__ __forceinline__ float hex_speed_all(const MethodScalars& ms, const float* u) {
  if constexpr (FLUX == CVW_EULER) {
    const float inv = frcp(u[0]);
    const float v2 = (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) * inv * inv;
    const float p = (ms.fp[0] - 1.0f) * (u[4] - 0.5f * u[0] * v2);
    return fsqrt(v2) + fsqrt(fmaxf(ms.fp[0] * p * inv, 0.0f));
  } else {
    return hex_speed<FLUX>(ms, u[0]);
  }
}

// interface flux f*(u-, u+; n), n = sg e_d: local Lax-Friedrichs for the
// scalar laws, HLL with Davis wave-speed estimates for the Euler equations
template <int FLUX>
__device__ __forceinline__ void hex_num_flux(const MethodScalars& ms, const float* um, const float* up, int d,
                                             float sg, float* fs) {
  if constexpr (FLUX == CVW_EULER) {
    const float g = ms.fp[0];
    const float im = frcp(um[0]), ip = frcp(up[0]);
    const float vdm = um[1 + d] * im, vdp = up[1 + d] * ip;
    const float pm = (g - 1.0f) * (um[4] - 0.5f * (um[1] * um[1] + um[2] * um[2] + um[3] * um[3]) * im);
    const float pp = (g - 1.0f) * (up[4] - 0.5f * (up[1] * up[1] + up[2] * up[2] + up[3] * up[3]) * ip);
    const float vm = sg * vdm, vp = sg * vdp;
    const float cm = fsqrt(fmaxf(g * pm * im, 0.0f)), cp = fsqrt(fmaxf(g * pp * ip, 0.0f));
    const float SL = fminf(vm - cm, vp - cp);
    const float SR = fmaxf(vm + cm, vp + cp);
    float Fm[5], Fp[5];
    Fm[0] = um[0] * vm;
    Fp[0] = up[0] * vp;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      Fm[1 + a] = um[1 + a] * vm + (a == d ? sg * pm : 0.0f);
      Fp[1 + a] = up[1 + a] * vp + (a == d ? sg * pp : 0.0f);
    }
    Fm[4] = (um[4] + pm) * vm;
    Fp[4] = (up[4] + pp) * vp;
    const float inv = frcp(SR - SL);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const float mid = (SR * Fm[v] - SL * Fp[v] + SL * SR * (up[v] - um[v])) * inv;
      fs[v] = (SL >= 0.0f) ? Fm[v] : ((SR <= 0.0f) ? Fp[v] : mid);
    }
  } else {
    float lf = ms.lam_g;
    if (!(lf > 0.0f)) {
      if constexpr (FLUX == CVW_BURGERS) lf = fmaxf(fabsf(um[0]), fabsf(up[0])) * fabsf(ms.fp[d]);
      else lf = fabsf(ms.fp[d]);
    }
    fs[0] = 0.5f * sg * (hex_flux<FLUX>(ms, um[0], d) + hex_flux<FLUX>(ms, up[0], d)) - 0.5f * lf * (up[0] - um[0]);
  }
}

// ---------------------------------------------------------------------------
// vertex pass
// ---------------------------------------------------------------------------
// The multi-indices 1 <= |k| <= P in the order of the Hermite data (by |k|,
// then decreasing first, then decreasing second component) and the index of
// the monomial xi^k among the cell's monomials.
template <int P>
struct HexKSet {
  static constexpr int N1 = P + 1, NK = (P + 1) * (P + 2) * (P + 3) / 6 - 1;
  int x[NK], y[NK], z[NK], mono[NK];
  constexpr HexKSet() : x{}, y{}, z{}, mono{} {
    int t = 0;
    for (int n = 1; n <= P; ++n)
      for (int a = n; a >= 0; --a)
        for (int b = n - a; b >= 0; --b) {
          x[t] = a;
          y[t] = b;
          z[t] = n - a - b;
          mono[t] = a + N1 * (b + N1 * (n - a - b));
          ++t;
        }
  }
};
template <int P>
inline constexpr HexKSet<P> hex_kset{};

template <int P>
__global__ __launch_bounds__(256) void hex_vertex_kernel(const float* __restrict__ u, float* __restrict__ cand,
                                                         const int32_t* __restrict__ vent,
                                                         const HexTables* __restrict__ tab, int64_t Nv,
                                                         MethodScalars ms) {
  using S = HexShape<P>;
  constexpr int N1 = S::N1, NL = S::NL, NK = S::NK;
  constexpr HexKSet<P> ks = hex_kset<P>;
  const int64_t v = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (v >= Nv) return;
  // the patch in octant order: entry 8 v + l is the cell whose corner l is v
  const int4 ea = reinterpret_cast<const int4*>(vent + v * 8)[0];
  const int4 eb = reinterpret_cast<const int4*>(vent + v * 8)[1];
  const int32_t ent[8] = {ea.x, ea.y, ea.z, ea.w, eb.x, eb.y, eb.z, eb.w};
  double acc[NK], wsum = 0.0;
#pragma unroll
  for (int k = 0; k < NK; ++k) acc[k] = 0.0;
  float un[NL];
#pragma unroll
  for (int j = 0; j < NL; ++j) un[j] = u[static_cast<int64_t>(ent[0] >> 3) * NL + j];
  // one corner per iteration (the same corner across the wavefront, so the
  // end-value tables are read through the scalar unit); the next patch cell's
  // values are requested before the current one is used
#pragma unroll 1
  for (int l = 0; l < 8; ++l) {
    float uc[NL];
#pragma unroll
    for (int j = 0; j < NL; ++j) uc[j] = un[j];
    const int64_t cn = ent[l < 7 ? l + 1 : 7] >> 3;
#pragma unroll
    for (int j = 0; j < NL; ++j) un[j] = u[cn * NL + j];
    // corner signs of local vertex l: x+ for l = 1, 2, 5, 6; y+ for 2, 3, 6, 7; z+ for 4..7
    const int sx = (l ^ (l >> 1)) & 1, sy = (l >> 1) & 1, sz = (l >> 2) & 1;
    const double u0 = static_cast<double>(uc[0]);
    // D^k u at the corner, one direction at a time: X[m][b][c] = sum_a l_a^{(m)}(s_x) u_abc,
    // Y[mx][my][c] = sum_b l_b^{(my)}(s_y) X[mx][b][c], D = sum_c l_c^{(mz)}(s_z) Y[mx][my][c]
    double X[N1][N1][N1];
#pragma unroll
    for (int b = 0; b < N1; ++b)
#pragma unroll
      for (int c = 0; c < N1; ++c) {
        double r[N1];
#pragma unroll
        for (int a = 0; a < N1; ++a) r[a] = static_cast<double>(uc[a + N1 * (b + N1 * c)]) - u0;
#pragma unroll
        for (int m = 0; m < N1; ++m) {
          double s = 0.0;
#pragma unroll
          for (int a = 0; a < N1; ++a) s = fma(tab->E1[m][sx][a], r[a], s);
          X[m][b][c] = s;
        }
      }
    double Y[N1][N1][N1];
#pragma unroll
    for (int mx = 0; mx < N1; ++mx)
#pragma unroll
      for (int my = 0; mx + my < N1; ++my)
#pragma unroll
        for (int c = 0; c < N1; ++c) {
          double s = 0.0;
#pragma unroll
          for (int b = 0; b < N1; ++b) s = fma(tab->E1[my][sy][b], X[mx][b][c], s);
          Y[mx][my][c] = s;
        }
    double H[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < N1; ++c) s = fma(tab->E1[ks.z[k]][sz][c], Y[ks.x[k]][ks.y[k]][c], s);
      H[k] = s * tab->hk[k];
    }
    double b2 = 0.0;
#pragma unroll
    for (int k = 0; k < NK; ++k) b2 = fma(tab->hb[k] * H[k], H[k], b2);
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
    for (int k = 0; k < NK; ++k) acc[k] = fma(w, H[k], acc[k]);
    wsum += w;
  }
  const double iw = 1.0 / wsum;
#pragma unroll
  for (int k = 0; k < NK; ++k) cand[v * NK + k] = static_cast<float>(acc[k] * iw);
}

// ---------------------------------------------------------------------------
// cell pass
// ---------------------------------------------------------------------------
// alpha~^2 at node (ta, tb, tc) (eq. alpha_prelim with the pointwise
// semi-norm): sum_k h_e^{2|k|} |D^k u|^2 over 1 <= |k| <= p, from the
// reference first derivatives g (already at the node) and, for p = 2, the
// second derivatives along the node's lines (l'' at the nodes) and across
// them (l' x l'); wa folds h_e^{2|k|} and the factors (2/h_d)^{2 k_d}.
template <int P>
__device__ __forceinline__ float hex_atil2(const HexTables* __restrict__ tab, const float* su, int ta, int tb, int tc,
                                           const float (&g)[3]) {
  constexpr int N1 = P + 1;
  float a2 = tab->wa[0] * g[0] * g[0] + tab->wa[1] * g[1] * g[1] + tab->wa[2] * g[2] * g[2];
  if constexpr (P == 2) {
    float xx = 0.0f, yy = 0.0f, zz = 0.0f, xy = 0.0f, xz = 0.0f, yz = 0.0f;
#pragma unroll
    for (int i = 0; i < N1; ++i) {
      xx = fmaf(tab->D2[ta][i], su[i + N1 * (tb + N1 * tc)], xx);
      yy = fmaf(tab->D2[tb][i], su[ta + N1 * (i + N1 * tc)], yy);
      zz = fmaf(tab->D2[tc][i], su[ta + N1 * (tb + N1 * i)], zz);
#pragma unroll
      for (int j = 0; j < N1; ++j) {
        xy = fmaf(tab->D1[ta][i] * tab->D1[tb][j], su[i + N1 * (j + N1 * tc)], xy);
        xz = fmaf(tab->D1[ta][i] * tab->D1[tc][j], su[i + N1 * (tb + N1 * j)], xz);
        yz = fmaf(tab->D1[tb][i] * tab->D1[tc][j], su[ta + N1 * (i + N1 * j)], yz);
      }
    }
    // multi-index order (2,0,0), (1,1,0), (1,0,1), (0,2,0), (0,1,1), (0,0,2)
    a2 = fmaf(tab->wa[3] * xx, xx, a2);
    a2 = fmaf(tab->wa[4] * xy, xy, a2);
    a2 = fmaf(tab->wa[5] * xz, xz, a2);
    a2 = fmaf(tab->wa[6] * yy, yy, a2);
    a2 = fmaf(tab->wa[7] * yz, yz, a2);
    a2 = fmaf(tab->wa[8] * zz, zz, a2);
  }
  return a2;
}

// monomials A, B (index a + n1 b + n1^2 c) with exponents of equal parity in
// every direction: the only pairs where the semi-norm Gram matrix can be
// nonzero (the reference cell is symmetric about its centre)
template <int N1>
constexpr bool hex_pair(int A, int B) {
  return ((A % N1 + B % N1) % 2 == 0) && (((A / N1) % N1 + (B / N1) % N1) % 2 == 0) &&
         ((A / (N1 * N1) + B / (N1 * N1)) % 2 == 0);
}

// c^T G c for the coefficients c of monomials MONO[0..N) (row and column of
// the constant vanish); G is read with compile-time offsets, i.e. through the
// scalar unit
template <int N1, int N, typename IDX>
__device__ __forceinline__ double hex_quad(const double (&c)[N], IDX mono, const HexTables* __restrict__ tab) {
  double q = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const int A = mono(i);
    if (A == 0) continue;
    double t = 0.0;
#pragma unroll
    for (int j = i + 1; j < N; ++j) {
      const int B = mono(j);
      if (B == 0 || !hex_pair<N1>(A, B)) continue;
      t = fma(tab->G[A][B], c[j], t);
    }
    q = fma(c[i], fma(2.0, t, tab->G[A][A] * c[i]), q);
  }
  return q;
}

// Jiang-Shu weight of a candidate with semi-norm b and linear weight lin
__device__ __forceinline__ float hex_weight(const MethodScalars& ms, float lin, float b) {
  if (ms.fast_exp) {
    const float tt = ms.eps_c + b;
    return lin / (tt * tt);
  }
  return lin * powf(ms.eps_c + powf(b, ms.q_beta), -ms.r);
}

// Sensor pass: one thread per cell.  The block's nodal values are staged
// through LDS (coalesced reads); each thread then works in registers: the
// monomial coefficients of its cell (three one-dimensional passes), their
// semi-norm, the eight vertex candidates re-expanded about the centre one at
// a time (their semi-norms, weights and weighted sum), the difference
// u_h - u_h^{e,*} and its semi-norm, gamma_e (eq. finalweno, eq. gamma).
// Coefficients, re-expansions and quadratic forms in float64; the weights,
// square roots and the ratio in float32 (relative rounding 1e-7 in gamma_e).
template <int P>
__global__ __launch_bounds__(256) void hex_sensor_kernel(const float* __restrict__ u, float* __restrict__ gamma,
                                                         const float* __restrict__ cand,
                                                         const int32_t* __restrict__ cell_vtx,
                                                         const HexTables* __restrict__ tab, int64_t E,
                                                         MethodScalars ms) {
  using S = HexShape<P>;
  constexpr int N1 = S::N1, NL = S::NL, NK = S::NK;
  constexpr HexKSet<P> ks = hex_kset<P>;
  __shared__ float su[256 * NL];
  const int64_t base = static_cast<int64_t>(blockIdx.x) * 256;
  const int64_t ncell = E - base < 256 ? E - base : 256;
  for (int64_t i = threadIdx.x; i < ncell * NL; i += 256) su[i] = u[base * NL + i];
  __syncthreads();
  if (threadIdx.x >= ncell) return;
  const int64_t e = base + threadIdx.x;
  const int4 va = reinterpret_cast<const int4*>(cell_vtx + e * 8)[0];
  const int4 vb = reinterpret_cast<const int4*>(cell_vtx + e * 8)[1];
  const int32_t vid[8] = {va.x, va.y, va.z, va.w, vb.x, vb.y, vb.z, vb.w};

  // monomial coefficients of u - u_0 (node 0's value: constants give exact zeros)
  double c[NL];
  {
    const float* ue = su + threadIdx.x * NL;     // stride NL (odd for p = 2): no bank conflicts
    const double u00 = static_cast<double>(ue[0]);
    c[0] = 0.0;
#pragma unroll
    for (int j = 1; j < NL; ++j) c[j] = static_cast<double>(ue[j]) - u00;
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {                  // x, then y, then z
    const int st = d == 0 ? 1 : (d == 1 ? N1 : N1 * N1);
#pragma unroll
    for (int r = 0; r < NL / N1; ++r) {
      const int b0 = d == 0 ? r * N1 : (d == 1 ? (r % N1) + N1 * N1 * (r / N1) : r);
      double in[N1];
#pragma unroll
      for (int j = 0; j < N1; ++j) in[j] = c[b0 + st * j];
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        double v = 0.0;
#pragma unroll
        for (int j = 0; j < N1; ++j) v = fma(tab->T1[a][j], in[j], v);
        c[b0 + st * a] = v;
      }
    }
  }
  const double n02 = hex_quad<N1>(c, [](int i) { return i; }, tab);

  // the eight vertex candidates, re-expanded about the centre
  double acc[NK];
#pragma unroll
  for (int a = 0; a < NK; ++a) acc[a] = 0.0;
  float wv = 0.0f;
  double wvd = 0.0;
  // one vertex per iteration (a rolled loop: one copy of the quadratic form
  // and of the weight); the next vertex's candidate is requested before the
  // current one is used
  float cn[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) cn[k] = cand[static_cast<int64_t>(vid[0]) * NK + k];
#pragma unroll 1
  for (int l = 0; l < 8; ++l) {
    float cl[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) cl[k] = cn[k];
    const int32_t vn = vid[l < 7 ? l + 1 : 7];
#pragma unroll
    for (int k = 0; k < NK; ++k) cn[k] = cand[static_cast<int64_t>(vn) * NK + k];
    double sl[NK];
#pragma unroll
    for (int a = 0; a < NK; ++a) {
      double v = 0.0;
#pragma unroll
      for (int k = 0; k < NK; ++k)
        if (ks.x[k] >= ks.x[a] && ks.y[k] >= ks.y[a] && ks.z[k] >= ks.z[a])
          v = fma(tab->R[l][a][k], static_cast<double>(cl[k]), v);
      sl[a] = v;
    }
    const double b2 = hex_quad<N1>(sl, [](int i) { return hex_kset<P>.mono[i]; }, tab);
    const float w = hex_weight(ms, ms.lin_w, fsqrt(static_cast<float>(fmax(b2, 0.0))));
    wv += w;
    wvd += static_cast<double>(w);
#pragma unroll
    for (int a = 0; a < NK; ++a) acc[a] = fma(static_cast<double>(w), sl[a], acc[a]);
  }
  const float n0 = fsqrt(static_cast<float>(fmax(n02, 0.0)));
  const float wsum = hex_weight(ms, 1.0f - 8.0f * ms.lin_w, n0) + wv;
  // u_h - u_h^{e,*} = sum_{l >= 1} omega_l (u_h - s_l), omega_l = w_l / sum w
  const double iw = 1.0 / static_cast<double>(wsum);
  const double osum = wvd * iw;
#pragma unroll
  for (int A = 0; A < NL; ++A) c[A] *= osum;
#pragma unroll
  for (int a = 0; a < NK; ++a) c[ks.mono[a]] = fma(-iw, acc[a], c[ks.mono[a]]);
  const double d2 = hex_quad<N1>(c, [](int i) { return i; }, tab);
  float gam = 1.0f;
  if (n02 > 0.0) {
    float ratio = fminf(1.0f, fsqrt(static_cast<float>(fmax(d2, 0.0))) / n0);
    if (!ms.fast_exp) ratio = powf(ratio, ms.q_sensor);
    gam = 1.0f - ratio;
  }
  gamma[e] = gam;
}

template <int P, int FLUX>
__global__ __launch_bounds__(256) void hex_eval_kernel(const float* __restrict__ u, const float* __restrict__ u0,
                                                       float* __restrict__ out, float* __restrict__ gamma_out,
                                                       float* __restrict__ alpha_out,
                                                       const float* __restrict__ gamma_in,
                                                       const int32_t* __restrict__ nbr,
                                                       const HexTables* __restrict__ tab, int64_t E, int64_t nblk,
                                                       MethodScalars ms, int mode, float dt, float a0, float b0,
                                                       uint32_t* __restrict__ status) {
  using S = HexShape<P>;
  constexpr int N1 = S::N1, NL = S::NL, TEAM = S::TEAM, CPB = S::CPB, NV = HexNV<FLUX>::value;
  __shared__ float su[CPB][NV][NL];
  __shared__ float sn[CPB][6][NV][NL];
  __shared__ float sv[CPB][3][NL];
  // systems: the weighted flux at every face point of the cell, item f NP + pq
  constexpr int NP = N1 * N1, NI = 6 * NP;
  __shared__ float sf[CPB][NV > 1 ? NV : 1][NV > 1 ? NI : 1];
  const int slot = threadIdx.x / TEAM, t = threadIdx.x % TEAM;
  const bool lane_on = t < NL;
  const int tn = lane_on ? t : 0;
  const int ta = tn % N1, tb = (tn / N1) % N1, tc = tn / (N1 * N1);
  const float W = tab->w1[ta] * tab->w1[tb] * tab->w1[tc] * tab->W0;
  // the lane's rows and columns of the tables, in registers for the whole loop
  // (the loop's wavefront fences keep the compiler from hoisting these loads)
  float dr[3][N1], dc[3][N1], lw[3][2], le[3][2];
#pragma unroll
  for (int j = 0; j < N1; ++j) {
    dr[0][j] = tab->D1[ta][j];
    dr[1][j] = tab->D1[tb][j];
    dr[2][j] = tab->D1[tc][j];
    dc[0][j] = tab->D1[j][ta];
    dc[1][j] = tab->D1[j][tb];
    dc[2][j] = tab->D1[j][tc];
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int ad = d == 0 ? ta : (d == 1 ? tb : tc);
    const float wt = d == 0 ? tab->w1[tb] * tab->w1[tc] : (d == 1 ? tab->w1[ta] * tab->w1[tc] : tab->w1[ta] * tab->w1[tb]);
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      lw[d][s] = tab->Lend[s][ad] * wt * tab->Jf[d];
      le[d][s] = tab->Lend[s][ad];
    }
  }
  const bool plain = ms.sensor_kind != CVW_SENSOR_FIXED;
  bool nonfinite = false;
  // software pipeline: the next block's nodal values, gamma_e and neighbour
  // ids are requested at the top of an iteration, the neighbours' nodal
  // values half-way through (clamped, unconditional loads, so that no wait
  // sits at the load); variable v of cell e at (v E + e) NL
  float pu[NV], pg = 0.0f, pn[6][NV];
  int32_t pid[6];
  auto fetch_a = [&](int64_t b) {
    const int64_t ec = b * CPB + slot < E ? b * CPB + slot : E - 1;
#pragma unroll
    for (int v = 0; v < NV; ++v) pu[v] = u[(v * E + ec) * NL + tn];
    pg = plain ? gamma_in[ec] : ms.fixed_gamma;
#pragma unroll
    for (int f = 0; f < 6; ++f) pid[f] = nbr[ec * 6 + f];
  };
  auto fetch_b = [&]() {
#pragma unroll
    for (int f = 0; f < 6; ++f)
#pragma unroll
      for (int v = 0; v < NV; ++v) pn[f][v] = u[(v * E + pid[f]) * NL + tn];
  };
  fetch_a(blockIdx.x);
  fetch_b();
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t e = blk * CPB + slot;
    const bool cell_on = e < E;
    const bool on = lane_on && cell_on;
    // ---- nodal values of the cell and of its six face neighbours
    float uv[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) uv[v] = on ? pu[v] : 0.0f;
    const float gam = pg;                // gamma_e: from the sensor pass, or the fixed value
    if (lane_on) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        su[slot][v][t] = uv[v];
#pragma unroll
        for (int f = 0; f < 6; ++f) sn[slot][f][v][t] = on ? pn[f][v] : 0.0f;
      }
    }
    wave_sync();
    const int64_t nxt = blk + gridDim.x < nblk ? blk + gridDim.x : blk;
    fetch_a(nxt);

    // ---- viscosity (eq. lostab) and the physical gradient of the sensor field at the node
    float lam = ms.lam_g;
    if (!(lam > 0.0f)) lam = team_maxf<TEAM>(on ? hex_speed_all<FLUX>(ms, uv) : 0.0f);
    const float nu = lam * tab->nuf;
    float gr[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < N1; ++j) {
      gr[0] = fmaf(dr[0][j], su[slot][0][j + N1 * (tb + N1 * tc)], gr[0]);
      gr[1] = fmaf(dr[1][j], su[slot][0][ta + N1 * (j + N1 * tc)], gr[1]);
      gr[2] = fmaf(dr[2][j], su[slot][0][ta + N1 * (tb + N1 * j)], gr[2]);
    }
    fetch_b();
    const float gref[3] = {gr[0], gr[1], gr[2]};      // reference derivatives
#pragma unroll
    for (int d = 0; d < 3; ++d) gr[d] *= tab->sc[d];

    // ---- shock-capturing weights of the sensor field (cells with gamma_e < C_gamma)
    float alpha = 1.0f;
    if (ms.sc_on && gam < ms.c_gamma) {
      const float at = fsqrt(hex_atil2<P>(tab, su[slot][0], ta, tb, tc, gref));
      const float f = lane_on ? (1.0f - gam) * (gr[0] * gr[0] + gr[1] * gr[1] + gr[2] * gr[2]) : 0.0f;
      const float Sv = team_sumf<TEAM>(W * f), Tv = team_sumf<TEAM>(W * at * f);
      if (Sv > 0.0f && Tv > 0.0f) alpha = at * (Sv / Tv);
    }
    if (mode == MODE_SENSOR) {
      if (on && t == 0 && gamma_out) gamma_out[e] = gam;
      if (on && alpha_out) alpha_out[e * NL + t] = alpha;
      wave_sync();
      continue;
    }

    // ---- volume terms: -grad phi_j . f(u) + nu alpha (1 - gamma) grad phi_j . grad u,
    // one variable at a time through the team's LDS slot
    const float gs = nu * alpha * (1.0f - gam);
    // the node's velocity and pressure (systems), for the fluxes of every variable
    float vel[3] = {0.0f, 0.0f, 0.0f}, pres = 0.0f;
    if constexpr (FLUX == CVW_EULER) {
      const float inv = frcp(uv[0]);
      vel[0] = uv[1] * inv;
      vel[1] = uv[2] * inv;
      vel[2] = uv[3] * inv;
      pres = (ms.fp[0] - 1.0f) * (uv[4] - 0.5f * uv[0] * (vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2]));
    }
    float r[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      float g[3] = {gr[0], gr[1], gr[2]};
      if (v > 0) {
        g[0] = g[1] = g[2] = 0.0f;
#pragma unroll
        for (int j = 0; j < N1; ++j) {
          g[0] = fmaf(dr[0][j], su[slot][v][j + N1 * (tb + N1 * tc)], g[0]);
          g[1] = fmaf(dr[1][j], su[slot][v][ta + N1 * (j + N1 * tc)], g[1]);
          g[2] = fmaf(dr[2][j], su[slot][v][ta + N1 * (tb + N1 * j)], g[2]);
        }
#pragma unroll
        for (int d = 0; d < 3; ++d) g[d] *= tab->sc[d];
      }
      if (v > 0) wave_sync();                       // the previous variable's terms are read
      if (lane_on) {
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          float fv;
          if constexpr (FLUX == CVW_EULER)   // f_d of variable v: m_d, m_a v_d + p delta_ad, (E + p) v_d
            fv = v == 0 ? uv[1 + d] : (v < 4 ? uv[v] * vel[d] + (v - 1 == d ? pres : 0.0f) : (uv[4] + pres) * vel[d]);
          else
            fv = hex_flux<FLUX>(ms, uv[0], d);
          sv[slot][d][t] = W * tab->sc[d] * (gs * g[d] - fv);
        }
      }
      wave_sync();
      float rv = 0.0f;
#pragma unroll
      for (int q = 0; q < N1; ++q) {
        rv = fmaf(dc[0][q], sv[slot][0][q + N1 * (tb + N1 * tc)], rv);
        rv = fmaf(dc[1][q], sv[slot][1][ta + N1 * (q + N1 * tc)], rv);
        rv = fmaf(dc[2][q], sv[slot][2][ta + N1 * (tb + N1 * q)], rv);
      }
      r[v] = rv;
    }

    // ---- interface terms: face f = 2 d + s, the neighbour read through its
    // face f ^ 1.  A system evaluates each face point's flux once (the N1
    // lanes on the point's normal line share it through LDS) and then lifts
    // it along the lines; a scalar law lets every lane evaluate its own.
    if constexpr (NV > 1) {
#pragma unroll
      for (int k = 0; k < (NI + TEAM - 1) / TEAM; ++k) {
        const int i = t + k * TEAM;
        if (i < NI) {
          const int f = i / NP, pq = i % NP, d = f >> 1, s = f & 1, p = pq % N1, q = pq / N1;
          float um[NV], up[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            um[v] = 0.0f;
            up[v] = 0.0f;
#pragma unroll
            for (int m = 0; m < N1; ++m) {
              const int idx = d == 0 ? m + N1 * (p + N1 * q) : (d == 1 ? p + N1 * (m + N1 * q) : p + N1 * (q + N1 * m));
              um[v] = fmaf(tab->Lend[s][m], su[slot][v][idx], um[v]);
              up[v] = fmaf(tab->Lend[1 - s][m], sn[slot][f][v][idx], up[v]);
            }
          }
          float fs[NV];
          hex_num_flux<FLUX>(ms, um, up, d, s ? 1.0f : -1.0f, fs);
          const float wq = tab->w1[p] * tab->w1[q] * tab->Jf[d];
#pragma unroll
          for (int v = 0; v < NV; ++v) sf[slot][v][i] = wq * fs[v];
        }
      }
      wave_sync();
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const int d = f >> 1, s = f & 1;
        const int pq = d == 0 ? tb + N1 * tc : (d == 1 ? ta + N1 * tc : ta + N1 * tb);
#pragma unroll
        for (int v = 0; v < NV; ++v) r[v] = fmaf(le[d][s], sf[slot][v][f * NP + pq], r[v]);
      }
    }
#pragma unroll(NV == 1 ? 6 : 1)
    for (int f = 0; f < (NV == 1 ? 6 : 0); ++f) {
      const int d = f >> 1, s = f & 1;
      float lws = 0.0f;
#pragma unroll
      for (int k = 0; k < 6; ++k) lws = k == f ? lw[k >> 1][k & 1] : lws;
      {
        float um[NV], up[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          um[v] = 0.0f;
          up[v] = 0.0f;
#pragma unroll
          for (int j = 0; j < N1; ++j) {
            const int idx = d == 0 ? j + N1 * (tb + N1 * tc) : (d == 1 ? ta + N1 * (j + N1 * tc) : ta + N1 * (tb + N1 * j));
            um[v] = fmaf(tab->Lend[s][j], su[slot][v][idx], um[v]);
            up[v] = fmaf(tab->Lend[1 - s][j], sn[slot][2 * d + s][v][idx], up[v]);
          }
        }
        float fs[NV];
        hex_num_flux<FLUX>(ms, um, up, d, s ? 1.0f : -1.0f, fs);
#pragma unroll
        for (int v = 0; v < NV; ++v) r[v] = fmaf(lws, fs[v], r[v]);
      }
    }

    // ---- output
    if (on) {
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int64_t idx = (v * E + e) * NL + t;
        float o;
        if (mode == MODE_RESIDUAL) {
          o = r[v];
        } else {
          const float base = (a0 != 0.0f) ? a0 * u0[idx] : 0.0f;
          o = base + b0 * (uv[v] - dt * r[v] / W);
        }
        nonfinite = nonfinite || !isfinite(o);
        out[idx] = o;
      }
      if (t == 0 && gamma_out) gamma_out[e] = gam;
    }
    wave_sync();
  }
  if (__ballot(nonfinite) && (threadIdx.x & 63) == 0) atomicOr(status, ST_NONFINITE);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static unsigned hex_blocks(int64_t n, int per) { return static_cast<unsigned>((n + per - 1) / per); }

cvw_status hex_candidates(const cvw_mesh* m, const cvw_params* prm, const float* u, float* cand, hipStream_t s) {
  const MethodScalars ms = make_scalars(prm);
  const dim3 g(hex_blocks(m->Nv, 256)), b(256);
  switch (m->degree) {
    case 1: hipLaunchKernelGGL(hex_vertex_kernel<1>, g, b, 0, s, u, cand, m->d_vtx_ent, m->d_hext, m->Nv, ms); break;
    case 2: hipLaunchKernelGGL(hex_vertex_kernel<2>, g, b, 0, s, u, cand, m->d_vtx_ent, m->d_hext, m->Nv, ms); break;
    default: set_error("hexahedra: degree 1 or 2"); return CVW_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

template <int P, int FLUX>
static void launch_hex_eval(const cvw_mesh* m, const MethodScalars& ms, int mode, const float* u, const float* u0,
                            float* out, float* gamma, float* alpha, const float* cand, float* gbuf, uint32_t* status,
                            float dt, float a0, float b0, hipStream_t s) {
  constexpr int CPB = HexShape<P>::CPB;
  const int64_t nblk = (m->E + CPB - 1) / CPB;
  const unsigned grid = static_cast<unsigned>(std::min<int64_t>(nblk, 16384));
  // the sensor pass writes gamma_e into the caller's array when there is one, else into the scratch
  float* g = gamma ? gamma : gbuf;
  if (ms.sensor_kind != CVW_SENSOR_FIXED)
    hipLaunchKernelGGL((hex_sensor_kernel<P>), dim3(hex_blocks(m->E, 256)), dim3(256), 0, s, u, g, cand, m->d_cell_vtx,
                       m->d_hext, m->E, ms);
  // gamma_e is already in the caller's array when the sensor pass wrote it there
  float* gout = (ms.sensor_kind != CVW_SENSOR_FIXED && gamma) ? nullptr : gamma;
  hipLaunchKernelGGL((hex_eval_kernel<P, FLUX>), dim3(grid), dim3(256), 0, s, u, u0, out, gout, alpha, g, m->d_nbr,
                     m->d_hext, m->E, nblk, ms, mode, dt, a0, b0, status);
}

cvw_status hex_eval(const cvw_mesh* m, const cvw_params* prm, int mode, const float* u, const float* u0, float* out,
                    float* gamma, float* alpha, const float* cand, float* gbuf, uint32_t* status, float dt, float a0,
                    float b0, hipStream_t s) {
  const MethodScalars ms = make_scalars(prm);
  const int fl = prm->flux;
  switch (m->degree) {
    case 1:
      if (fl == CVW_BURGERS) launch_hex_eval<1, CVW_BURGERS>(m, ms, mode, u, u0, out, gamma, alpha, cand, gbuf, status, dt, a0, b0, s);
      else if (fl == CVW_EULER) launch_hex_eval<1, CVW_EULER>(m, ms, mode, u, u0, out, gamma, alpha, cand, gbuf, status, dt, a0, b0, s);
      else launch_hex_eval<1, CVW_ADVECT_CONST>(m, ms, mode, u, u0, out, gamma, alpha, cand, gbuf, status, dt, a0, b0, s);
      break;
    case 2:
      if (fl == CVW_BURGERS) launch_hex_eval<2, CVW_BURGERS>(m, ms, mode, u, u0, out, gamma, alpha, cand, gbuf, status, dt, a0, b0, s);
      else if (fl == CVW_EULER) launch_hex_eval<2, CVW_EULER>(m, ms, mode, u, u0, out, gamma, alpha, cand, gbuf, status, dt, a0, b0, s);
      else launch_hex_eval<2, CVW_ADVECT_CONST>(m, ms, mode, u, u0, out, gamma, alpha, cand, gbuf, status, dt, a0, b0, s);
      break;
    default: set_error("hexahedra: degree 1 or 2"); return CVW_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

}  // namespace cvw
