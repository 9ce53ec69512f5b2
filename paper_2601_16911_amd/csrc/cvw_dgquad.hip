// DG on congruent axis-aligned quadrilaterals (Lagrange basis at the Gauss
// points, collocated (p+1)^2 Gauss rule), p = 1..3, on gfx950.
//
// Two kernels per residual evaluation:
//
//  * dgq_vertex_kernel  -- one thread per mesh vertex x_i.  Walks the vertex
//    patch C(x_i) in CSR order, evaluates the Hermite data D^k u_h^e(x_i) of
//    each cell of the patch (Taylor expansion, eq. taylorsol), the pointwise
//    indicator beta = ||u_h^e||_{x_i}^q (eq. pointsnorm) and the Jiang-Shu
//    weight (eps + beta)^{-r}, and writes the vertex candidate data
//    c_i[k] = sum omega_e^i D^k u_h^e(x_i) (eq. taylorcand).  No atomics.
//
//  * dgq_eval_kernel -- one 16-lane DPP row per cell, node (a, b) on lane
//    a + 4 b.  Each lane evaluates, at its own node / quadrature point, the
//    derivatives of the cell solution and of the v_e vertex candidates; row
//    reductions give the element semi-norms (eq. snorm), the cell WENO
//    weights, ||u_h^e - u_h^{e,*}||_e (FP64) and gamma_e (eq. gamma), the
//    wave speed lambda_e and nu_e (eq. lostab), and the sums of the
//    shock-capturing weights alpha_q (eq. alphaq).  The same lanes then
//    assemble the residual: volume flux and stabilisation contracted with the
//    1D derivative matrix along rows / columns, LLF / HLL interface fluxes on
//    the boundary lanes, and optionally the SSP-RK stage update with the
//    diagonal (exact, collocated) mass matrix.
//
// All intra-cell exchanges are DPP moves inside the 16-lane row (quad
// broadcasts along x, row rotations along y); no LDS is used.
#include <cstdlib>

#include "cvw_device.h"
#include "cvw_dgq_common.h"

namespace cvw {

// Derivatives D^k (|k| = 1..P, KSet order) at z + (X, Y) of the degree-P
// polynomial whose derivatives at z are c (Taylor expansion, eq. taylorsol)
template <int P>
__device__ __forceinline__ void taylor_move(const float (&c)[KSet<P>::NK], float X, float Y,
                                            float (&o)[KSet<P>::NK]) {
  constexpr int NK = KSet<P>::NK;
  constexpr KSet<P> ks = kset<P>;
  constexpr float inv_n[4] = {1.0f, 1.0f, 0.5f, 1.0f / 3.0f};
  float px[P + 1], py[P + 1];
  px[0] = 1.0f;
  py[0] = 1.0f;
#pragma unroll
  for (int n = 1; n <= P; ++n) {
    px[n] = px[n - 1] * X * inv_n[n];
    py[n] = py[n - 1] * Y * inv_n[n];
  }
#pragma unroll
  for (int t = 0; t < NK; ++t) {
    float s = c[t];
#pragma unroll
    for (int t2 = NK - 1; t2 >= 0; --t2) {
      const int i = ks.x[t2] - ks.x[t], j = ks.y[t2] - ks.y[t];
      if (t2 != t && i >= 0 && j >= 0) s = fmaf(c[t2], (i == 0) ? py[j] : (j == 0) ? px[i] : px[i] * py[j], s);
    }
    o[t] = s;
  }
}

// sum_k h_e^{2|k|-2} x_k y_k over |k| = 1..P (the weights of eq. snorm, d = 2)
template <int P>
__device__ __forceinline__ float order_weighted_dot(const float (&x)[KSet<P>::NK], const float (&y)[KSet<P>::NK],
                                                    float he2) {
  constexpr KSet<P> ks = kset<P>;
  float s[P + 1] = {};
#pragma unroll
  for (int t = 0; t < KSet<P>::NK; ++t) {
    const int o = ks.x[t] + ks.y[t];
    s[o] = fmaf(x[t], y[t], s[o]);
  }
  float r = s[P];
#pragma unroll
  for (int o = P - 1; o >= 1; --o) r = fmaf(he2, r, s[o]);
  return r;
}

// Cell mean of sum_k h_e^{2|k|-2} (D^k p)^2 (eq. snorm divided by |e|) for the
// degree-P polynomial p with derivatives ch at the centre of a hx x hy cell.
// Exact: D^k p has degree <= 2 in the centred coordinates (X, Y); written in
// the orthogonal basis 1, X, (X^2 - hx^2/12)/2, Y, XY, ... its mean square is a
// sum of squares with the weights mean(X^2) = hx^2/12,
// mean(((X^2 - hx^2/12)/2)^2) = hx^4/720, mean(X^2 Y^2) = hx^2 hy^2/144.
template <int P>
__device__ __forceinline__ float centred_seminorm_mean(const float (&ch)[KSet<P>::NK], float mx2, float my2,
                                                      float qx4, float qy4, float he2) {
  constexpr int NK = KSet<P>::NK;
  constexpr KSet<P> ks = kset<P>;
  float ms[NK];
#pragma unroll
  for (int t = 0; t < NK; ++t) {
    float A = ch[t], rest = 0.0f;
#pragma unroll
    for (int t2 = 0; t2 < NK; ++t2) {
      const int i = ks.x[t2] - ks.x[t], j = ks.y[t2] - ks.y[t];
      if (t2 == t || i < 0 || j < 0) continue;
      const float c = ch[t2];
      if (i == 1 && j == 0) rest = fmaf(c * mx2, c, rest);
      if (i == 0 && j == 1) rest = fmaf(c * my2, c, rest);
      if (i == 1 && j == 1) rest = fmaf(c * (mx2 * my2), c, rest);
      if (i == 2 && j == 0) {
        A = fmaf(c, 0.5f * mx2, A);
        rest = fmaf(c * qx4, c, rest);
      }
      if (i == 0 && j == 2) {
        A = fmaf(c, 0.5f * my2, A);
        rest = fmaf(c * qy4, c, rest);
      }
    }
    ms[t] = fmaf(A, A, rest);
  }
  float one[NK];
#pragma unroll
  for (int t = 0; t < NK; ++t) one[t] = 1.0f;
  return order_weighted_dot<P>(ms, one, he2);
}

__device__ __forceinline__ float ipow(float x, int n) {
  float r = 1.0f;
  for (int i = 0; i < n; ++i) r *= x;
  return r;
}

// ---------------------------------------------------------------------------
// vertex stage
// ---------------------------------------------------------------------------
// Hermite data of one patch cell at the vertex (corner lv of the cell):
// Ek[t] = h_e^{|k|} D^k u_h^e(x_i); returns sum_k Ek^2 = ||u_h^e||_{x_i}^2.
// The vertex is moved to the reference corner (-1, -1) by mirroring the data,
// l_i^{(m)}(1) = (-1)^m l_{P-i}^{(m)}(-1): rows through the load addresses,
// columns by selects.  MX (MY) = 0: the vertex is at xi = -1 (eta = -1); 1: at
// +1; 2: taken from lv at run time.  Every variant performs the same
// floating-point operations on the same values (sign changes are exact), so a
// vertex's result does not depend on the variant its wave takes.
template <int P, int MX, int MY>
__device__ __forceinline__ double vertex_cell(const float* __restrict__ ue, int lv, const VertexTables& vt,
                                              double (&Ek)[KSet<P>::NK]) {
  constexpr int N1 = P + 1, NLOC = N1 * N1, NK = KSet<P>::NK;
  constexpr KSet<P> ks = kset<P>;
  const bool fx = (MX == 2) ? (lv == 1 || lv == 2) : (MX == 1);
  const bool fy = (MY == 2) ? (lv >= 2) : (MY == 1);
  float rf[NLOC];
#pragma unroll
  for (int bb = 0; bb < N1; ++bb) {
    const float* row = ue + N1 * (fy ? P - bb : bb);
    float v[N1];
    if constexpr (N1 == 4) {
      const float4 v4 = *reinterpret_cast<const float4*>(row);
      v[0] = v4.x;
      v[1] = v4.y;
      v[2] = v4.z;
      v[3] = v4.w;
    } else {
#pragma unroll
      for (int aa = 0; aa < N1; ++aa) v[aa] = row[aa];
    }
#pragma unroll
    for (int aa = 0; aa < N1; ++aa) rf[aa + N1 * bb] = fx ? v[P - aa] : v[aa];
  }
  // derivatives of the data relative to the corner's nodal value, so that
  // constant data gives exactly zero Hermite data (differences of two floats
  // are exact in float64); float64 because high derivatives of smooth data
  // cancel strongly.  One node column j at a time:
  //   T_j[m] = sum_i L[m][i] (u_ij - u_00),   D^k = sum_j L[ky][j] T_j[kx]
  const double r0 = static_cast<double>(rf[0]);
#pragma unroll
  for (int j = 0; j < N1; ++j) {
    // the corner node's own difference is zero: column 0 starts at i = 1
    const int ib = (j == 0) ? 1 : 0;
    double rc[N1];
#pragma unroll
    for (int ii = ib; ii < N1; ++ii) rc[ii] = static_cast<double>(rf[ii + N1 * j]) - r0;
    double Tj[N1];
#pragma unroll
    for (int m = 0; m < N1; ++m) {
      double sacc = vt.L[m][ib] * rc[ib];
#pragma unroll
      for (int ii = ib + 1; ii < N1; ++ii) sacc = fma(vt.L[m][ii], rc[ii], sacc);
      Tj[m] = sacc;
    }
#pragma unroll
    for (int t = 0; t < NK; ++t)
      Ek[t] = (j == 0) ? vt.L[ks.y[t]][0] * Tj[ks.x[t]] : fma(vt.L[ks.y[t]][j], Tj[ks.x[t]], Ek[t]);
  }
  double b2 = 0.0;
#pragma unroll
  for (int t = 0; t < NK; ++t) {
    const bool flip = (fx && (ks.x[t] & 1)) != (fy && (ks.y[t] & 1));
    Ek[t] *= flip ? -vt.sk[t] : vt.sk[t];
    b2 = fma(Ek[t], Ek[t], b2);
  }
  return b2;
}

// The candidate data of vertex i.
template <int P>
__device__ __forceinline__ void dgq_vertex_at(const float* __restrict__ u, float* __restrict__ cand,
                                              const int32_t* __restrict__ vptr, const int32_t* __restrict__ vent,
                                              int64_t i, const VertexTables& vt, const MethodScalars& ms) {
  constexpr int N1 = P + 1, NLOC = N1 * N1, NK = KSet<P>::NK;
  constexpr KSet<P> ks = kset<P>;
  double acc[NK];
#pragma unroll
  for (int t = 0; t < NK; ++t) acc[t] = 0.0;
  double wsum = 0.0;
  const int beg = vptr[i], end = vptr[i + 1];
  for (int it = beg; it < end; ++it) {
    const int ent = vent[it];
    const int e = ent >> 2, lv = ent & 3;
    const float* ue = u + static_cast<int64_t>(e) * NLOC;
    // on structured meshes the it-th patch cell of neighbouring vertices sits
    // at the same corner: then the whole wave takes a variant with the
    // mirroring fixed at compile time
    double Ek[NK], b2;
    const int lv0 = __builtin_amdgcn_readfirstlane(lv);
    if (__builtin_amdgcn_ballot_w64(lv != lv0) == 0) {
      switch (lv0) {
        case 0: b2 = vertex_cell<P, 0, 0>(ue, lv, vt, Ek); break;
        case 1: b2 = vertex_cell<P, 1, 0>(ue, lv, vt, Ek); break;
        case 2: b2 = vertex_cell<P, 1, 1>(ue, lv, vt, Ek); break;
        default: b2 = vertex_cell<P, 0, 1>(ue, lv, vt, Ek); break;
      }
    } else {
      b2 = vertex_cell<P, 2, 2>(ue, lv, vt, Ek);
    }
    // weight (eps + beta)^{-r}, beta = ||u_h^e||_{x_i}^q; for r = 2, q = 1 from
    // the hardware float64 square root and reciprocal (about single
    // precision: the weights enter a normalised average)
    double w;
    if (ms.fast_exp) {
      const double den = ms.eps_vd + __builtin_amdgcn_sqrt(b2);
      w = __builtin_amdgcn_rcp(den * den);
    } else {
      const double beta = pow(sqrt(b2), static_cast<double>(ms.q_beta));
      w = pow(ms.eps_vd + beta, -static_cast<double>(ms.r));
    }
#pragma unroll
    for (int t = 0; t < NK; ++t) acc[t] = fma(w, Ek[t], acc[t]);
    wsum += w;
  }
  const double inv = 1.0 / wsum;
  float* out = cand + i * NK;
#pragma unroll
  for (int t = 0; t < NK; ++t) out[t] = static_cast<float>(acc[t] * inv * vt.hinv[ks.x[t] + ks.y[t]]);
}

// One block of 256 vertices (logical block index blk).
template <int P>
__device__ __forceinline__ void dgq_vertex_body(const float* __restrict__ u, float* __restrict__ cand,
                                                const int32_t* __restrict__ vptr, const int32_t* __restrict__ vent,
                                                int64_t Nv, int64_t blk, const VertexTables& vt,
                                                const MethodScalars& ms) {
  const int64_t i = blk * VTX_PER_BLOCK + threadIdx.x;
  if (i >= Nv) return;
  dgq_vertex_at<P>(u, cand, vptr, vent, i, vt, ms);
}

template <int P>
__global__ __launch_bounds__(256) void dgq_vertex_kernel(const float* __restrict__ u, float* __restrict__ cand,
                                                         const int32_t* __restrict__ vptr,
                                                         const int32_t* __restrict__ vent, int64_t Nv,
                                                         int64_t nbp, VertexTables vt, MethodScalars ms) {
  dgq_vertex_body<P>(u, cand, vptr, vent, Nv, xcd_block(blockIdx.x, nbp), vt, ms);
}

// The listed vertices vlist[0 .. *count) only (the grid covers every vertex;
// threads past the count leave).
template <int P>
__global__ __launch_bounds__(256) void dgq_vertex_list_kernel(const float* __restrict__ u, float* __restrict__ cand,
                                                              const int32_t* __restrict__ vptr,
                                                              const int32_t* __restrict__ vent, int64_t Nv,
                                                              VertexTables vt, MethodScalars ms,
                                                              const uint32_t* __restrict__ count,
                                                              const int32_t* __restrict__ vlist) {
  const int64_t k = blockIdx.x * 256LL + threadIdx.x;
  if (k >= static_cast<int64_t>(*count) || k >= Nv) return;
  dgq_vertex_at<P>(u, cand, vptr, vent, vlist[k], vt, ms);
}

// ---------------------------------------------------------------------------
// cell stage + residual
// ---------------------------------------------------------------------------
template <int P>
__device__ __forceinline__ float rowsum4(const float (&c)[MAXP + 1], float x) {
  // sum_i c[i] * x(node (i, b))  for i <= P
  float s = c[0] * qbcast<0>(x);
  if constexpr (P >= 1) s = fmaf(c[1], qbcast<1>(x), s);
  if constexpr (P >= 2) s = fmaf(c[2], qbcast<2>(x), s);
  if constexpr (P >= 3) s = fmaf(c[3], qbcast<3>(x), s);
  return s;
}
__device__ __forceinline__ float colsum4(const float (&c)[4], float x) {
  // sum_s c[s] * x(node (a, src row of rotation s)); c[] already matches the source row
  float s = c[0] * x;
  s = fmaf(c[1], rrot<1>(x), s);
  s = fmaf(c[2], rrot<2>(x), s);
  s = fmaf(c[3], rrot<3>(x), s);
  return s;
}
// value held by node (a, J) of the own column
template <int J>
__device__ __forceinline__ float colbcast(float x, const int (&srcb)[4]) {
  float r = x;
  const float r1 = rrot<1>(x), r2 = rrot<2>(x), r3 = rrot<3>(x);
  r = (srcb[1] == J) ? r1 : r;
  r = (srcb[2] == J) ? r2 : r;
  r = (srcb[3] == J) ? r3 : r;
  return r;
}

// One block of 16 cells (logical block index blk); sl = the lane tables in LDS.
// BUF: the state arrays (all variables) and the candidates are each under
// 4 GiB and are accessed as raw buffers with 32-bit offsets.  OPEN: the mesh
// has boundary faces (negative neighbour codes); closed meshes compile
// without the boundary branches.
template <int P, int FLUX, bool BUF = false, bool OPEN = false>
__device__ __forceinline__ void dgq_eval_body(
    const float* __restrict__ u, const float* __restrict__ u0, float* __restrict__ out,
    float* __restrict__ gamma_out, float* __restrict__ alpha_out, const float* __restrict__ cand,
    const int32_t* __restrict__ cell_vtx, const int32_t* __restrict__ nbr, const LaneRec* sl,
    const TensorTables& tab, int64_t E, int64_t blk, const CellGeo& G, const MethodScalars& ms,
    int mode, float dt, float a0, float b0, uint32_t* __restrict__ status,
    const float* __restrict__ gamma_in = nullptr) {
  constexpr int N1 = P + 1, NLOC = N1 * N1, NK = KSet<P>::NK;
  constexpr int NV = NVar<FLUX>::value;
  constexpr KSet<P> ks = kset<P>;
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int q = tid & 15;
  const int a = q & 3, b = q >> 2;
  const int64_t e = blk * 16 + (tid >> 4);
  if (e >= E) return;                          // whole 16-lane rows leave together
  const LaneRec& L = sl[q];
  const bool nd = (a <= P) && (b <= P);
  const int node = a + N1 * b;
  const float sx = G.sx, sy = G.sy;
  const float wa = L.misc[4], wb = L.misc[5];
  const float Wq = nd ? wa * wb * G.area4 : 0.0f;

  // byte offset of the own node in a variable's block, and the block size
  [[maybe_unused]] const uint32_t offn = BUF ? static_cast<uint32_t>((e * NLOC + node) * 4) : 0u;
  [[maybe_unused]] const uint32_t sbytes = BUF ? static_cast<uint32_t>(E * NLOC * 4) : 0u;

  // ---- state ---------------------------------------------------------------
  float uv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    float dummy = 0.0f;
    if constexpr (FLUX == CVW_EULER) dummy = (v == 0) ? 1.0f : (v == 3 ? 2.5f : 0.0f);
    if constexpr (BUF)
      uv[v] = nd ? buf_load(buf_rsrc(u, sbytes * NV), offn, v * sbytes) : dummy;
    else
      uv[v] = nd ? u[(static_cast<int64_t>(v) * E + e) * NLOC + node] : dummy;
  }
  // vertex candidate data: lane a of each quad fetches vertex a, then quad
  // broadcasts give every lane all four (eq. taylorcand output)
  // neighbour of the lane's face point (degree 3), fetched early
  const int32_t en_pre = (P == 3) ? nbr[e * 4 + L.slot] : 0;
  // gamma_e given (a sensor pass ran before: fused plain, learned) or fixed:
  // the sensor-field derivatives below then serve only the shock-capturing
  // weights, which are active only where gamma_e < c_gamma
  const bool given = (gamma_in != nullptr);
  const bool plain = !given && (ms.sensor_kind == CVW_SENSOR_PLAIN);
  const float gpre = given ? gamma_in[e] : ms.fixed_gamma;
  const bool need_du = plain || (ms.sc_on && __ballot(static_cast<double>(gpre) < ms.c_gammad) != 0);
  float myc[NK] = {};
  if (plain) {
    const int64_t vid = cell_vtx[e * 4 + a];
#pragma unroll
    for (int t = 0; t < NK; ++t) {
      if constexpr (BUF)
        myc[t] = buf_load(buf_rsrc(cand, 0xFFFFFFFFu), static_cast<uint32_t>(vid * NK * 4), 4u * t);
      else
        myc[t] = cand[vid * NK + t];
    }
  }

  // ---- sensor-field derivatives at the own point (eq. taylorsol) ------------
  // float64: high derivatives of smooth data cancel; the data is taken relative
  // to its value at node (0, 0) so that constant data gives exactly zero
  // (needed by the plain sensor and by the shock-capturing weights only)
  float Du[NK] = {};
  if (need_du) {
    double rho = nd ? static_cast<double>(uv[0]) : 0.0;
    const double ref = rowbcastd<0>(rho);          // node (0, 0) = lane 0 of the row
    rho = nd ? rho - ref : 0.0;
    double Rm[N1];
    Rm[0] = rho;
#pragma unroll
    for (int m = 1; m < N1; ++m) {
      double sacc = L.DX[m - 1][0] * qbcastd<0>(rho);
      if constexpr (P >= 1) sacc = fma(L.DX[m - 1][1], qbcastd<1>(rho), sacc);
      if constexpr (P >= 2) sacc = fma(L.DX[m - 1][2], qbcastd<2>(rho), sacc);
      if constexpr (P >= 3) sacc = fma(L.DX[m - 1][3], qbcastd<3>(rho), sacc);
      Rm[m] = sacc;
    }
    // reference derivatives, rounded to float, times (2/hx)^kx (2/hy)^ky
    float spx[N1], spy[N1];
    spx[0] = 1.0f;
    spy[0] = 1.0f;
#pragma unroll
    for (int n = 1; n < N1; ++n) {
      spx[n] = spx[n - 1] * sx;
      spy[n] = spy[n - 1] * sy;
    }
#pragma unroll
    for (int t = 0; t < NK; ++t) {
      const int kx = ks.x[t], ky = ks.y[t];
      double sacc;
      if (ky == 0) {
        sacc = Rm[kx];
      } else {
        sacc = L.DY[ky - 1][0] * Rm[kx];
        sacc = fma(L.DY[ky - 1][1], rrotd<1>(Rm[kx]), sacc);
        sacc = fma(L.DY[ky - 1][2], rrotd<2>(Rm[kx]), sacc);
        sacc = fma(L.DY[ky - 1][3], rrotd<3>(Rm[kx]), sacc);
      }
      Du[t] = static_cast<float>(sacc) * (spx[kx] * spy[ky]);
    }
  }
  const float he2 = G.he2;
  // sum_k h_e^{2|k|-2} (D^k u_h)^2 at the own point: the integrand of eq. snorm
  // (d = 2) and, times h_e^2, the pointwise indicator of eq. alphaq
  const float sw = order_weighted_dot<P>(Du, Du, he2);

  // ---- sensor gamma_e (cell stage of the cell-vertex reconstruction) --------
  float gam;
  if (!plain) {
    gam = gpre;                                // given per cell, or the fixed value
  } else {
    // The vertex candidates p_l (eq. taylorcand) are re-expanded about the
    // cell centre, one vertex per quad lane (lane a holds vertex a; the rows
    // repeat it), and their element semi-norms taken in closed form (the
    // Gauss rule integrates them exactly).  The blend sum_l omega_l p_l is one
    // polynomial again, evaluated once per quadrature point for eq. gamma.
    const float xq = L.misc[6], yq = L.misc[7];
    const float n2 = row_sum(Wq * sw);
    const float xl = (a == 1 || a == 2) ? 1.0f : -1.0f, yl = (a >= 2) ? 1.0f : -1.0f;
    float ch[NK];
    taylor_move<P>(myc, -xl * G.hhx, -yl * G.hhy, ch);
    const float b2v = 4.0f * G.area4 * centred_seminorm_mean<P>(ch, G.mx2, G.my2, G.qx4, G.qy4, he2);
    float w0, wv;
    if (ms.fast_exp) {
      const float d0 = ms.eps_c + fsqrt(n2), dv = ms.eps_c + fsqrt(b2v);
      w0 = (1.0f - 4.0f * ms.lin_w) * frcp(d0 * d0);
      wv = ms.lin_w * frcp(dv * dv);
    } else {
      w0 = (1.0f - 4.0f * ms.lin_w) * powf(ms.eps_c + powf(sqrtf(n2), ms.q_beta), -ms.r);
      wv = ms.lin_w * powf(ms.eps_c + powf(sqrtf(b2v), ms.q_beta), -ms.r);
    }
    const float wq = quad_sum(wv);                   // sum over the four vertices
    const float oinv = frcp(w0 + wq);
    const float whv = wv * oinv;
    float cb[NK], db[NK], dl[NK];
#pragma unroll
    for (int t = 0; t < NK; ++t) cb[t] = quad_sum(whv * ch[t]);
    taylor_move<P>(cb, xq * G.hhx, yq * G.hhy, db);
    // u_h - u* = sum_l omega_l (u_h - p_l) with the normalised weights
    const float wrest = wq * oinv;
#pragma unroll
    for (int t = 0; t < NK; ++t) dl[t] = fmaf(wrest, Du[t], -db[t]);
    const float d2 = row_sum(Wq * order_weighted_dot<P>(dl, dl, he2));
    if (n2 > 0.0f) {
      const float mr = fminf(1.0f, fsqrt(d2 / n2));      // n2 may be subnormal: IEEE division
      gam = 1.0f - (ms.fast_exp ? mr : powf(mr, ms.q_sensor));
    } else {
      gam = 1.0f;
    }
  }

  // ---- viscosity and shock-capturing weights -------------------------------
  float lam;
  if (ms.lam_g > 0.0f) {
    lam = ms.lam_g;
  } else {
    lam = row_max(nd ? wave_speed<FLUX>(ms, uv, 0.0f, 0.0f) : 0.0f);
  }
  const float nu = lam * G.nuf;
  const float atil = fsqrt(he2 * sw);
  const float g2 = Du[0] * Du[0] + Du[1] * Du[1];
  const float fq = (1.0f - gam) * g2;
  const float S = row_sum(Wq * fq);
  const float T = row_sum(Wq * atil * fq);
  const bool sc_active = ms.sc_on && (static_cast<double>(gam) < ms.c_gammad) && (S > 0.0f) && (T > 0.0f);
  const float alpha = sc_active ? atil * (S / T) : 1.0f;      // T may be subnormal: IEEE division

  if (mode == MODE_SENSOR) {
    if (q == 0) gamma_out[e] = gam;
    if (nd && alpha_out) alpha_out[e * NLOC + node] = alpha;
    return;
  }
  if (gamma_out && q == 0) gamma_out[e] = gam;

  // ---- volume terms ---------------------------------------------------------
  const float coef = nu * (1.0f - gam) * alpha;
  float fx[NV], fy[NV];
  phys_flux<FLUX>(ms, uv, 0.0f, 0.0f, fx, fy);
  float r[NV];
  // face traces of the own node values.  P < 3: all four sides; P = 3: only
  // the two each lane can need (its own x side; the S side in rows 0, 1 and
  // the N side in rows 2, 3), see the interface terms
  float tW[NV], tE[NV], tS[NV], tN[NV];
  if constexpr (P == 3) {
    // contractions along the row (quad broadcasts) and the column (row
    // rotations) as DPP-fused multiply-adds; the 2/h factors ride on the weights
    const float Wqx = Wq * sx, Wqy = Wq * sy, cfx = coef * sx, cfy = coef * sy;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      float gx, gy, sXs, sYs;
      qdot4x2(uv[v], L.CX1, L.OX, gx, sXs);
      rdot4x2(uv[v], L.CY1, L.OY, gy, sYs);
      tW[v] = sXs;                // x-side trace (W on a = 0, E otherwise)
      tS[v] = sYs;                // y-side trace (S in rows 0, 1; N in rows 2, 3)
      const float WFx = Wqx * (cfx * gx - fx[v]);
      const float WFy = Wqy * (cfy * gy - fy[v]);
      r[v] = qdot4(WFx, L.TX) + rdot4(WFy, L.TY);
    }
  } else {
    // p < 3: the same fused contractions over the whole quad / column; the
    // lane tables are zero beyond p and so are the values of the unused lanes
    const float Wqx = Wq * sx, Wqy = Wq * sy, cfx = coef * sx, cfy = coef * sy;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const float uvv = nd ? uv[v] : 0.0f;
      const float gx = qdotp<P>(uvv, L.CX1), gy = rdotp<P>(uvv, L.CY1);
      tW[v] = qdotp<P>(uvv, L.BX0);
      tE[v] = qdotp<P>(uvv, L.BX1);
      tS[v] = rdotp<P>(uvv, L.BY0);
      tN[v] = rdotp<P>(uvv, L.BY1);
      const float WFx = Wqx * (cfx * gx - fx[v]);
      const float WFy = Wqy * (cfy * gy - fy[v]);
      r[v] = qdotp<P>(WFx, L.TX) + rdotp<P>(WFy, L.TY);
    }
  }

  // ---- interface terms -------------------------------------------------------
  const int64_t stride = E * NLOC;
  // the previous stage's values of the stage update, in flight during the faces
  float u0v[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v)
    if constexpr (BUF)
      u0v[v] = (mode != MODE_RESIDUAL && a0 != 0.0f && nd) ? buf_load(buf_rsrc(u0, sbytes * NV), offn, v * sbytes)
                                                           : 0.0f;
    else
      u0v[v] = (mode != MODE_RESIDUAL && a0 != 0.0f && nd) ? u0[(static_cast<int64_t>(v) * E + e) * NLOC + node]
                                                           : 0.0f;
  if constexpr (P == 3) {
    // One face quadrature point per lane (4 faces x 4 points = 16 lanes; the
    // assignment and the lane's coefficients are in its lane record)
    const bool xf = (a == 0 || a == 3);
    const bool inner = !xf && (b == 1 || b == 2);
    const bool bnd = OPEN && en_pre < 0;               // a boundary face: exterior state from its data
    const int64_t enc = bnd ? 0 : en_pre;
    const float* un0 = u + enc * NLOC + L.noff;
    const int nst = L.nstep;
    float um[NV], up[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      // the inner lanes take the corner columns' y-side traces from the lanes
      // a = 0 / 3 of their row (rows 1 / 2 hold S / N traces)
      const float tc = dpp<(0 | (0 << 2) | (3 << 4) | (3 << 6))>(tS[v]);
      um[v] = xf ? tW[v] : (inner ? tc : tS[v]);
      float s2 = 0.0f;
      if (!bnd) {
        if constexpr (BUF) {
          const uint32_t o0 = static_cast<uint32_t>((enc * NLOC + L.noff) * 4);
#pragma unroll
          for (int ii = 0; ii < N1; ++ii)
            s2 = fmaf(L.FB[ii], buf_load(buf_rsrc(u, sbytes * NV), o0 + 4u * nst * ii, v * sbytes), s2);
        } else {
          const float* un = un0 + v * stride;
#pragma unroll
          for (int ii = 0; ii < N1; ++ii) s2 = fmaf(L.FB[ii], un[nst * ii], s2);
        }
      }
      up[v] = s2;
    }
    if (bnd) ghost_state<FLUX>(ms, en_pre, um, L.nx, L.ny, up);
    float fs[NV];
    num_flux<FLUX>(ms, um, up, L.nx, L.ny, 0.0f, 0.0f, fs);
    const float wpt = fmaf(L.fwx, G.hy, L.fwy * G.hx);
    // distribution: W / E along the own row from the lanes a = 0 / 3; S / N of
    // column a from the lanes named in the lane record (lane permutes)
    const int rowbase = (tid & 63) & ~15;
    const int addrS = 4 * (rowbase + L.srcS), addrN = 4 * (rowbase + L.srcN);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const float fl = wpt * fs[v];
      const float fS0 = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addrS, __builtin_bit_cast(int, fl)));
      const float fNP = __builtin_bit_cast(float, __builtin_amdgcn_ds_bpermute(addrN, __builtin_bit_cast(int, fl)));
      r[v] = qfma03(r[v], fl, L.misc[0], L.misc[1]);
      r[v] = fmaf(L.misc[2], fS0, r[v]);
      r[v] = fmaf(L.misc[3], fNP, r[v]);
    }
  } else {
    float fW[NV], fE[NV], fS[NV], fN[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) fW[v] = fE[v] = fS[v] = fN[v] = 0.0f;
    if (nd && (a == 0 || a == P)) {
      const bool west = (a == 0);
      const int32_t code = nbr[e * 4 + (west ? 3 : 1)];
      float up[NV];
      if (!OPEN || code >= 0) {
        const int64_t en = code;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const float* un = u + v * stride + en * NLOC + N1 * b;
          float s2 = 0.0f;
#pragma unroll
          for (int ii = 0; ii < N1; ++ii) s2 = fmaf(west ? tab.B[1][ii] : tab.B[0][ii], un[ii], s2);
          up[v] = s2;
        }
      } else {
        ghost_state<FLUX>(ms, code, west ? tW : tE, west ? -1.0f : 1.0f, 0.0f, up);
      }
      float fs[NV];
      num_flux<FLUX>(ms, west ? tW : tE, up, west ? -1.0f : 1.0f, 0.0f, 0.0f, 0.0f, fs);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (west) fW[v] = wb * G.hhy * fs[v];
        else fE[v] = wb * G.hhy * fs[v];
      }
    }
    if (nd && (b == 0 || b == P)) {
      const bool south = (b == 0);
      const int32_t code = nbr[e * 4 + (south ? 0 : 2)];
      float up[NV];
      if (!OPEN || code >= 0) {
        const int64_t en = code;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const float* un = u + v * stride + en * NLOC + a;
          float s2 = 0.0f;
#pragma unroll
          for (int jj = 0; jj < N1; ++jj) s2 = fmaf(south ? tab.B[1][jj] : tab.B[0][jj], un[N1 * jj], s2);
          up[v] = s2;
        }
      } else {
        ghost_state<FLUX>(ms, code, south ? tS : tN, 0.0f, south ? -1.0f : 1.0f, up);
      }
      float fs[NV];
      num_flux<FLUX>(ms, south ? tS : tN, up, 0.0f, south ? -1.0f : 1.0f, 0.0f, 0.0f, fs);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (south) fS[v] = wa * G.hhx * fs[v];
        else fN[v] = wa * G.hhx * fs[v];
      }
    }
    // distribute the face fluxes: west / east along the own row, south / north
    // from row 0 / row P of the own column
    const int s0 = b & 3, sP = (b - P) & 3;   // rotations that bring row 0 / row P
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const float r1 = rrot<1>(fS[v]), r2 = rrot<2>(fS[v]), r3 = rrot<3>(fS[v]);
      const float fS0 = (s0 == 0) ? fS[v] : (s0 == 1) ? r1 : (s0 == 2) ? r2 : r3;
      const float n1 = rrot<1>(fN[v]), n2 = rrot<2>(fN[v]), n3 = rrot<3>(fN[v]);
      const float fNP = (sP == 0) ? fN[v] : (sP == 1) ? n1 : (sP == 2) ? n2 : n3;
      r[v] = fmaf(L.misc[0], qbcast<0>(fW[v]), r[v]);
      r[v] = fmaf(L.misc[1], qbcast<P>(fE[v]), r[v]);
      r[v] = fmaf(L.misc[2], fS0, r[v]);
      r[v] = fmaf(L.misc[3], fNP, r[v]);
    }

  }

  // ---- output -----------------------------------------------------------------
  const float invWq = nd ? frcp(Wq) : 0.0f;
  bool nonfinite = false, inadmissible = false;
  if (nd) {
    inadmissible = !state_admissible<FLUX>(ms, uv);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int64_t idx = (static_cast<int64_t>(v) * E + e) * NLOC + node;
      float val;
      if (mode == MODE_RESIDUAL) {
        val = r[v];
      } else {
        const float Lv = -r[v] * invWq;
        const float base = (a0 != 0.0f) ? a0 * u0v[v] : 0.0f;
        val = base + b0 * (uv[v] + dt * Lv);
      }
      nonfinite = nonfinite || !isfinite(val);
      if constexpr (BUF)
        buf_store(val, buf_rsrc(out, sbytes * NV), offn, v * sbytes);
      else
        out[idx] = val;
    }
  }
  const unsigned long long m1 = __ballot(nonfinite), m2 = __ballot(inadmissible);
  if ((m1 | m2) && (tid & 63) == __builtin_ctzll(m1 | m2))
    atomicOr(status, (m1 ? ST_NONFINITE : 0u) | (m2 ? ST_NONPOSITIVE : 0u));
}

// Degree 1, four cells per 16-lane row: cell (tid >> 2) of the 64-cell tile
// blk, node (a, b) = (l & 1, l >> 1) on lane l = tid & 3 of its quad, so every
// exchange inside a cell is a quad permutation.  Each lane evaluates one point
// of an x face (side a, point b) and one of a y face (side b, point a).  The
// same steps as the 16-lane body: derivatives of the sensor field (float64),
// gamma_e (eq. gamma; the candidates' first derivatives are constant, so their
// centred expansion is the candidate itself), lambda_e, alpha_q, volume and
// interface terms, stage update.
template <int FLUX, bool BUF = false, bool OPEN = false>
__device__ __forceinline__ void dgq_eval_body_p1(
    const float* __restrict__ u, const float* __restrict__ u0, float* __restrict__ out,
    float* __restrict__ gamma_out, float* __restrict__ alpha_out, const float* __restrict__ cand,
    const int32_t* __restrict__ cell_vtx, const int32_t* __restrict__ nbr, const LaneRec1* sl, int64_t E,
    int64_t blk, const CellGeo& G, const MethodScalars& ms, int mode, float dt, float a0, float b0,
    uint32_t* __restrict__ status, const float* __restrict__ gamma_in = nullptr) {
  constexpr int P = 1, NLOC = 4, NK = 2;
  constexpr int NV = NVar<FLUX>::value;
  int tid = threadIdx.x;
  asm volatile("" : "+v"(tid));
  const int l = tid & 3;
  const int a = l & 1, b = l >> 1;
  const int64_t e = blk * 64 + (tid >> 2);
  if (e >= E) return;                          // whole quads leave together
  const LaneRec1& L = sl[l];
  const float sx = G.sx, sy = G.sy, he2 = G.he2;
  const float Wq = L.wa * L.wb * G.area4;
  const int64_t stride = E * NLOC;
  [[maybe_unused]] const uint32_t offn = BUF ? static_cast<uint32_t>((e * NLOC + l) * 4) : 0u;
  [[maybe_unused]] const uint32_t sbytes = BUF ? static_cast<uint32_t>(stride * 4) : 0u;

  float uv[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    if constexpr (BUF)
      uv[v] = buf_load(buf_rsrc(u, sbytes * NV), offn, v * sbytes);
    else
      uv[v] = u[v * stride + e * NLOC + l];
  }
  // neighbours across the lane's x and y face points, fetched early
  const int32_t enx = nbr[e * 4 + L.slotx], eny = nbr[e * 4 + L.sloty];
  const bool given = (gamma_in != nullptr);
  const bool plain = !given && (ms.sensor_kind == CVW_SENSOR_PLAIN);
  const float gpre = given ? gamma_in[e] : ms.fixed_gamma;
  const bool need_du = plain || (ms.sc_on && __ballot(static_cast<double>(gpre) < ms.c_gammad) != 0);
  float myc[NK] = {};
  if (plain) {                                 // lane l fetches vertex l (eq. taylorcand output)
    const int64_t vid = cell_vtx[e * 4 + l];
#pragma unroll
    for (int t = 0; t < NK; ++t) myc[t] = cand[vid * NK + t];
  }

  // first derivatives of the sensor field at the own node, float64, relative
  // to node (0, 0) of the cell
  float Du[NK] = {};
  if (need_du) {
    double rho = static_cast<double>(uv[0]);
    rho -= qbcastd<0>(rho);
    constexpr int X0 = 0 | (0 << 2) | (2 << 4) | (2 << 6), X1 = 1 | (1 << 2) | (3 << 4) | (3 << 6);
    constexpr int Y0 = 0 | (1 << 2) | (0 << 4) | (1 << 6), Y1 = 2 | (3 << 2) | (2 << 4) | (3 << 6);
    const double dx = fma(L.DX[1], dppd<X1>(rho), L.DX[0] * dppd<X0>(rho));
    const double dy = fma(L.DY[1], dppd<Y1>(rho), L.DY[0] * dppd<Y0>(rho));
    Du[0] = static_cast<float>(dx) * sx;
    Du[1] = static_cast<float>(dy) * sy;
  }
  const float sw = order_weighted_dot<P>(Du, Du, he2);

  float gam;
  if (!plain) {
    gam = gpre;
  } else {
    const float n2 = quad_sum(Wq * sw);
    // the candidates' derivatives are constant: the centred expansion is the
    // candidate data itself, its semi-norm |e| (c_x^2 + c_y^2)
    const float b2v = 4.0f * G.area4 * centred_seminorm_mean<P>(myc, G.mx2, G.my2, G.qx4, G.qy4, he2);
    float w0, wv;
    if (ms.fast_exp) {
      const float d0 = ms.eps_c + fsqrt(n2), dv = ms.eps_c + fsqrt(b2v);
      w0 = (1.0f - 4.0f * ms.lin_w) * frcp(d0 * d0);
      wv = ms.lin_w * frcp(dv * dv);
    } else {
      w0 = (1.0f - 4.0f * ms.lin_w) * powf(ms.eps_c + powf(sqrtf(n2), ms.q_beta), -ms.r);
      wv = ms.lin_w * powf(ms.eps_c + powf(sqrtf(b2v), ms.q_beta), -ms.r);
    }
    const float wq = quad_sum(wv);
    const float oinv = frcp(w0 + wq);
    const float whv = wv * oinv;
    const float wrest = wq * oinv;
    float dl[NK];
#pragma unroll
    for (int t = 0; t < NK; ++t) dl[t] = fmaf(wrest, Du[t], -quad_sum(whv * myc[t]));
    const float d2 = quad_sum(Wq * order_weighted_dot<P>(dl, dl, he2));
    if (n2 > 0.0f) {
      const float mr = fminf(1.0f, fsqrt(d2 / n2));      // n2 may be subnormal: IEEE division
      gam = 1.0f - (ms.fast_exp ? mr : powf(mr, ms.q_sensor));
    } else {
      gam = 1.0f;
    }
  }

  const float lam = (ms.lam_g > 0.0f) ? ms.lam_g : quad_max(wave_speed<FLUX>(ms, uv, 0.0f, 0.0f));
  const float nu = lam * G.nuf;
  const float atil = fsqrt(he2 * sw);
  const float g2 = Du[0] * Du[0] + Du[1] * Du[1];
  const float fq = (1.0f - gam) * g2;
  const float S = quad_sum(Wq * fq);
  const float T = quad_sum(Wq * atil * fq);
  const bool sc_active = ms.sc_on && (static_cast<double>(gam) < ms.c_gammad) && (S > 0.0f) && (T > 0.0f);
  const float alpha = sc_active ? atil * (S / T) : 1.0f;      // T may be subnormal: IEEE division

  if (mode == MODE_SENSOR) {
    if (l == 0) gamma_out[e] = gam;
    if (alpha_out) alpha_out[e * NLOC + l] = alpha;
    return;
  }
  if (gamma_out && l == 0) gamma_out[e] = gam;

  // ---- volume terms and own traces ------------------------------------------
  const float coef = nu * (1.0f - gam) * alpha;
  const float Wqx = Wq * sx, Wqy = Wq * sy, cfx = coef * sx, cfy = coef * sy;
  float fx[NV], fy[NV], r[NV], tX[NV], tY[NV];
  phys_flux<FLUX>(ms, uv, 0.0f, 0.0f, fx, fy);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const float gx = qx2(uv[v], L.CX1[0], L.CX1[1]), gy = qy2(uv[v], L.CY1[0], L.CY1[1]);
    tX[v] = qx2(uv[v], L.OX[0], L.OX[1]);
    tY[v] = qy2(uv[v], L.OY[0], L.OY[1]);
    const float WFx = Wqx * (cfx * gx - fx[v]);
    const float WFy = Wqy * (cfy * gy - fy[v]);
    r[v] = qx2(WFx, L.TX[0], L.TX[1]) + qy2(WFy, L.TY[0], L.TY[1]);
  }

  // ---- interface terms: x face (side a, point b) and y face (side b, point a)
  float px[NV], py[NV];
  // boundary faces (negative neighbour codes) take the exterior state of their data
  const bool bx_ = OPEN && enx < 0, by_ = OPEN && eny < 0;
  const int64_t ecx = bx_ ? 0 : enx, ecy = by_ ? 0 : eny;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int64_t ox = v * stride + ecx * NLOC + 2 * b;
    const int64_t oy = v * stride + ecy * NLOC + a;
    px[v] = 0.0f;
    py[v] = 0.0f;
    if constexpr (BUF) {
      const __amdgpu_buffer_rsrc_t ru = buf_rsrc(u, sbytes * NV);
      const uint32_t bx = static_cast<uint32_t>((ecx * NLOC + 2 * b) * 4);
      const uint32_t by = static_cast<uint32_t>((ecy * NLOC + a) * 4);
      if (!bx_) px[v] = fmaf(L.FX[1], buf_load(ru, bx + 4u, v * sbytes), L.FX[0] * buf_load(ru, bx, v * sbytes));
      if (!by_) py[v] = fmaf(L.FY[1], buf_load(ru, by + 8u, v * sbytes), L.FY[0] * buf_load(ru, by, v * sbytes));
    } else {
      if (!bx_) px[v] = fmaf(L.FX[1], u[ox + 1], L.FX[0] * u[ox]);
      if (!by_) py[v] = fmaf(L.FY[1], u[oy + 2], L.FY[0] * u[oy]);
    }
  }
  if (bx_) ghost_state<FLUX>(ms, enx, tX, L.nx, 0.0f, px);
  if (by_) ghost_state<FLUX>(ms, eny, tY, 0.0f, L.ny, py);
  float fsx[NV], fsy[NV];
  num_flux<FLUX>(ms, tX, px, L.nx, 0.0f, 0.0f, 0.0f, fsx);
  num_flux<FLUX>(ms, tY, py, 0.0f, L.ny, 0.0f, 0.0f, fsy);
  const float wx = L.wb * G.hhy, wy = L.wa * G.hhx;      // face weights of the two points
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    // W / E fluxes of the own row from the lanes (0, b) / (1, b), S / N fluxes
    // of the own column from the lanes (a, 0) / (a, 1)
    r[v] += qx2(wx * fsx[v], L.lift[0], L.lift[1]) + qy2(wy * fsy[v], L.lift[2], L.lift[3]);
  }

  // ---- output -------------------------------------------------------------------
  const float invWq = frcp(Wq);
  bool nonfinite = false;
  const bool inadmissible = !state_admissible<FLUX>(ms, uv);
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    float val;
    if (mode == MODE_RESIDUAL) {
      val = r[v];
    } else {
      float base = 0.0f;
      if (a0 != 0.0f) {
        if constexpr (BUF)
          base = a0 * buf_load(buf_rsrc(u0, sbytes * NV), offn, v * sbytes);
        else
          base = a0 * u0[v * stride + e * NLOC + l];
      }
      val = base + b0 * (uv[v] + dt * (-r[v] * invWq));
    }
    nonfinite = nonfinite || !isfinite(val);
    if constexpr (BUF)
      buf_store(val, buf_rsrc(out, sbytes * NV), offn, v * sbytes);
    else
      out[v * stride + e * NLOC + l] = val;
  }
  const unsigned long long m1 = __ballot(nonfinite), m2 = __ballot(inadmissible);
  if ((m1 | m2) && (tid & 63) == __builtin_ctzll(m1 | m2))
    atomicOr(status, (m1 ? ST_NONFINITE : 0u) | (m2 ? ST_NONPOSITIVE : 0u));
}

// 256-thread blocks: all loads in flight before the LDS stores
__device__ __forceinline__ void load_lane_tables(const LaneRec* __restrict__ lanes, LaneRec* sl) {
  const float4* src = reinterpret_cast<const float4*>(lanes);
  float4* dst = reinterpret_cast<float4*>(sl);
  constexpr int n4 = 16 * sizeof(LaneRec) / 16;
  constexpr int it = (n4 + 255) / 256;
  float4 tmp[it];
#pragma unroll
  for (int k = 0; k < it; ++k) {
    const int i = threadIdx.x + 256 * k;
    if (i < n4) tmp[k] = src[i];
  }
#pragma unroll
  for (int k = 0; k < it; ++k) {
    const int i = threadIdx.x + 256 * k;
    if (i < n4) dst[i] = tmp[k];
  }
}

#ifndef CVW_EVAL_WPE
#define CVW_EVAL_WPE
#endif
template <int P, int FLUX, bool BUF, bool OPEN>
__global__ __launch_bounds__(256) CVW_EVAL_WPE void dgq_eval_kernel(
    const float* __restrict__ u, const float* __restrict__ u0, float* __restrict__ out,
    float* __restrict__ gamma_out, float* __restrict__ alpha_out, const float* __restrict__ cand,
    const int32_t* __restrict__ cell_vtx, const int32_t* __restrict__ nbr, const LaneRec* __restrict__ lanes,
    TensorTables tab, int64_t E, int64_t ntile, int64_t tpb, CellGeo G, MethodScalars ms,
    int mode, float dt, float a0, float b0, uint32_t* __restrict__ status, const float* __restrict__ gamma_in) {
  // per-lane tables: one copy per block in LDS
  __shared__ LaneRec sl[16];
  load_lane_tables(lanes, sl);
  __syncthreads();
  // each block walks a contiguous run of tpb tiles of 16 cells; the blocks of
  // one XCD hold consecutive runs (neighbour rows share its L2)
  const int64_t first = xcd_block(blockIdx.x, gridDim.x) * tpb;
  for (int64_t t = 0; t < tpb; ++t) {
    const int64_t blk = first + t;
    if (blk >= ntile) break;
    // keeps the lane-table reads inside the loop (hoisted, they would hold
    // every table entry in registers for the whole run)
    CellGeo g = G;
    asm volatile("" : "+s"(g.hx), "+s"(g.hy), "+s"(g.he), "+s"(g.sx), "+s"(g.sy), "+s"(g.he2), "+s"(g.mx2),
                 "+s"(g.my2), "+s"(g.qx4), "+s"(g.qy4), "+s"(g.area4), "+s"(g.hhx), "+s"(g.hhy), "+s"(g.nuf)
                 :: "memory");
    if constexpr (P == 1)
      dgq_eval_body_p1<FLUX, BUF, OPEN>(u, u0, out, gamma_out, alpha_out, cand, cell_vtx, nbr,
                                  reinterpret_cast<const LaneRec1*>(sl), E, blk, g, ms, mode, dt, a0, b0, status,
                                  gamma_in);
    else
      dgq_eval_body<P, FLUX, BUF, OPEN>(u, u0, out, gamma_out, alpha_out, cand, cell_vtx, nbr, sl, tab, E, blk, g, ms,
                                  mode, dt, a0, b0, status, gamma_in);
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static int64_t pad8(int64_t n) { return (n + 7) / 8 * 8; }

template <int P>
static void launch_vertex(const cvw_mesh* m, const MethodScalars& ms, const float* u, float* cand,
                          const uint32_t* vcount, const int32_t* vlist, hipStream_t s) {
  const int64_t nb = pad8((m->Nv + VTX_PER_BLOCK - 1) / VTX_PER_BLOCK);
  const VertexTables vt = make_vertex_tables(m->tens, m->hx, m->hy, m->he, P);
  if (vlist)
    hipLaunchKernelGGL(dgq_vertex_list_kernel<P>, dim3(static_cast<unsigned>((m->Nv + 255) / 256)), dim3(256), 0,
                       s, u, cand, m->d_vtx_ptr, m->d_vtx_ent, m->Nv, vt, ms, vcount, vlist);
  else
    hipLaunchKernelGGL(dgq_vertex_kernel<P>, dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, u, cand,
                       m->d_vtx_ptr, m->d_vtx_ent, m->Nv, nb, vt, ms);
}

cvw_status dgquad_candidates(const cvw_mesh* m, const cvw_params* prm, const float* u, float* cand,
                             hipStream_t s, const uint32_t* vcount, const int32_t* vlist) {
  const MethodScalars ms = make_scalars(prm);
  switch (m->degree) {
    case 1: launch_vertex<1>(m, ms, u, cand, vcount, vlist, s); break;
    case 2: launch_vertex<2>(m, ms, u, cand, vcount, vlist, s); break;
    case 3: launch_vertex<3>(m, ms, u, cand, vcount, vlist, s); break;
    default: set_error("degree not supported on the GPU path"); return CVW_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

// grid of the fused cell pass: a few resident rounds of 256-thread blocks
#ifndef CVW_EVAL_GRID
#define CVW_EVAL_GRID 8192
#endif
static constexpr int64_t EVAL_GRID = CVW_EVAL_GRID;

// CVW_WIDE_ADDRESSING=1 in the environment selects the 64-bit addressed cell
// pass for every mesh (the two variants compute bitwise the same results; the
// switch lets small meshes exercise the path of the > 4 GiB states)
static bool wide_addressing_forced() {
  const char* v = std::getenv("CVW_WIDE_ADDRESSING");
  return v && v[0] == '1';
}

template <int P, int FLUX>
static void launch_eval(const cvw_mesh* m, const MethodScalars& ms, int mode, const float* u, const float* u0,
                        float* out, float* gamma, float* alpha, const float* cand, uint32_t* status, float dt,
                        float a0, float b0, const float* gamma_in, hipStream_t s) {
  const int64_t ntile = (m->E + cells_per_tile(P) - 1) / cells_per_tile(P);
  const int64_t nb = pad8(std::min<int64_t>(ntile, m->eval_grid > 0 ? m->eval_grid : EVAL_GRID));
  const int64_t tpb = (ntile + nb - 1) / nb;
  // raw-buffer addressing when the state (all variables) and the candidates fit in 32-bit byte offsets
  constexpr int64_t NV = NVar<FLUX>::value;
  const bool buf = !wide_addressing_forced() && m->E * m->nloc * NV * 4 < (int64_t(1) << 32) - 4096 &&
                   m->Nv * m->nk * 4 < (int64_t(1) << 32) - 4096;
  const CellGeo geo = make_cell_geo(m->hx, m->hy, m->he, P);
  // one variant per addressing mode and per closed / open mesh
  auto kern = buf ? (m->closed ? dgq_eval_kernel<P, FLUX, true, false> : dgq_eval_kernel<P, FLUX, true, true>)
                  : (m->closed ? dgq_eval_kernel<P, FLUX, false, false> : dgq_eval_kernel<P, FLUX, false, true>);
  hipLaunchKernelGGL(kern, dim3(static_cast<unsigned>(nb)), dim3(256), 0, s, u, u0, out, gamma, alpha, cand,
                     m->d_cell_vtx, m->d_nbr, m->d_lanes, m->tens, m->E, ntile, tpb, geo, ms, mode, dt, a0, b0, status,
                     gamma_in);
}

template <int P>
static cvw_status eval_p(const cvw_mesh* m, const MethodScalars& ms, int flux, int mode, const float* u,
                         const float* u0, float* out, float* gamma, float* alpha, const float* cand,
                         uint32_t* status, float dt, float a0, float b0, const float* gin, hipStream_t s) {
  switch (flux) {
    case CVW_ADVECT_CONST:
      launch_eval<P, CVW_ADVECT_CONST>(m, ms, mode, u, u0, out, gamma, alpha, cand, status, dt, a0, b0, gin, s);
      break;
    case CVW_BURGERS:
      launch_eval<P, CVW_BURGERS>(m, ms, mode, u, u0, out, gamma, alpha, cand, status, dt, a0, b0, gin, s);
      break;
    case CVW_KPP:
      launch_eval<P, CVW_KPP>(m, ms, mode, u, u0, out, gamma, alpha, cand, status, dt, a0, b0, gin, s);
      break;
    case CVW_EULER:
      launch_eval<P, CVW_EULER>(m, ms, mode, u, u0, out, gamma, alpha, cand, status, dt, a0, b0, gin, s);
      break;
    default:
      set_error("flux not supported by the DG quadrilateral path (position-dependent velocity needs cell coordinates)");
      return CVW_EUNSUPPORTED;
  }
  return CVW_OK;
}

cvw_status dgquad_eval(const cvw_mesh* m, const cvw_params* prm, int mode, const float* u, const float* u0,
                       float* out, float* gamma, float* alpha, const float* cand, uint32_t* status, float dt,
                       float a0, float b0, hipStream_t s, const float* gamma_in) {
  const MethodScalars ms = make_scalars(prm);
  if (ms.sensor_kind == CVW_SENSOR_LEARNED && !gamma_in) { set_error("learned sensor without its gamma"); return CVW_EINVAL; }
  cvw_status st;
  switch (m->degree) {
    case 1: st = eval_p<1>(m, ms, prm->flux, mode, u, u0, out, gamma, alpha, cand, status, dt, a0, b0, gamma_in, s); break;
    case 2: st = eval_p<2>(m, ms, prm->flux, mode, u, u0, out, gamma, alpha, cand, status, dt, a0, b0, gamma_in, s); break;
    case 3: st = eval_p<3>(m, ms, prm->flux, mode, u, u0, out, gamma, alpha, cand, status, dt, a0, b0, gamma_in, s); break;
    default: set_error("degree not supported on the GPU path"); return CVW_EUNSUPPORTED;
  }
  if (st != CVW_OK) return st;
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

// ---------------------------------------------------------------------------
// Features of the learned sensor, one thread per cell (float64):
// 4 x 9 vertex mismatch slots h^|k| (c_i[k] - D^k s^e(x_i)) / sigma_e,
// 9 centre slots h^|k| D^k s^e(x_c) / sigma_e, log10(sigma_e / sigma_ref),
// the largest and the mean per-vertex mismatch 2-norm; sigma_e =
// ||s^e||_e + 1e-12 sigma_ref (eq. snorm, collocated Gauss rule, exact).
// Orders above p are zero.  Stored as bfloat16 [E][48].
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void dgq_feat_kernel(const float* __restrict__ u, const float* __restrict__ cand,
                                                       const int32_t* __restrict__ cell_vtx, TensorTables tab,
                                                       int64_t E, double hx, double hy, double he,
                                                       double sigma_ref, uint16_t* __restrict__ feat) {
  constexpr int N1 = P + 1, NLOC = N1 * N1, NK = KSet<P>::NK;
  constexpr KSet<P> ks = kset<P>;
  const int64_t e = blockIdx.x * 256LL + threadIdx.x;
  if (e >= E) return;
  double r[NLOC];
  {
    const float* ue = u + e * NLOC;
    const double r0 = ue[0];
#pragma unroll
    for (int j = 0; j < NLOC; ++j) r[j] = static_cast<double>(ue[j]) - r0;
  }
  const double sx = 2.0 / hx, sy = 2.0 / hy;
  double sc[NK], hk[NK], wk[NK];
#pragma unroll
  for (int t = 0; t < NK; ++t) {
    const int kx = ks.x[t], ky = ks.y[t];
    sc[t] = dpow(sx, kx) * dpow(sy, ky);
    hk[t] = dpow(he, kx + ky);
    wk[t] = dpow(he * he, kx + ky - 1);
  }
  // sigma_e: semi-norm on the Gauss nodes
  double n2 = 0.0;
#pragma unroll
  for (int a = 0; a < N1; ++a) {
    double T[N1][N1];   // T[m][j] = sum_i l_i^{(m)}(xi_a) r[i][j]
#pragma unroll
    for (int m = 0; m < N1; ++m)
#pragma unroll
      for (int j = 0; j < N1; ++j) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < N1; ++i) s = fma(tab.Dd[m][a][i], r[i + N1 * j], s);
        T[m][j] = s;
      }
#pragma unroll
    for (int b = 0; b < N1; ++b) {
      double pq = 0.0;
#pragma unroll
      for (int t = 0; t < NK; ++t) {
        double d = 0.0;
#pragma unroll
        for (int j = 0; j < N1; ++j) d = fma(tab.Dd[ks.y[t]][b][j], T[ks.x[t]][j], d);
        d *= sc[t];
        pq = fma(wk[t] * d, d, pq);
      }
      n2 = fma(tab.wd[a] * tab.wd[b] * 0.25 * hx * hy, pq, n2);
    }
  }
  const double sigma = sqrt(n2) + 1e-12 * sigma_ref;
  const double inv = 1.0 / sigma;
  float f[48];
#pragma unroll
  for (int t = 0; t < 48; ++t) f[t] = 0.0f;
  double nmax = 0.0, nsum = 0.0;
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const bool fx = (l == 1) || (l == 2), fy = (l >= 2);
    double Tx[N1][N1];   // Tx[m][j] = sum_i l_i^{(m)}(+-1) r[i][j]
#pragma unroll
    for (int m = 0; m < N1; ++m)
#pragma unroll
      for (int j = 0; j < N1; ++j) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < N1; ++i) {
          const double Lx = fx ? ((m & 1) ? -tab.Ld[m][P - i] : tab.Ld[m][P - i]) : tab.Ld[m][i];
          s = fma(Lx, r[i + N1 * j], s);
        }
        Tx[m][j] = s;
      }
    const int64_t vtx = cell_vtx[e * 4 + l];
    double nrm = 0.0;
#pragma unroll
    for (int t = 0; t < NK; ++t) {
      const int kx = ks.x[t], ky = ks.y[t];
      double d = 0.0;
#pragma unroll
      for (int j = 0; j < N1; ++j) {
        const double Ly = fy ? ((ky & 1) ? -tab.Ld[ky][P - j] : tab.Ld[ky][P - j]) : tab.Ld[ky][j];
        d = fma(Ly, Tx[kx][j], d);
      }
      const double mis = hk[t] * (static_cast<double>(cand[vtx * NK + t]) - d * sc[t]) * inv;
      f[9 * l + t] = static_cast<float>(mis);
      nrm = fma(mis, mis, nrm);
    }
    nrm = sqrt(nrm);
    nmax = fmax(nmax, nrm);
    nsum += nrm;
  }
#pragma unroll
  for (int t = 0; t < NK; ++t) {
    const int kx = ks.x[t], ky = ks.y[t];
    double d = 0.0;
#pragma unroll
    for (int j = 0; j < N1; ++j) {
      double s = 0.0;
#pragma unroll
      for (int i = 0; i < N1; ++i) s = fma(tab.Cd[kx][i], r[i + N1 * j], s);
      d = fma(tab.Cd[ky][j], s, d);
    }
    f[36 + t] = static_cast<float>(hk[t] * d * sc[t] * inv);
  }
  f[45] = static_cast<float>(log10(sigma / sigma_ref));
  f[46] = static_cast<float>(nmax);
  f[47] = static_cast<float>(0.25 * nsum);
  uint4* dst = reinterpret_cast<uint4*>(feat + e * 48);
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    uint32_t w[4];
#pragma unroll
    for (int h = 0; h < 4; ++h)
      w[h] = static_cast<uint32_t>(bf16_bits(f[8 * q + 2 * h])) |
             (static_cast<uint32_t>(bf16_bits(f[8 * q + 2 * h + 1])) << 16);
    dst[q] = make_uint4(w[0], w[1], w[2], w[3]);
  }
}

cvw_status dgquad_features(const cvw_mesh* m, const float* u, const float* cand, double sigma_ref, uint16_t* feat,
                           hipStream_t s) {
  const dim3 g(static_cast<unsigned>((m->E + 255) / 256)), b(256);
  switch (m->degree) {
    case 1: hipLaunchKernelGGL(dgq_feat_kernel<1>, g, b, 0, s, u, cand, m->d_cell_vtx, m->tens, m->E, m->hx, m->hy, m->he, sigma_ref, feat); break;
    case 2: hipLaunchKernelGGL(dgq_feat_kernel<2>, g, b, 0, s, u, cand, m->d_cell_vtx, m->tens, m->E, m->hx, m->hy, m->he, sigma_ref, feat); break;
    case 3: hipLaunchKernelGGL(dgq_feat_kernel<3>, g, b, 0, s, u, cand, m->d_cell_vtx, m->tens, m->E, m->hx, m->hy, m->he, sigma_ref, feat); break;
    default: set_error("degree not supported on the GPU path"); return CVW_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

}  // namespace cvw

namespace cvw {

// ---------------------------------------------------------------------------
// float64 totals sum_e int_{K_e} u_h dx (collocated Gauss weights), fixed-order
// reductions: thread partials over a fixed grid-stride set, a shared-memory
// tree per block, then one block sums the block partials in index order.
// ---------------------------------------------------------------------------
constexpr int TOT_BLOCKS = 1024;

__global__ __launch_bounds__(256) void totals_partial_kernel(const float* __restrict__ u, double* __restrict__ part,
                                                             int64_t E, int nloc, int n1, TensorTables tab,
                                                             double jac) {
  __shared__ double sh[256];
  const int v = blockIdx.y;
  const int64_t n = E * nloc;
  const float* uv = u + static_cast<int64_t>(v) * n;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += static_cast<int64_t>(gridDim.x) * 256) {
    const int j = static_cast<int>(i % nloc);
    const int a = j % n1, b = j / n1;
    acc += static_cast<double>(uv[i]) * static_cast<double>(tab.w[a < 4 ? a : 0]) * static_cast<double>(tab.w[b < 4 ? b : 0]);
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[v * TOT_BLOCKS + blockIdx.x] = sh[0] * jac;
}

__global__ __launch_bounds__(256) void totals_final_kernel(const double* __restrict__ part, double* __restrict__ res,
                                                           int nblocks) {
  __shared__ double sh[256];
  const int v = blockIdx.x;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nblocks; i += 256) acc += part[v * TOT_BLOCKS + i];
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) res[v] = sh[0];
}

cvw_status totals_f32(const cvw_mesh* m, int nvar, const float* u, double* part, double* res, hipStream_t s) {
  const int n1 = m->degree + 1;
  const double jac = 0.25 * m->hx * m->hy;
  const int64_t n = m->E * m->nloc;
  int nb = static_cast<int>(std::min<int64_t>(TOT_BLOCKS, (n + 255) / 256));
  hipLaunchKernelGGL(totals_partial_kernel, dim3(nb, nvar), dim3(256), 0, s, u, part, m->E, m->nloc, n1, m->tens, jac);
  hipLaunchKernelGGL(totals_final_kernel, dim3(nvar), dim3(256), 0, s, part, res, nb);
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

}  // namespace cvw

namespace cvw {

// ---------------------------------------------------------------------------
// Batched stage over many independent meshes: per pass one launch per degree
// covers every instance of that degree.  Work items (instance, block) are
// walked by the blocks with a fixed stride; each item runs the same block body
// as the single-mesh kernels, so results are bitwise those of the single-mesh
// path.  The cell pass is launched once per (degree, flux) present.
// ---------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(256) void batch_vertex_kernel(const BatchInst* __restrict__ inst,
                                                           const int2* __restrict__ items, int n_items,
                                                           const TensorTables* __restrict__ tabs, int stage) {
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int2 w = items[it];
    const BatchInst& I = inst[w.x];
    dgq_vertex_body<P>(I.u_in[stage], I.cand, I.vptr, I.vent, I.Nv, w.y, I.vt, I.ms);
  }
}

template <int P, int FLUX>
__global__ __launch_bounds__(256) void batch_eval_kernel(const BatchInst* __restrict__ inst,
                                                         const int2* __restrict__ items, int n_items,
                                                         const TensorTables* __restrict__ tabs,
                                                         const LaneRec* __restrict__ lanes, int stage) {
  __shared__ LaneRec sl[16];
  load_lane_tables(lanes + 16 * P, sl);
  __syncthreads();
  const float A0[3] = {0.0f, 0.75f, 1.0f / 3.0f}, B0[3] = {1.0f, 0.25f, 2.0f / 3.0f};
  const float a0 = A0[stage], b0 = B0[stage];
  const TensorTables& tab = tabs[P];
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int2 w = items[it];
    const BatchInst& I = inst[w.x];
    if constexpr (P == 1)
      dgq_eval_body_p1<FLUX>(I.u_in[stage], I.u, I.u_out[stage], nullptr, nullptr, I.cand, I.cell_vtx, I.nbr,
                             reinterpret_cast<const LaneRec1*>(sl), I.E, w.y, I.g, I.ms, MODE_STAGE, I.dt, a0, b0,
                             I.status, I.gam);
    else
      dgq_eval_body<P, FLUX>(I.u_in[stage], I.u, I.u_out[stage], nullptr, nullptr, I.cand, I.cell_vtx, I.nbr, sl,
                             tab, I.E, w.y, I.g, I.ms, MODE_STAGE, I.dt, a0, b0, I.status, I.gam);
  }
}

cvw_status batch_vertex_pass(int P, const BatchInst* inst, const int2* items, int n_items, const TensorTables* tabs,
                             int stage, int grid, hipStream_t s) {
  if (n_items <= 0) return CVW_OK;
  const dim3 g(std::max(1, std::min(grid, n_items))), b(256);
  switch (P) {
    case 1: hipLaunchKernelGGL(batch_vertex_kernel<1>, g, b, 0, s, inst, items, n_items, tabs, stage); break;
    case 2: hipLaunchKernelGGL(batch_vertex_kernel<2>, g, b, 0, s, inst, items, n_items, tabs, stage); break;
    case 3: hipLaunchKernelGGL(batch_vertex_kernel<3>, g, b, 0, s, inst, items, n_items, tabs, stage); break;
    default: set_error("degree not supported on the GPU path"); return CVW_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

template <int P>
static void launch_batch_eval(int flux, dim3 g, const BatchInst* inst, const int2* items, int n_items,
                              const TensorTables* tabs, const LaneRec* lanes, int stage, hipStream_t s) {
  const dim3 b(256);
  switch (flux) {
    case CVW_ADVECT_CONST:
      hipLaunchKernelGGL((batch_eval_kernel<P, CVW_ADVECT_CONST>), g, b, 0, s, inst, items, n_items, tabs, lanes, stage);
      break;
    case CVW_BURGERS:
      hipLaunchKernelGGL((batch_eval_kernel<P, CVW_BURGERS>), g, b, 0, s, inst, items, n_items, tabs, lanes, stage);
      break;
    default:
      hipLaunchKernelGGL((batch_eval_kernel<P, CVW_KPP>), g, b, 0, s, inst, items, n_items, tabs, lanes, stage);
      break;
  }
}

cvw_status batch_eval_pass(int P, int flux, const BatchInst* inst, const int2* items, int n_items,
                           const TensorTables* tabs, const LaneRec* lanes, int stage, int grid, hipStream_t s) {
  if (n_items <= 0) return CVW_OK;
  if (flux != CVW_ADVECT_CONST && flux != CVW_BURGERS && flux != CVW_KPP) {
    set_error("batched stages: scalar fluxes on DG quadrilaterals"); return CVW_EUNSUPPORTED;
  }
  const dim3 g(std::max(1, std::min(grid, n_items)));
  switch (P) {
    case 1: launch_batch_eval<1>(flux, g, inst, items, n_items, tabs, lanes, stage, s); break;
    case 2: launch_batch_eval<2>(flux, g, inst, items, n_items, tabs, lanes, stage, s); break;
    case 3: launch_batch_eval<3>(flux, g, inst, items, n_items, tabs, lanes, stage, s); break;
    default: set_error("degree not supported on the GPU path"); return CVW_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

}  // namespace cvw
