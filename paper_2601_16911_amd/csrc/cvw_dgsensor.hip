// Fused sensor pass for DG on a structured periodic grid of congruent
// axis-aligned quadrilaterals (cells numbered e = i + nx j), p = 1..3, gfx950.
//
// One 256-thread block per 16 x 16 tile of cells, one thread per cell; the
// vertex stage and the cell stage of the cell-vertex reconstruction (Sec. 3.2)
// meet in LDS, so the sensor field is read from HBM once and only gamma_e is
// written back.
//
//  (A) Every cell of the tile and of its one-cell halo ring turns its nodal
//      values of the sensor field (variable 0) into Legendre coefficients
//      c_mn (float64, data taken relative to node (0, 0) so that constants
//      give exactly zero), and from them its Hermite data at the four corners
//      (eq. taylorsol, reference derivatives, by the closed values of
//      P_m^{(k)}(+-1)).  The pointwise indicator beta = ||u_h^e||_{x_i}
//      (eq. pointsnorm) gives the Jiang-Shu weight w = (eps + beta)^{-r};
//      w and w D^k u_h^e(x_i) are summed per vertex in LDS, corner by corner
//      (one contribution per vertex per round: no atomics, fixed order).
//  (B) Each tile cell reads its four vertex candidates (eq. taylorcand),
//      moves them to the cell centre, writes them and its own polynomial in
//      tensor Legendre coefficients and takes every element semi-norm
//      (eq. snorm) in closed form from those coefficients (the derivative of
//      a Legendre series is a Legendre series; the P_j are orthogonal).  The
//      weights of eq. finalweno, the blend and ||u_h^e - u_h^{e,*}||_e give
//      gamma_e (eq. gamma).
//
// Reference coordinates xi = 2 (x - x_c) / h_x, eta likewise; the nodes are
// the Gauss points, lexicographic with x fastest.
#include "cvw_device.h"
#include "cvw_dgq_common.h"

namespace cvw {

namespace {

// n! for n <= 7 (a table, so that device code never calls a function for it)
constexpr double FACT[8] = {1.0, 1.0, 2.0, 6.0, 24.0, 120.0, 720.0, 5040.0};
constexpr double cfact(int n) { return FACT[n]; }

// Legendre tables of degree < N1
template <int N1>
struct Leg {
  double D[N1][N1][N1];   // D[k][j][m]: coefficient of P_j in the k-th derivative of P_m
  double E[N1][N1];       // E[k][m] = P_m^{(k)}(+1); P_m^{(k)}(-1) = (-1)^{m+k} E[k][m]
  double M[4][N1];        // xi^a / a! = sum_j M[a][j] P_j (a <= 3)
  double Nr[N1];          // int_{-1}^{1} P_j^2 = 2 / (2j + 1)
  constexpr Leg() : D{}, E{}, M{}, Nr{} {
    double D1[N1][N1] = {};
    for (int j = 0; j < N1; ++j)
      for (int m = 0; m < N1; ++m) D1[j][m] = (m > j && ((m - j) & 1)) ? 2.0 * j + 1.0 : 0.0;
    for (int j = 0; j < N1; ++j) D[0][j][j] = 1.0;
    for (int k = 1; k < N1; ++k)
      for (int j = 0; j < N1; ++j)
        for (int m = 0; m < N1; ++m) {
          double s = 0.0;
          for (int i = 0; i < N1; ++i) s += D1[j][i] * D[k - 1][i][m];
          D[k][j][m] = s;
        }
    for (int k = 0; k < N1; ++k)
      for (int m = 0; m < N1; ++m) {
        double p2 = 1.0;
        for (int i = 0; i < k; ++i) p2 *= 2.0;
        E[k][m] = (m >= k) ? cfact(m + k) / (cfact(m - k) * p2 * cfact(k)) : 0.0;
      }
    const double Mx[4][4] = {{1.0, 0.0, 0.0, 0.0},
                             {0.0, 1.0, 0.0, 0.0},
                             {1.0 / 6.0, 0.0, 1.0 / 3.0, 0.0},
                             {0.0, 1.0 / 10.0, 0.0, 1.0 / 15.0}};
    for (int a = 0; a < 4; ++a)
      for (int j = 0; j < N1; ++j) M[a][j] = Mx[a][j];
    for (int j = 0; j < N1; ++j) Nr[j] = 2.0 / (2.0 * j + 1.0);
  }
};
template <int N1>
inline constexpr Leg<N1> leg{};

constexpr int TS = 16;            // tile side in cells
constexpr int NVX = TS + 1;       // tile side in vertices

// sum_k Sk[k] int_ref |d^k p|^2 for p = sum C[m][n] P_m(xi) P_n(eta) over
// 1 <= |k| <= P (eq. snorm, squared; Sk carries h_e^{2|k|-2}, the map and the
// cell area).  TOT: C[m][n] = 0 for m + n > P (a total-degree polynomial).
template <int P, bool TOT>
__device__ __forceinline__ float seminorm_sq(const float (&C)[P + 1][P + 1], const float* Sk) {
  constexpr int N1 = P + 1;
  constexpr KSet<P> ks = kset<P>;
  constexpr Leg<N1> L = leg<N1>;
  float total = 0.0f;
  // one x-derivative order at a time: X[j][n] = sum_m D[kx][j][m] C[m][n],
  // then every multi-index (kx, ky) of the set with that kx
#pragma unroll
  for (int kx = 0; kx < N1; ++kx) {
    float X[N1][N1];
#pragma unroll
    for (int j = 0; j < N1; ++j)
#pragma unroll
      for (int n = 0; n < N1; ++n) {
        float s = 0.0f;
        bool any = false;
#pragma unroll
        for (int m = 0; m < N1; ++m) {
          if (L.D[kx][j][m] == 0.0 || (TOT && m + n > P)) continue;
          s = any ? fmaf(static_cast<float>(L.D[kx][j][m]), C[m][n], s) : static_cast<float>(L.D[kx][j][m]) * C[m][n];
          any = true;
        }
        X[j][n] = s;
      }
#pragma unroll
    for (int t = 0; t < KSet<P>::NK; ++t) {
      if (ks.x[t] != kx) continue;
      const int ky = ks.y[t];
      float acc = 0.0f;
#pragma unroll
      for (int j = 0; j + kx < N1; ++j)
#pragma unroll
        for (int l = 0; l + ky < N1; ++l) {
          float v = 0.0f;
          bool any = false;
#pragma unroll
          for (int n = 0; n < N1; ++n) {
            if (L.D[ky][l][n] == 0.0) continue;
            if (TOT) {   // skip products known to be zero
              bool nz = false;
#pragma unroll
              for (int m = 0; m < N1; ++m) nz = nz || (L.D[kx][j][m] != 0.0 && m + n <= P);
              if (!nz) continue;
            }
            v = any ? fmaf(static_cast<float>(L.D[ky][l][n]), X[j][n], v)
                    : static_cast<float>(L.D[ky][l][n]) * X[j][n];
            any = true;
          }
          if (any) acc = fmaf(static_cast<float>(L.Nr[j] * L.Nr[l]) * v, v, acc);
        }
      total = fmaf(Sk[t], acc, total);
    }
  }
  return total;
}

// Tensor Legendre coefficients (m + n <= P, the constant omitted) of the
// total-degree polynomial with reference derivatives d[k] at the cell centre
template <int P>
__device__ __forceinline__ void taylor_to_legendre(const float (&d)[KSet<P>::NK], float (&C)[P + 1][P + 1]) {
  constexpr int N1 = P + 1;
  constexpr KSet<P> ks = kset<P>;
  constexpr Leg<N1> L = leg<N1>;
#pragma unroll
  for (int m = 0; m < N1; ++m)
#pragma unroll
    for (int n = 0; n < N1; ++n) {
      float s = 0.0f;
      bool any = false;
      if (m + n <= P && (m + n) > 0) {
#pragma unroll
        for (int t = 0; t < KSet<P>::NK; ++t) {
          const double c = L.M[ks.x[t]][m] * L.M[ks.y[t]][n];
          if (c == 0.0) continue;
          s = any ? fmaf(static_cast<float>(c), d[t], s) : static_cast<float>(c) * d[t];
          any = true;
        }
      }
      C[m][n] = s;
    }
}

// Corner data of one cell: Legendre coefficients of its sensor field (float64
// in, float out) and, per corner l (SW, SE, NE, NW), the Jiang-Shu weight
// W[l] and the weighted reference Hermite data WH[l][k].
template <int P>
__device__ __forceinline__ void cell_corners(const float* __restrict__ ue, const SensorTileArgs& A,
                                             const MethodScalars& ms, float (&cf)[P + 1][P + 1],
                                             float (&W)[4], float (&WH)[4][KSet<P>::NK]) {
  constexpr int N1 = P + 1, NK = KSet<P>::NK;
  constexpr KSet<P> ks = kset<P>;
  constexpr Leg<N1> L = leg<N1>;
  float uf[N1 * N1];
  if constexpr (N1 == 4) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const float4 v = reinterpret_cast<const float4*>(ue)[j];
      uf[4 * j] = v.x;
      uf[4 * j + 1] = v.y;
      uf[4 * j + 2] = v.z;
      uf[4 * j + 3] = v.w;
    }
  } else if constexpr (N1 == 2) {
    const float4 v = *reinterpret_cast<const float4*>(ue);
    uf[0] = v.x;
    uf[1] = v.y;
    uf[2] = v.z;
    uf[3] = v.w;
  } else {
#pragma unroll
    for (int i = 0; i < N1 * N1; ++i) uf[i] = ue[i];
  }
  // data relative to node (0, 0): exact in float64
  const double r0 = static_cast<double>(uf[0]);
  // x transform: tx[m][j] = sum_i T[m][i] (u_ij - u_00)
  double tx[N1][N1];
#pragma unroll
  for (int j = 0; j < N1; ++j) {
    double r[N1];
#pragma unroll
    for (int i = 0; i < N1; ++i) r[i] = static_cast<double>(uf[i + N1 * j]) - r0;
#pragma unroll
    for (int m = 0; m < N1; ++m) {
      // node (0, 0) itself contributes exactly zero: row 0 starts at i = 1
      const int ib = (j == 0) ? 1 : 0;
      double s = A.T[m][ib] * r[ib];
#pragma unroll
      for (int i = ib + 1; i < N1; ++i) s = fma(A.T[m][i], r[i], s);
      tx[m][j] = s;
    }
  }
  // y transform: c[m][n] = sum_j T[n][j] tx[m][j] (c[0][0] is not needed)
  double c[N1][N1];
#pragma unroll
  for (int m = 0; m < N1; ++m)
#pragma unroll
    for (int n = 0; n < N1; ++n) {
      if (m == 0 && n == 0) {
        c[0][0] = 0.0;
        continue;
      }
      double s = A.T[n][0] * tx[m][0];
#pragma unroll
      for (int j = 1; j < N1; ++j) s = fma(A.T[n][j], tx[m][j], s);
      c[m][n] = s;
      cf[m][n] = static_cast<float>(s);
    }
  cf[0][0] = 0.0f;
  // corner values, one x-derivative order kx at a time: at xi = +-1,
  // g[n] = sum_m c[m][n] P_m^{(kx)}(+-1) = Ev +- Od; then at eta = +-1 every
  // multi-index (kx, ky) of the set the same way
  float H[4][NK];
#pragma unroll
  for (int kx = 0; kx < N1; ++kx) {
    double gp[N1], gm[N1];
#pragma unroll
    for (int n = 0; n < N1; ++n) {
      double ev = 0.0, od = 0.0;
#pragma unroll
      for (int m = kx; m < N1; ++m) {
        if (((m - kx) & 1) == 0) ev = fma(L.E[kx][m], c[m][n], ev);
        else od = fma(L.E[kx][m], c[m][n], od);
      }
      gp[n] = ev + od;
      gm[n] = ev - od;
    }
#pragma unroll
    for (int t = 0; t < NK; ++t) {
      if (ks.x[t] != kx) continue;
      const int ky = ks.y[t];
#pragma unroll
      for (int sxp = 0; sxp < 2; ++sxp) {
        double ev = 0.0, od = 0.0;
#pragma unroll
        for (int n = ky; n < N1; ++n) {
          const double g = sxp ? gp[n] : gm[n];
          if (((n - ky) & 1) == 0) ev = fma(L.E[ky][n], g, ev);
          else od = fma(L.E[ky][n], g, od);
        }
        // corners: SW (-,-) 0, SE (+,-) 1, NE (+,+) 2, NW (-,+) 3
        H[sxp ? 1 : 0][t] = static_cast<float>(ev - od);
        H[sxp ? 2 : 3][t] = static_cast<float>(ev + od);
      }
    }
  }
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    float b2 = 0.0f;
#pragma unroll
    for (int t = 0; t < NK; ++t) {
      const float ek = A.sk[t] * H[l][t];
      b2 = fmaf(ek, ek, b2);
    }
    float w;
    if (ms.fast_exp) {
      const float den = ms.eps_v + fsqrt(b2);
      w = frcp(den * den);
    } else {
      w = powf(ms.eps_v + powf(sqrtf(b2), ms.q_beta), -ms.r);
    }
    W[l] = w;
#pragma unroll
    for (int t = 0; t < NK; ++t) WH[l][t] = w * H[l][t];
  }
}

}  // namespace

// gamma_e of the own cell from its Legendre coefficients cf and the vertex
// sums in V (cell stage of the reconstruction)
template <int P>
__device__ __forceinline__ float cell_gamma(const float (&cf)[P + 1][P + 1], const float (&V)[KSet<P>::NK + 1][NVX * NVX],
                                            int ci, int cj, const SensorTileArgs& A, const MethodScalars& ms) {
  constexpr int N1 = P + 1, NK = KSet<P>::NK;
  constexpr KSet<P> ks = kset<P>;
  const float n2 = seminorm_sq<P, false>(cf, A.Sk);
  float Dc[4][NK];       // candidates' reference derivatives at the cell centre
  float bl2[4];
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const int dx = (l == 1 || l == 2) ? 1 : 0, dy = (l >= 2) ? 1 : 0;
    const int v = (ci + dx) + NVX * (cj + dy);
    const float inv = frcp(V[NK][v]);
    float cv[NK];
#pragma unroll
    for (int k = 0; k < NK; ++k) cv[k] = V[k][v] * inv;
    // Taylor expansion about the corner (sx, sy) = (2 dx - 1, 2 dy - 1), moved
    // to the centre: D^m p(0) = sum_{k >= m} c[k] (-sx)^{kx-mx} (-sy)^{ky-my} / ((kx-mx)! (ky-my)!)
#pragma unroll
    for (int m = 0; m < NK; ++m) {
      float s = cv[m];
#pragma unroll
      for (int k = 0; k < NK; ++k) {
        const int ex = ks.x[k] - ks.x[m], ey = ks.y[k] - ks.y[m];
        if (k == m || ex < 0 || ey < 0) continue;
        // (-sx)^ex: sx = -1 (dx = 0) gives +1, sx = +1 (dx = 1) gives (-1)^ex
        const double sgn = (((ex & 1) && dx) ? -1.0 : 1.0) * (((ey & 1) && dy) ? -1.0 : 1.0);
        s = fmaf(static_cast<float>(sgn / (cfact(ex) * cfact(ey))), cv[k], s);
      }
      Dc[l][m] = s;
    }
    float C[N1][N1];
    taylor_to_legendre<P>(Dc[l], C);
    bl2[l] = seminorm_sq<P, true>(C, A.Sk);
  }
  // weights of eq. finalweno: linear weights 1 - 4 lin_w (cell), lin_w (vertices)
  float w0, wv[4];
  if (ms.fast_exp) {
    const float d0 = ms.eps_c + fsqrt(n2);
    w0 = (1.0f - 4.0f * ms.lin_w) * frcp(d0 * d0);
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const float dv = ms.eps_c + fsqrt(bl2[l]);
      wv[l] = ms.lin_w * frcp(dv * dv);
    }
  } else {
    w0 = (1.0f - 4.0f * ms.lin_w) * powf(ms.eps_c + powf(sqrtf(n2), ms.q_beta), -ms.r);
#pragma unroll
    for (int l = 0; l < 4; ++l) wv[l] = ms.lin_w * powf(ms.eps_c + powf(sqrtf(bl2[l]), ms.q_beta), -ms.r);
  }
  const float wq = (wv[0] + wv[1]) + (wv[2] + wv[3]);
  const float oinv = frcp(w0 + wq);
  // u_h - u* = sum_{l >= 1} omega_l (u_h - p_l) = (1 - omega_0) u_h - sum omega_l p_l
  float db[NK];
#pragma unroll
  for (int k = 0; k < NK; ++k) {
    float s = wv[0] * Dc[0][k];
    s = fmaf(wv[1], Dc[1][k], s);
    s = fmaf(wv[2], Dc[2][k], s);
    s = fmaf(wv[3], Dc[3][k], s);
    db[k] = s * oinv;
  }
  float Cb[N1][N1];
  taylor_to_legendre<P>(db, Cb);
  const float wrest = wq * oinv;
  float dl[N1][N1];
#pragma unroll
  for (int m = 0; m < N1; ++m)
#pragma unroll
    for (int n = 0; n < N1; ++n) dl[m][n] = fmaf(wrest, cf[m][n], -Cb[m][n]);
  const float d2 = seminorm_sq<P, false>(dl, A.Sk);
  float g = 1.0f;
  if (n2 > 0.0f) {
    const float mr = fminf(1.0f, fsqrt(d2 / n2));     // n2 may be subnormal: IEEE division
    g = 1.0f - (ms.fast_exp ? mr : powf(mr, ms.q_sensor));
  }
  return g;
}

// mode TILE_ALL: gamma of every cell.  TILE_FALLBACK: only the tiles whose
// flag is set, and there only the cells whose gamma holds NaN (the learned
// sensor's hand-over); the flag is cleared.  TILE_AUDIT: gamma is not written;
// the block's sum and maximum of |gamma_plain - g_ref| go to part[2 lb + 0, 1].
// One 16 x 16 tile lb of a mesh (the whole block); the block's threads call
// it together (every exit is block-uniform).  The opening barrier lets a
// block walk several tiles: the previous tile's readers of the LDS vertex
// sums are done before this tile overwrites them.
template <int P>
__device__ __forceinline__ void sensor_tile_body(const float* __restrict__ u, float* __restrict__ gamma,
                                                 const SensorTileArgs& A, const MethodScalars& ms, int64_t lb,
                                                 int mode, uint8_t* __restrict__ tile_flag,
                                                 const float* __restrict__ g_ref, double* __restrict__ part) {
  constexpr int N1 = P + 1, NLOC = N1 * N1, NK = KSet<P>::NK;
  __shared__ float V[NK + 1][NVX * NVX];   // per vertex: sum w D^k (k < NK), sum w (NK)
  __syncthreads();
  if (mode == TILE_FALLBACK && tile_flag[lb] == 0) return;
  const int TI = static_cast<int>(lb % A.tiles_x), TJ = static_cast<int>(lb / A.tiles_x);
  const int i0 = TI * TS, j0 = TJ * TS;
  const int w = min(TS, A.nx - i0), hgt = min(TS, A.ny - j0);
  const int t = threadIdx.x;
  const int ci = t & (TS - 1), cj = t / TS;
  const bool own = ci < w && cj < hgt;
  // the halo ring: rows j = -1 and j = hgt (i = -1 .. w), columns i = -1 and i = w (j = 0 .. hgt - 1)
  const int nh = 2 * (w + 2) + 2 * hgt;
  const bool halo = t < nh;
  int hi = 0, hj = 0;
  if (halo) {
    if (t < w + 2) {
      hi = t - 1;
      hj = -1;
    } else if (t < 2 * (w + 2)) {
      hi = t - (w + 2) - 1;
      hj = hgt;
    } else if (t < 2 * (w + 2) + hgt) {
      hi = -1;
      hj = t - 2 * (w + 2);
    } else {
      hi = w;
      hj = t - 2 * (w + 2) - hgt;
    }
  }
  auto cell_of = [&](int li, int lj) -> int64_t {
    int gi = i0 + li, gj = j0 + lj;
    gi = gi < 0 ? gi + A.nx : (gi >= A.nx ? gi - A.nx : gi);
    gj = gj < 0 ? gj + A.ny : (gj >= A.ny ? gj - A.ny : gj);
    return static_cast<int64_t>(gi) + static_cast<int64_t>(A.nx) * gj;
  };

  // the halo cell first: its corners that touch the tile's vertices (one or
  // two) go to LDS, so that its registers are free again for the own cell
  constexpr int NH = 2 * (TS + 2) + 2 * TS;
  __shared__ float Hs[2][NK + 1][NH];
  int hc0 = -1, hc1 = -1;
  if (halo) {
    float cfh[N1][N1], Wh[4], WHh[4][NK];
    cell_corners<P>(u + cell_of(hi, hj) * NLOC, A, ms, cfh, Wh, WHh);
    int c = 0;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int vx = hi + ((l == 1 || l == 2) ? 1 : 0), vy = hj + ((l >= 2) ? 1 : 0);
      if (vx >= 0 && vx <= w && vy >= 0 && vy <= hgt) {
#pragma unroll
        for (int k = 0; k < NK; ++k) Hs[c][k][t] = WHh[l][k];
        Hs[c][NK][t] = Wh[l];
        if (c == 0) hc0 = l;
        else hc1 = l;
        ++c;
      }
    }
  }
  float cf[N1][N1];
  float Wo[4], WHo[4][NK];
  if (own) cell_corners<P>(u + cell_of(ci, cj) * NLOC, A, ms, cf, Wo, WHo);
  // vertex sums, one corner per round: corner l of cell (i, j) is vertex
  // (i + dx_l, j + dy_l); each vertex of [0, w] x [0, hgt] has exactly one
  // corner-l cell among the tile and its halo, and the corner-0 round covers
  // them all
#pragma unroll
  for (int l = 0; l < 4; ++l) {
    const int dx = (l == 1 || l == 2) ? 1 : 0, dy = (l >= 2) ? 1 : 0;
    if (own) {
      const int v = (ci + dx) + NVX * (cj + dy);
#pragma unroll
      for (int k = 0; k < NK; ++k) V[k][v] = (l == 0) ? WHo[l][k] : V[k][v] + WHo[l][k];
      V[NK][v] = (l == 0) ? Wo[l] : V[NK][v] + Wo[l];
    }
    if (hc0 == l || hc1 == l) {
      const int sl = (hc0 == l) ? 0 : 1;
      const int v = (hi + dx) + NVX * (hj + dy);
#pragma unroll
      for (int k = 0; k < NK; ++k) V[k][v] = (l == 0) ? Hs[sl][k][t] : V[k][v] + Hs[sl][k][t];
      V[NK][v] = (l == 0) ? Hs[sl][NK][t] : V[NK][v] + Hs[sl][NK][t];
    }
    __syncthreads();
  }
  if (mode == TILE_FALLBACK && t == 0) tile_flag[lb] = 0;   // every thread has read it
  float g = 1.0f;
  if (own) g = cell_gamma<P>(cf, V, ci, cj, A, ms);
  if (mode == TILE_AUDIT) {
    // fixed-order block sums (float64) of the deviation from g_ref
    __shared__ double rs[256], rm[256];
    double d = 0.0;
    if (own) {
      const float r = g_ref[cell_of(ci, cj)];
      d = isnan(r) ? 1.0 : fabs(static_cast<double>(g) - static_cast<double>(r));
    }
    rs[t] = d;
    rm[t] = d;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
      if (t < h) {
        rs[t] += rs[t + h];
        rm[t] = fmax(rm[t], rm[t + h]);
      }
      __syncthreads();
    }
    if (t == 0) {
      part[2 * lb] = rs[0];
      part[2 * lb + 1] = rm[0];
    }
    return;
  }
  if (!own) return;
  const int64_t e = cell_of(ci, cj);
  if (mode == TILE_FALLBACK && !isnan(gamma[e])) return;
  gamma[e] = g;
}

template <int P>
__global__ __launch_bounds__(256, 4) void dgq_sensor_tile_kernel(const float* __restrict__ u, float* __restrict__ gamma,
                                                              SensorTileArgs A, MethodScalars ms, int64_t nb_padded,
                                                              int mode, uint8_t* __restrict__ tile_flag,
                                                              const float* __restrict__ g_ref,
                                                              double* __restrict__ part) {
  const int64_t lb = xcd_block(blockIdx.x, nb_padded);
  if (lb >= A.ntiles) return;                           // the whole block leaves
  sensor_tile_body<P>(u, gamma, A, ms, lb, mode, tile_flag, g_ref, part);
}

// Batched stages: the fused pass over the (instance, tile) items of every
// instance of degree P, a fixed stride walk; each tile runs the single-mesh
// body, so gamma is bitwise that of the single-mesh pass.
template <int P>
__global__ __launch_bounds__(256, 4) void batch_sensor_kernel(const BatchInst* __restrict__ inst,
                                                           const int2* __restrict__ items, int n_items, int stage) {
  for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
    const int2 w = items[it];
    const BatchInst& I = inst[w.x];
    sensor_tile_body<P>(I.u_in[stage], I.gam, I.sa, I.ms, w.y, TILE_ALL, nullptr, nullptr, nullptr);
  }
}

// Sum of the audit's block partials in a fixed order: out[0] = mean, out[1] =
// largest |gamma_plain - gamma_learned| over the E cells; a mean above tol sets
// the latch (status word 2: the plain sensor takes every cell from then on)
// and the ST_LEARNED_OFF bit.
__global__ __launch_bounds__(256) void audit_finalize_kernel(const double* __restrict__ part, int64_t ntiles,
                                                             int64_t E, double tol, uint32_t* __restrict__ status,
                                                             double* __restrict__ out) {
  __shared__ double rs[256], rm[256];
  const int t = threadIdx.x;
  double a = 0.0, b = 0.0;
  for (int64_t i = t; i < ntiles; i += 256) {
    a += part[2 * i];
    b = fmax(b, part[2 * i + 1]);
  }
  rs[t] = a;
  rm[t] = b;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (t < h) {
      rs[t] += rs[t + h];
      rm[t] = fmax(rm[t], rm[t + h]);
    }
    __syncthreads();
  }
  if (t == 0) {
    const double mean = rs[0] / static_cast<double>(E);
    out[0] = mean;
    out[1] = rm[0];
    if (!(mean <= tol)) {
      status[2] = 1u;
      atomicOr(status, ST_LEARNED_OFF);
    }
  }
}

// ---------------------------------------------------------------------------
// launcher
// ---------------------------------------------------------------------------
SensorTileArgs make_sensor_tile_args(const cvw_mesh* m) {
  SensorTileArgs A{};
  const int p = m->degree, n1 = p + 1;
  // T[m][i] = (2m + 1) / 2 w_i P_m(xi_i): Legendre coefficients from Gauss-node values
  for (int i = 0; i < n1; ++i) {
    const double x = m->tens.xi[i];
    double P0 = 1.0, P1 = x;
    for (int k = 0; k < n1; ++k) {
      double Pk;
      if (k == 0) Pk = 1.0;
      else if (k == 1) Pk = x;
      else {
        Pk = ((2.0 * k - 1.0) * x * P1 - (k - 1.0) * P0) / k;
        P0 = P1;
        P1 = Pk;
      }
      A.T[k][i] = 0.5 * (2.0 * k + 1.0) * m->tens.wd[i] * Pk;
    }
  }
  const double hx = m->hx, hy = m->hy, he = m->he;
  auto pw = [](double x, int n) { double r = 1.0; for (int i = 0; i < n; ++i) r *= x; return r; };
  int t = 0;
  for (int n = 1; n <= p; ++n)
    for (int j = 0; j <= n; ++j) {
      const int kx = n - j, ky = j;
      A.sk[t] = static_cast<float>(pw(he, n) * pw(2.0 / hx, kx) * pw(2.0 / hy, ky));
      A.Sk[t] = static_cast<float>(0.25 * hx * hy * pw(he, 2 * n - 2) * pw(2.0 / hx, 2 * kx) * pw(2.0 / hy, 2 * ky));
      ++t;
    }
  A.nx = static_cast<int>(m->grid_nx);
  A.ny = static_cast<int>(m->grid_ny);
  A.tiles_x = (A.nx + TS - 1) / TS;
  A.tiles_y = (A.ny + TS - 1) / TS;
  A.ntiles = static_cast<int64_t>(A.tiles_x) * A.tiles_y;
  return A;
}

cvw_status dgquad_sensor_tile(const cvw_mesh* m, const cvw_params* prm, const float* u, float* gamma, hipStream_t s,
                              int mode, uint8_t* tile_flag, const float* g_ref, double* part) {
  if (m->grid_nx <= 0) { set_error("fused sensor pass needs a structured periodic grid"); return CVW_EUNSUPPORTED; }
  // the plain sensor's constants whatever the params' kind (the fallback and
  // the audit of the learned sensor run it too)
  MethodScalars ms = make_scalars(prm);
  ms.sensor_kind = CVW_SENSOR_PLAIN;
  const SensorTileArgs A = make_sensor_tile_args(m);
  const int64_t nb = (A.ntiles + 7) / 8 * 8;
  const dim3 g(static_cast<unsigned>(nb)), b(256);
  switch (m->degree) {
    case 1: hipLaunchKernelGGL(dgq_sensor_tile_kernel<1>, g, b, 0, s, u, gamma, A, ms, nb, mode, tile_flag, g_ref, part); break;
    case 2: hipLaunchKernelGGL(dgq_sensor_tile_kernel<2>, g, b, 0, s, u, gamma, A, ms, nb, mode, tile_flag, g_ref, part); break;
    case 3: hipLaunchKernelGGL(dgq_sensor_tile_kernel<3>, g, b, 0, s, u, gamma, A, ms, nb, mode, tile_flag, g_ref, part); break;
    default: set_error("degree not supported on the GPU path"); return CVW_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

cvw_status batch_sensor_pass(int P, const BatchInst* inst, const int2* items, int n_items, int stage, int grid,
                             hipStream_t s) {
  if (n_items <= 0) return CVW_OK;
  const dim3 g(std::max(1, std::min(grid, n_items))), b(256);
  switch (P) {
    case 1: hipLaunchKernelGGL(batch_sensor_kernel<1>, g, b, 0, s, inst, items, n_items, stage); break;
    case 2: hipLaunchKernelGGL(batch_sensor_kernel<2>, g, b, 0, s, inst, items, n_items, stage); break;
    case 3: hipLaunchKernelGGL(batch_sensor_kernel<3>, g, b, 0, s, inst, items, n_items, stage); break;
    default: set_error("degree not supported on the GPU path"); return CVW_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

int64_t sensor_tiles(const cvw_mesh* m) {
  return m->grid_nx <= 0 ? 0 : ((m->grid_nx + TS - 1) / TS) * ((m->grid_ny + TS - 1) / TS);
}

cvw_status dgquad_audit_finalize(const cvw_mesh* m, const double* part, double tol, uint32_t* status, double* out,
                                 hipStream_t s) {
  hipLaunchKernelGGL(audit_finalize_kernel, dim3(1), dim3(256), 0, s, part, sensor_tiles(m), m->E, tol, status, out);
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

}  // namespace cvw
