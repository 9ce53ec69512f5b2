// HWENO limiter on DG quadrilaterals, gfx950 (the kernels behind cvw_limit).
#include "cvw_device.h"
#include "cvw_dgq_common.h"
#include "cvw_limit.h"

namespace cvw {

// ---------------------------------------------------------------------------
// HWENO limiter: the cell-vertex reconstruction u_h^{e,*} (eq. finalweno)
// overwrites u_h^e on the cells whose sensor value is below a threshold, with
// the vertex candidates' cell averages corrected to that of u_h^e (Sec. 3.2).
// With the candidates written about the cell centre,
//   u_h^{e,*} = w_0 u_h^e + (1 - w_0) mean(u_h^e) + V - mean(V),
//   V(x) = sum_{|k|>=1} cb_k (x - x_c)^k / k!,  cb = sum_{l>=1} w_l D^k u_{h,l}(x_c),
// since the constant terms of the candidates cancel in the correction.  One
// thread per (cell, variable), float64 inside, each variable with its own
// candidates and weights (componentwise).
// ---------------------------------------------------------------------------
template <int P>
__device__ __forceinline__ void taylor_move_d(const double (&c)[KSet<P>::NK], double X, double Y,
                                              double (&o)[KSet<P>::NK]) {
  constexpr int NK = KSet<P>::NK;
  constexpr KSet<P> ks = kset<P>;
  constexpr double inv_n[4] = {1.0, 1.0, 0.5, 1.0 / 3.0};
  double px[P + 1], py[P + 1];
  px[0] = py[0] = 1.0;
#pragma unroll
  for (int n = 1; n <= P; ++n) {
    px[n] = px[n - 1] * X * inv_n[n];
    py[n] = py[n - 1] * Y * inv_n[n];
  }
#pragma unroll
  for (int t = 0; t < NK; ++t) {
    double s = c[t];
#pragma unroll
    for (int t2 = 0; t2 < NK; ++t2) {
      const int i = ks.x[t2] - ks.x[t], j = ks.y[t2] - ks.y[t];
      if (t2 != t && i >= 0 && j >= 0) s = fma(c[t2], px[i] * py[j], s);
    }
    o[t] = s;
  }
}

// sum_k h_e^{2|k|-2} int_K (D^k p)^2 (eq. snorm, d = 2) for the polynomial of
// total degree <= P with derivatives ch at the centre of an hx x hy cell:
// D^k p has degree <= 2 in the centred (X, Y) and its mean square is a sum of
// squares in the orthogonal basis 1, X, (X^2 - hx^2/12)/2, Y, XY, ...
template <int P>
__device__ __forceinline__ double centred_seminorm_d(const double (&ch)[KSet<P>::NK], double hx, double hy,
                                                    double he2) {
  constexpr int NK = KSet<P>::NK;
  constexpr KSet<P> ks = kset<P>;
  const double mx2 = hx * hx / 12.0, my2 = hy * hy / 12.0;
  const double qx4 = hx * hx * hx * hx / 720.0, qy4 = hy * hy * hy * hy / 720.0;
  double tot = 0.0;
#pragma unroll
  for (int t = 0; t < NK; ++t) {
    double A = ch[t], rest = 0.0;
#pragma unroll
    for (int t2 = 0; t2 < NK; ++t2) {
      const int i = ks.x[t2] - ks.x[t], j = ks.y[t2] - ks.y[t];
      if (t2 == t || i < 0 || j < 0) continue;
      const double c = ch[t2];
      if (i == 1 && j == 0) rest += mx2 * c * c;
      if (i == 0 && j == 1) rest += my2 * c * c;
      if (i == 1 && j == 1) rest += mx2 * my2 * c * c;
      if (i == 2 && j == 0) {
        A += 0.5 * mx2 * c;
        rest += qx4 * c * c;
      }
      if (i == 0 && j == 2) {
        A += 0.5 * my2 * c;
        rest += qy4 * c * c;
      }
    }
    tot += dpow(he2, ks.x[t] + ks.y[t] - 1) * (A * A + rest);
  }
  return hx * hy * tot;
}

// Appends the ids of the selected threads of a block (a multiple of 64
// threads, at most 1024) to
// list[0 .. *count): one atomic per block (atomics on one address serialise
// in the cache, so they are kept few), the threads in order behind it (the
// blocks in any order).  Every thread of the block must call it.
__device__ __forceinline__ void append_selected(bool sel, int64_t id, uint32_t* __restrict__ count,
                                                int32_t* __restrict__ list) {
  __shared__ uint32_t wbase[16];
  __shared__ uint32_t bbase;
  const uint64_t mask = __builtin_amdgcn_ballot_w64(sel);
  const uint32_t below = __builtin_amdgcn_mbcnt_hi(static_cast<uint32_t>(mask >> 32),
                                                   __builtin_amdgcn_mbcnt_lo(static_cast<uint32_t>(mask), 0u));
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) wbase[wave] = static_cast<uint32_t>(__builtin_popcountll(mask));
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < static_cast<int>(blockDim.x >> 6); ++w) {
      const uint32_t c = wbase[w];
      wbase[w] = run;
      run += c;
    }
    bbase = run ? atomicAdd(count, run) : 0u;
  }
  __syncthreads();
  if (sel) list[bbase + wbase[wave] + below] = static_cast<int32_t>(id);
}

// Cells to reconstruct: list[0 .. count[0]) (any order: every cell's result
// is its own).
__global__ __launch_bounds__(1024) void dgq_limit_select_kernel(const float* __restrict__ gamma, int64_t E,
                                                                double threshold, uint32_t* __restrict__ count,
                                                                int32_t* __restrict__ list) {
  const int64_t e = blockIdx.x * 1024LL + threadIdx.x;
  append_selected(e < E && static_cast<double>(gamma[e]) < threshold, e, count, list);
}

// Vertices of the selected cells: vlist[0 .. count[1]).
__global__ __launch_bounds__(1024) void dgq_limit_select_vertices_kernel(const uint8_t* __restrict__ vflag,
                                                                         int64_t Nv, uint32_t* __restrict__ count,
                                                                         int32_t* __restrict__ vlist) {
  const int64_t i = blockIdx.x * 1024LL + threadIdx.x;
  append_selected(i < Nv && vflag[i] != 0, i, count + 1, vlist);
}

__global__ void dgq_limit_clear_kernel(uint32_t* __restrict__ count) {
  if (threadIdx.x < 2) count[threadIdx.x] = 0u;
}

__global__ __launch_bounds__(256) void dgq_limit_clear_flags_kernel(uint8_t* __restrict__ vflag, int64_t Nv) {
  const int64_t i = blockIdx.x * 256LL + threadIdx.x;
  if (i < Nv) vflag[i] = 0;
}

// flags the vertices of the listed cells (their candidates are needed)
__global__ __launch_bounds__(256) void dgq_limit_mark_kernel(const uint32_t* __restrict__ count,
                                                             const int32_t* __restrict__ list,
                                                             const int32_t* __restrict__ cell_vtx,
                                                             uint8_t* __restrict__ vflag, int64_t E) {
  const int64_t k = blockIdx.x * 256LL + threadIdx.x;
  if (k >= static_cast<int64_t>(*count) || k >= E) return;
  const int64_t e = list[k];
#pragma unroll
  for (int l = 0; l < 4; ++l) vflag[cell_vtx[e * 4 + l]] = 1;
}

// One thread per (listed cell, variable) (the grid covers every cell; threads
// past the count leave), or with list == nullptr per (cell, variable).  Cells
// not reconstructed have been copied from u to out beforehand where they differ.
template <int P, int NV>
__global__ __launch_bounds__(256) void dgq_limit_kernel(const float* __restrict__ u, float* __restrict__ out,
                                                        const float* __restrict__ cand,
                                                        const uint32_t* __restrict__ count,
                                                        const int32_t* __restrict__ list,
                                                        const int32_t* __restrict__ cell_vtx, TensorTables tab,
                                                        LimitNodes ln, int64_t E, int64_t Nv, double hx, double hy,
                                                        double he, MethodScalars ms) {
  constexpr int N1 = P + 1, NLOC = N1 * N1, NK = KSet<P>::NK;
  constexpr KSet<P> ks = kset<P>;
  const int64_t k = (blockIdx.x * 256LL + threadIdx.x) / NV;
  const int v = static_cast<int>((blockIdx.x * 256LL + threadIdx.x) % NV);
  if (k >= (list ? static_cast<int64_t>(*count) : E)) return;
  const int64_t e = list ? list[k] : k;
  const double sx = 2.0 / hx, sy = 2.0 / hy, he2 = he * he;
  const double lin = ms.lin_wd, lin0 = 1.0 - 4.0 * ms.lin_wd;
  const double q = static_cast<double>(ms.q_beta), rr = static_cast<double>(ms.r);
  int32_t vtx[4];
#pragma unroll
  for (int l = 0; l < 4; ++l) vtx[l] = cell_vtx[e * 4 + l];
  {
    const float* ue = u + (static_cast<int64_t>(v) * E + e) * NLOC;
    float* oe = out + (static_cast<int64_t>(v) * E + e) * NLOC;
    float raw[NLOC];
#pragma unroll
    for (int j = 0; j < NLOC; ++j) raw[j] = ue[j];
    // data relative to the first node (exact differences in float64)
    const double r0 = raw[0];
    double r[NLOC];
#pragma unroll
    for (int j = 0; j < NLOC; ++j) r[j] = static_cast<double>(raw[j]) - r0;
    // element semi-norm of u_h^e on the collocated Gauss rule (exact for it)
    double n2 = 0.0, mean_r = 0.0;
#pragma unroll 1
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
          d *= dpow(sx, ks.x[t]) * dpow(sy, ks.y[t]);
          pq = fma(dpow(he2, ks.x[t] + ks.y[t] - 1) * d, d, pq);
        }
        n2 = fma(ln.w[a] * ln.w[b] * 0.25 * hx * hy, pq, n2);
        mean_r = fma(ln.w[a] * ln.w[b] * 0.25, r[a + N1 * b], mean_r);
      }
    }
    // nonlinear weights of the cell candidate and the four vertex candidates
    // (the vertices' Taylor data moved to the cell centre)
    const float* cv = cand + static_cast<int64_t>(v) * Nv * NK;
    auto wfun = [&](double g, double b2) {
      const double beta = ms.fast_exp ? sqrt(b2) : pow(sqrt(b2), q);
      const double den = ms.eps_cd + beta;
      return ms.fast_exp ? g / (den * den) : g * pow(den, -rr);
    };
    double wl[4];
    const double w0 = wfun(lin0, n2);
    double tot = w0;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      double c[NK], ch[NK];
#pragma unroll
      for (int t = 0; t < NK; ++t) c[t] = static_cast<double>(cv[static_cast<int64_t>(vtx[l]) * NK + t]);
      const double xl = (l == 1 || l == 2) ? 0.5 * hx : -0.5 * hx, yl = (l >= 2) ? 0.5 * hy : -0.5 * hy;
      taylor_move_d<P>(c, -xl, -yl, ch);
      wl[l] = wfun(lin, centred_seminorm_d<P>(ch, hx, hy, he2));
      tot += wl[l];
    }
    const double om0 = w0 / tot;
    double cb[NK], wrest = 0.0;
#pragma unroll
    for (int t = 0; t < NK; ++t) cb[t] = 0.0;
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      double c[NK], ch[NK];
#pragma unroll
      for (int t = 0; t < NK; ++t) c[t] = static_cast<double>(cv[static_cast<int64_t>(vtx[l]) * NK + t]);
      const double xl = (l == 1 || l == 2) ? 0.5 * hx : -0.5 * hx, yl = (l >= 2) ? 0.5 * hy : -0.5 * hy;
      taylor_move_d<P>(c, -xl, -yl, ch);
      const double om = wl[l] / tot;
      wrest += om;
#pragma unroll
      for (int t = 0; t < NK; ++t) cb[t] = fma(om, ch[t], cb[t]);
    }
    // mean of V over the cell: only (2, 0) and (0, 2) survive
    double meanV = 0.0;
#pragma unroll
    for (int t = 0; t < NK; ++t) {
      if (ks.x[t] == 2 && ks.y[t] == 0) meanV += cb[t] * hx * hx / 24.0;
      if (ks.x[t] == 0 && ks.y[t] == 2) meanV += cb[t] * hy * hy / 24.0;
    }
    const double base = r0 + wrest * mean_r - meanV;
#pragma unroll 1
    for (int b = 0; b < N1; ++b)
#pragma unroll
      for (int a = 0; a < N1; ++a) {
        const double X = 0.5 * hx * ln.xi[a], Y = 0.5 * hy * ln.xi[b];
        double V = 0.0;
#pragma unroll
        for (int t = 0; t < NK; ++t) {
          const int kx = ks.x[t], ky = ks.y[t];
          constexpr double fct[4] = {1.0, 1.0, 2.0, 6.0};
          V = fma(cb[t], dpow(X, kx) * dpow(Y, ky) / (fct[kx] * fct[ky]), V);
        }
        oe[a + N1 * b] = static_cast<float>(base + om0 * r[a + N1 * b] + V);
      }
  }
}

cvw_status limit_select(const float* gamma, int64_t E, double threshold, uint32_t* count, int32_t* list,
                        hipStream_t s) {
  hipLaunchKernelGGL(dgq_limit_clear_kernel, dim3(1), dim3(64), 0, s, count);
  hipLaunchKernelGGL(dgq_limit_select_kernel, dim3(static_cast<unsigned>((E + 1023) / 1024)), dim3(1024), 0, s, gamma,
                     E, threshold, count, list);
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

cvw_status dgquad_limit(const cvw_mesh* m, const cvw_params* prm, const float* u, float* out, float* cand,
                        const float* gamma, const LimitNodes& ln, double threshold, uint32_t* count,
                        int32_t* list, uint8_t* vflag, int32_t* vlist, hipStream_t s) {
  const MethodScalars ms = make_scalars(prm);
  const dim3 g(static_cast<unsigned>((m->E + 255) / 256)), b(256);
  const bool sys = prm->flux == CVW_EULER;
  const int nv = sys ? 4 : 1;
  const dim3 gv(static_cast<unsigned>((m->E * nv + 255) / 256));
  cvw_status st;
  // the plain sensor gives gamma_e <= 1: a threshold above 1 (and above a
  // fixed gamma) selects every cell, which are then taken in order without a
  // list, and every vertex needs the candidates of every variable
  if (threshold > 1.0 && (prm->sensor != CVW_SENSOR_FIXED || prm->fixed_gamma < threshold)) {
    list = nullptr;
    for (int v = 1; v < nv; ++v)
      if ((st = dgquad_candidates(m, prm, u + static_cast<int64_t>(v) * m->E * m->nloc,
                                  cand + static_cast<int64_t>(v) * m->Nv * m->nk, s)) != CVW_OK)
        return st;
  } else {
    if (out != u &&
        hipMemcpyAsync(out, u, static_cast<size_t>(m->E) * m->nloc * nv * sizeof(float), hipMemcpyDeviceToDevice,
                       s) != hipSuccess) {
      set_error("state copy failed"); return CVW_EDEVICE;
    }
    hipLaunchKernelGGL(dgq_limit_clear_kernel, dim3(1), dim3(64), 0, s, count);
    hipLaunchKernelGGL(dgq_limit_select_kernel, dim3(static_cast<unsigned>((m->E + 1023) / 1024)), dim3(1024), 0, s,
                       gamma, m->E, threshold, count, list);
    if (nv > 1) {
      // the other variables' candidates only at the vertices of selected cells
      hipLaunchKernelGGL(dgq_limit_clear_flags_kernel, dim3(static_cast<unsigned>((m->Nv + 255) / 256)), b, 0, s,
                         vflag, m->Nv);
      hipLaunchKernelGGL(dgq_limit_mark_kernel, g, b, 0, s, count, list, m->d_cell_vtx, vflag, m->E);
      hipLaunchKernelGGL(dgq_limit_select_vertices_kernel, dim3(static_cast<unsigned>((m->Nv + 1023) / 1024)),
                         dim3(1024), 0, s, vflag, m->Nv, count, vlist);
      for (int v = 1; v < nv; ++v)
        if ((st = dgquad_candidates(m, prm, u + static_cast<int64_t>(v) * m->E * m->nloc,
                                    cand + static_cast<int64_t>(v) * m->Nv * m->nk, s, count + 1, vlist)) !=
            CVW_OK)
          return st;
    }
  }
#define CVW_LIMIT_LAUNCH(P)                                                                                        \
  if (sys)                                                                                                          \
    hipLaunchKernelGGL((dgq_limit_kernel<P, 4>), gv, b, 0, s, u, out, cand, count, list, m->d_cell_vtx, m->tens, ln,\
                       m->E, m->Nv, m->hx, m->hy, m->he, ms);                                                       \
  else                                                                                                              \
    hipLaunchKernelGGL((dgq_limit_kernel<P, 1>), gv, b, 0, s, u, out, cand, count, list, m->d_cell_vtx, m->tens, ln,\
                       m->E, m->Nv, m->hx, m->hy, m->he, ms);
  switch (m->degree) {
    case 1: CVW_LIMIT_LAUNCH(1) break;
    case 2: CVW_LIMIT_LAUNCH(2) break;
    case 3: CVW_LIMIT_LAUNCH(3) break;
    default: set_error("degree not supported on the GPU path"); return CVW_EUNSUPPORTED;
  }
#undef CVW_LIMIT_LAUNCH
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

// ---------------------------------------------------------------------------
// Positivity limiter for the Euler equations (the Zhang-Shu scaling limiter
// the paper adds for its double Mach reflection run, Sec. 5, restated from the
// published construction).  One thread per cell, float64 inside.  Points Q:
// the Gauss nodes and the Gauss points of the four faces; eps = min(eps0,
// rhobar, p(Ubar)).  (1) density scaled towards its cell average until
// min_Q rho = eps; (2) the state scaled towards the cell average by the
// smallest t in [0, 1] at which the pressure along Ubar + t (U_q - Ubar) reaches
// eps (the root of a quadratic: 2 rho E - |m|^2 - 2 eps rho / (gamma - 1) is
// quadratic in t and positive at t = 0).  Cells already admissible are left
// as they are (out of place, the state is copied to out first).
// ---------------------------------------------------------------------------
// l_i(-1) of the element, float64 (face traces; l_i(+1) = l_{p-i}(-1) on the
// symmetric Gauss nodes)
struct PositivityTraces {
  double l0[MAXP + 1];
};

__device__ __forceinline__ double pos_root(double a, double b, double c) {
  // the root in [0, 1] of a t^2 + b t + c with c >= 0 > a + b + c
  if (fabs(a) <= 1e-14 * (fabs(b) + fabs(c))) return b != 0.0 ? fmin(1.0, fmax(0.0, -c / b)) : 0.0;
  const double disc = fmax(0.0, b * b - 4.0 * a * c);
  const double q = -0.5 * (b + copysign(sqrt(disc), b));
  const double t1 = q / a, t2 = (q != 0.0) ? c / q : 2.0;
  double t = 2.0;
  if (t1 >= 0.0 && t1 <= 1.0) t = t1;
  if (t2 >= 0.0 && t2 <= 1.0) t = fmin(t, t2);
  return t <= 1.0 ? t : 0.0;
}

// Stage 1, one thread per cell (512-thread blocks): the float32 pre-check below, the copy to
// out (out of place), and the list of cells that fail the pre-check:
// list[0 .. count[0]).
template <int P>
__global__ __launch_bounds__(512) void dgq_positivity_check_kernel(const float* __restrict__ u,
                                                                    float* __restrict__ out, int64_t E,
                                                                    PositivityTraces tr, double gam, double eps0,
                                                                    uint32_t* __restrict__ count,
                                                                    int32_t* __restrict__ list) {
  constexpr int N1 = P + 1, NLOC = N1 * N1, NQ = NLOC + 4 * N1;
  const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  bool pass = true;
  if (e < E)
  // float32 pre-check at the nodes and face points.  Each face value carries
  // the bound 1e-5 * sum |l_i u_i| on its float32 rounding (the true error is
  // below 4e-7 times that sum), and the density and pressure are bounded from
  // below with those errors.  A cell whose bounds clear 2 eps0 has float64
  // density and pressure >= eps0 >= eps at every point, so the float64 path
  // below would leave it unchanged: it is skipped.
  {
    bool clear = true;
    const float gm1f = static_cast<float>(gam - 1.0);
    const float tol = 2.0f * static_cast<float>(eps0);
    float F[4][NLOC];
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int j = 0; j < NLOC; ++j) F[v][j] = u[(static_cast<int64_t>(v) * E + e) * NLOC + j];
    if (out != u) {
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int j = 0; j < NLOC; ++j) out[(static_cast<int64_t>(v) * E + e) * NLOC + j] = F[v][j];
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
      float w[4], d[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (q < NLOC) {
          w[v] = F[v][q];
          d[v] = 0.0f;
        } else {
          const int f = (q - NLOC) / N1, k = (q - NLOC) % N1;
          float sv = 0.0f, sa = 0.0f;
#pragma unroll
          for (int i = 0; i < N1; ++i) {
            const float li = static_cast<float>((f == 0 || f == 2) ? tr.l0[i] : tr.l0[P - i]);
            const float x = (f < 2) ? F[v][i + N1 * k] : F[v][k + N1 * i];
            sv = fmaf(li, x, sv);
            sa = fmaf(fabsf(li), fabsf(x), sa);
          }
          w[v] = sv;
          d[v] = 1e-5f * sa;
        }
      }
      const float rlo = w[0] - d[0] - 1e-5f * fabsf(w[0]);
      const float mx = fabsf(w[1]) + d[1], my = fabsf(w[2]) + d[2];
      const float kin = 0.5f * (mx * mx + my * my) / rlo;
      const float elo = w[3] - d[3];
      const float plo = gm1f * (elo - kin - 1e-5f * (fabsf(elo) + kin));
      clear = clear && (rlo > tol) && (plo > tol);
    }
    pass = clear;
  }
  append_selected(e < E && !pass, e, count, list);
}

// Stage 2, one thread per listed cell (the grid covers every cell; threads
// past the count leave): the limiter in float64.  out already holds u.
template <int P>
__global__ __launch_bounds__(128) void dgq_positivity_kernel(const float* __restrict__ u, float* __restrict__ out,
                                                              int64_t E, LimitNodes ln, PositivityTraces tr,
                                                              double gam, double eps0,
                                                              const uint32_t* __restrict__ count,
                                                              const int32_t* __restrict__ list) {
  constexpr int N1 = P + 1, NLOC = N1 * N1, NQ = NLOC + 4 * N1;
  const int64_t k = blockIdx.x * 128LL + threadIdx.x;
  if (k >= static_cast<int64_t>(*count) || k >= E) return;
  const int64_t e = list[k];
  double U[4][NLOC];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int j = 0; j < NLOC; ++j) U[v][j] = u[(static_cast<int64_t>(v) * E + e) * NLOC + j];
  double m[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < N1; ++b)
#pragma unroll
      for (int a = 0; a < N1; ++a) s = fma(0.25 * ln.w[a] * ln.w[b], U[v][a + N1 * b], s);
    m[v] = s;
  }
  const double gm1 = gam - 1.0;
  auto pres = [&](double r, double mx, double my, double en) { return gm1 * (en - 0.5 * (mx * mx + my * my) / r); };
  const double eps = fmin(eps0, fmin(m[0], pres(m[0], m[1], m[2], m[3])));
  // the state at point q (nodes, then W, E, S, N face points)
  auto at = [&](const double (&V)[NLOC], int q) {
    if (q < NLOC) return V[q];
    const int f = (q - NLOC) / N1, k = (q - NLOC) % N1;
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < N1; ++i) {
      const double li = (f == 0 || f == 2) ? tr.l0[i] : tr.l0[P - i];       // l_i(-1) or l_i(+1)
      s = fma(li, (f < 2) ? V[i + N1 * k] : V[k + N1 * i], s);
    }
    return s;
  };
  // (1) density
  double rmin = 1e300;
#pragma unroll
  for (int q = 0; q < NQ; ++q) rmin = fmin(rmin, at(U[0], q));
  bool changed = false;
  if (rmin < eps) {
    const double th1 = fmin(1.0, (m[0] - eps) / (m[0] - rmin));
#pragma unroll
    for (int j = 0; j < NLOC; ++j) U[0][j] = m[0] + th1 * (U[0][j] - m[0]);
    changed = true;
  }
  // (2) pressure
  double th2 = 1.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double r = at(U[0], q), mx = at(U[1], q), my = at(U[2], q), en = at(U[3], q);
    if (pres(r, mx, my, en) >= eps) continue;
    const double dr = r - m[0], dx = mx - m[1], dy = my - m[2], de = en - m[3];
    const double k2 = 2.0 * eps / gm1;
    const double a = 2.0 * dr * de - (dx * dx + dy * dy);
    const double b = 2.0 * (m[0] * de + dr * m[3]) - 2.0 * (m[1] * dx + m[2] * dy) - k2 * dr;
    const double c = 2.0 * m[0] * m[3] - (m[1] * m[1] + m[2] * m[2]) - k2 * m[0];
    th2 = fmin(th2, pos_root(a, b, c));
  }
  if (th2 < 1.0) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int j = 0; j < NLOC; ++j) U[v][j] = m[v] + th2 * (U[v][j] - m[v]);
    changed = true;
  }
  if (!changed) return;                         // out holds u's values already
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int j = 0; j < NLOC; ++j) out[(static_cast<int64_t>(v) * E + e) * NLOC + j] = static_cast<float>(U[v][j]);
}

// The same limiter on DG triangles, one thread per cell, float64 inside: the
// state at the points Q (the volume rule's, where the scheme evaluates it,
// then the Gauss points of the three edges) from the float64 tables, the cell
// average as weights of the nodal values; a limited cell is written, an
// admissible one copied when not in place.
template <int P>
__global__ __launch_bounds__(128) void tri_positivity_kernel(const float* __restrict__ u, float* __restrict__ out,
                                                             int64_t E, const TriTables* __restrict__ T,
                                                             double gam, double eps0, int copy) {
  constexpr int NL = (P + 1) * (P + 2) / 2, NQV = (P + 1) * (P + 1), NQ = NQV + 3 * (P + 1);
  const int64_t e = blockIdx.x * 128LL + threadIdx.x;
  if (e >= E) return;
  double U[4][NL];
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int j = 0; j < NL; ++j) U[v][j] = u[(static_cast<int64_t>(v) * E + e) * NL + j];
  double m[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NL; ++j) s = fma(T->mwd[j], U[v][j], s);
    m[v] = s;
  }
  const double gm1 = gam - 1.0;
  auto pres = [&](double r, double mx, double my, double en) { return gm1 * (en - 0.5 * (mx * mx + my * my) / r); };
  const double eps = fmin(eps0, fmin(m[0], pres(m[0], m[1], m[2], m[3])));
  auto at = [&](const double (&V)[NL], int q) {
    double s = 0.0;
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const double b = (q < NQV) ? T->Bd[q][j] : T->Bfd[(q - NQV) / (P + 1)][(q - NQV) % (P + 1)][j];
      s = fma(b, V[j], s);
    }
    return s;
  };
  // (1) density
  double rmin = 1e300;
#pragma unroll
  for (int q = 0; q < NQ; ++q) rmin = fmin(rmin, at(U[0], q));
  bool changed = false;
  if (rmin < eps) {
    const double th1 = fmin(1.0, (m[0] - eps) / (m[0] - rmin));
#pragma unroll
    for (int j = 0; j < NL; ++j) U[0][j] = m[0] + th1 * (U[0][j] - m[0]);
    changed = true;
  }
  // (2) pressure: the smallest root in [0, 1] of p(Ubar + t (U_q - Ubar)) = eps over Q
  double th2 = 1.0;
#pragma unroll
  for (int q = 0; q < NQ; ++q) {
    const double r = at(U[0], q), mx = at(U[1], q), my = at(U[2], q), en = at(U[3], q);
    if (pres(r, mx, my, en) >= eps) continue;
    const double dr = r - m[0], dx = mx - m[1], dy = my - m[2], de = en - m[3];
    const double k2 = 2.0 * eps / gm1;
    const double a = 2.0 * dr * de - (dx * dx + dy * dy);
    const double b = 2.0 * (m[0] * de + dr * m[3]) - 2.0 * (m[1] * dx + m[2] * dy) - k2 * dr;
    const double c = 2.0 * m[0] * m[3] - (m[1] * m[1] + m[2] * m[2]) - k2 * m[0];
    th2 = fmin(th2, pos_root(a, b, c));
  }
  if (th2 < 1.0) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
#pragma unroll
      for (int j = 0; j < NL; ++j) U[v][j] = m[v] + th2 * (U[v][j] - m[v]);
    changed = true;
  }
  if (!changed && !copy) return;
#pragma unroll
  for (int v = 0; v < 4; ++v)
#pragma unroll
    for (int j = 0; j < NL; ++j) {
      const int64_t i = (static_cast<int64_t>(v) * E + e) * NL + j;
      out[i] = changed ? static_cast<float>(U[v][j]) : u[i];
    }
}

cvw_status tri_positivity(const cvw_mesh* m, const float* u, float* out, double gam, double eps0, hipStream_t s) {
  const dim3 g(static_cast<unsigned>((m->E + 127) / 128)), b(128);
  const int copy = (out != u) ? 1 : 0;
  switch (m->degree) {
    case 1: hipLaunchKernelGGL(tri_positivity_kernel<1>, g, b, 0, s, u, out, m->E, m->d_trit, gam, eps0, copy); break;
    case 2: hipLaunchKernelGGL(tri_positivity_kernel<2>, g, b, 0, s, u, out, m->E, m->d_trit, gam, eps0, copy); break;
    case 3: hipLaunchKernelGGL(tri_positivity_kernel<3>, g, b, 0, s, u, out, m->E, m->d_trit, gam, eps0, copy); break;
    default: set_error("degree not supported on the GPU path"); return CVW_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

cvw_status dgquad_positivity(const cvw_mesh* m, const float* u, float* out, const LimitNodes& ln, double gam,
                             double eps0, uint32_t* count, int32_t* list, hipStream_t s) {
  PositivityTraces tr{};
  for (int i = 0; i <= MAXP; ++i) tr.l0[i] = m->tens.Ld[0][i];
  hipLaunchKernelGGL(dgq_limit_clear_kernel, dim3(1), dim3(64), 0, s, count);
  constexpr int CHECK_BS = 512;      // measured: 1024, 512, 256 threads
  const dim3 g1(static_cast<unsigned>((m->E + CHECK_BS - 1) / CHECK_BS)), b1(CHECK_BS);
  const dim3 g2(static_cast<unsigned>((m->E + 127) / 128)), b2(128);
  switch (m->degree) {
#define CVW_POS(PP)                                                                                  \
  case PP:                                                                                           \
    hipLaunchKernelGGL(dgq_positivity_check_kernel<PP>, g1, b1, 0, s, u, out, m->E, tr, gam, eps0,   \
                       count, list);                                                                 \
    hipLaunchKernelGGL(dgq_positivity_kernel<PP>, g2, b2, 0, s, u, out, m->E, ln, tr, gam, eps0,     \
                       static_cast<const uint32_t*>(count), static_cast<const int32_t*>(list));      \
    break;
    CVW_POS(1)
    CVW_POS(2)
    CVW_POS(3)
#undef CVW_POS
    default: set_error("degree not supported on the GPU path"); return CVW_EUNSUPPORTED;
  }
  return hipGetLastError() == hipSuccess ? CVW_OK : CVW_EDEVICE;
}

}  // namespace cvw
