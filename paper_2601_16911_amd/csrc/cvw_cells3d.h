// Tables and launchers of the 3D cells: DG hexahedra (cvw_hex.hip) and DG
// tetrahedra (cvw_tet.hip).  Built by the mesh build (cvw_host.cpp).
#pragma once
#include "cvw_internal.h"

namespace cvw {

// Hexahedra: DG Q_p (p <= HEX_MAXP) on congruent axis-aligned boxes.  Local
// node a + n1 b + n1^2 c (x fastest) at the Gauss points; the polynomial of a
// cell in the monomials xi^A of its reference coordinates, A = (a, b, c),
// index a + n1 b + n1^2 c; multi-indices k, 1 <= |k| <= p, in the order of
// the Hermite data (by |k|, then decreasing first, then decreasing second
// component).  Built for the mesh's box sides (hx, hy, hz).
constexpr int HEX_MAXP = 2;
constexpr int HEX_N1 = HEX_MAXP + 1, HEX_NL = HEX_N1 * HEX_N1 * HEX_N1;
constexpr int HEX_NK = (HEX_MAXP + 1) * (HEX_MAXP + 2) * (HEX_MAXP + 3) / 6 - 1;
struct HexTables {
  int p, n1, nl, nk;
  float w1[HEX_N1];                      // Gauss weights on [-1, 1]
  float D1[HEX_N1][HEX_N1];              // l_j'(x_q)
  float D2[HEX_N1][HEX_N1];              // l_j''(x_q)
  float Lend[2][HEX_N1];                 // l_j(-1), l_j(+1)
  float sc[3];                           // 2 / h_d
  float W0;                              // hx hy hz / 8
  float Jf[3];                           // face Jacobian of the faces normal to axis d (area / 4)
  float he, nuf;                         // diam K_e, h_e / (2p)
  float wa[HEX_NK];                      // alpha~: h_e^{2|k|} prod_d (2 / h_d)^{2 k_d}
  int8_t kk[HEX_NK][3];                  // the multi-indices
  int8_t kmono[HEX_NL];                  // monomial A -> its index among the k (-1: A = 0 or |A| > p)
  double hb[HEX_NK];                     // vertex beta: h_e^{2|k|}
  double T1[HEX_N1][HEX_N1];             // u(xi) = sum_a (sum_j T1[a][j] u_j) xi^a along one direction
  double G[HEX_NL][HEX_NL];              // sum_k h_e^{2|k|-3} int_K D^k xi^A D^k xi^B dx
  double E1[HEX_N1][2][HEX_N1];          // l_j^{(m)}(-1), l_j^{(m)}(+1): reference derivatives at the ends
  double hk[HEX_NK];                     // prod_d (2 / h_d)^{k_d}: reference -> physical derivatives
  double R[8][HEX_NK][HEX_NK];           // vertex candidate of vertex l (Taylor data) -> coefficient of xi^a, a in k
};

// Tetrahedra: DG P_p (p <= TET_MAXP) at the equispaced lattice points of the
// reference tetrahedron (0,0,0), (1,0,0), (0,1,0), (0,0,1) (i fastest, then
// j, then k); volume rule the conical product of (p+1)^3 points; face f is
// opposite vertex f, its points Radon's symmetric 7-point rule on the face's
// vertices (f+1.., increasing).  Multi-indices as for hexahedra.
constexpr int TET_MAXP = 2;
constexpr int TET_NLOC = (TET_MAXP + 1) * (TET_MAXP + 2) * (TET_MAXP + 3) / 6;
constexpr int TET_NK = TET_NLOC - 1, TET_NQ = (TET_MAXP + 1) * (TET_MAXP + 1) * (TET_MAXP + 1), TET_NFP = 7;
struct TetTables {
  int p, nloc, nk, nq;
  double B[TET_NQ][TET_NLOC];            // phi_j at the volume points
  double G[3][TET_NQ][TET_NLOC];         // d phi_j / d xi_b at the volume points
  double H2[6][TET_NLOC];                // second reference derivatives (xx, xy, xz, yy, yz, zz; constant for p <= 2)
  double Gc[3][TET_NLOC];                // d phi_j / d xi_b at the centroid (1/4, 1/4, 1/4)
  double xq[TET_NQ][3], wq[TET_NQ];      // volume points and weights (the weights sum to 1/6)
  float Bs[TET_NQ][TET_NLOC];            // float32 copies for the residual: phi_j, d phi_j / d xi_b, weights
  float Gs[3][TET_NQ][TET_NLOC];
  float wqs[TET_NQ];
  double TV[4][TET_NK][TET_NLOC];        // reference derivatives D^m phi_j at reference vertex l, 1 <= |m| <= p
  float Bf[4][TET_NFP][TET_NLOC];        // phi_j at the points of face f
  float wf[TET_NFP];                     // face weights (sum 1/2)
  int8_t perm[6][TET_NFP];               // the rule point a point becomes under a permutation of the face's vertices
  float Minv[TET_NLOC][TET_NLOC];        // inverse reference mass matrix
  int8_t kk[TET_NK][3];                  // the multi-indices
};

// DG hexahedra (cvw_hex.hip): vertex candidates (one thread per vertex), the
// sensor pass (one thread per cell) and the cell pass (one team of lanes per
// cell, a lane per node);
// the sensor pass (unless the sensor is fixed) writes gamma_e into gamma, or
// into gbuf [E] when gamma is null, and the cell pass reads it from there
cvw_status hex_candidates(const cvw_mesh* m, const cvw_params* prm, const float* u, float* cand, hipStream_t s);
cvw_status hex_eval(const cvw_mesh* m, const cvw_params* prm, int mode, const float* u, const float* u0, float* out,
                    float* gamma, float* alpha, const float* cand, float* gbuf, uint32_t* status, float dt, float a0,
                    float b0, hipStream_t s);

// DG tetrahedra (cvw_tet.hip): vertex candidates (one thread per vertex), the
// sensor pass and the cell pass (one thread per cell); gamma and gbuf as above
cvw_status tet_candidates(const cvw_mesh* m, const cvw_params* prm, const float* u, float* cand, hipStream_t s);
cvw_status tet_eval(const cvw_mesh* m, const cvw_params* prm, int mode, const float* u, const float* u0, float* out,
                    float* gamma, float* alpha, const float* cand, float* gbuf, uint32_t* status, float dt, float a0,
                    float b0, hipStream_t s);

}  // namespace cvw
