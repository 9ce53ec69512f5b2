// Internal declarations shared by the host side and the kernel launchers of libcvw.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "cvw.h"

namespace cvw {

// status bits of the workspace status word
enum : uint32_t { ST_NONFINITE = 1u, ST_NONPOSITIVE = 2u, ST_PCG_STALL = 4u, ST_LEARNED_FALLBACK = 8u,
                  ST_LEARNED_OFF = 16u };
// the first 256 bytes of a workspace: word 0 the status bits, word 1 the
// cells the learned sensor handed to the plain one since the last poll, word 2
// the audit latch (nonzero: the plain sensor takes every cell)
enum { WS_STATUS = 0, WS_FALLBACK_COUNT = 1, WS_LEARNED_OFF = 2 };
// modes of the fused sensor pass
enum : int { TILE_ALL = 0, TILE_FALLBACK = 1, TILE_AUDIT = 2 };

// operation modes of the evaluation kernels
enum Mode : int { MODE_SENSOR = 0, MODE_RESIDUAL = 1, MODE_STAGE = 2 };

// vertices per 256-thread block of the DG quadrilateral vertex pass
constexpr int VTX_PER_BLOCK = 256;
// cells per 256-thread tile of the DG quadrilateral cell pass: one 16-lane row
// per cell, four cells per row at degree 1
constexpr int cells_per_tile(int p) { return p == 1 ? 64 : 16; }

constexpr int MAXP = 3;   // highest degree of the GPU path

// Reference tables of a tensor-product element of degree p on [-1, 1]
// (nodes: Gauss-Legendre for DG, Gauss-Lobatto for CG).  Filled on the host.
struct TensorTables {
  float xi[MAXP + 1];                 // 1D nodes
  float w[MAXP + 1];                  // 1D Gauss weights of the volume rule (p+1 points)
  float D[MAXP + 1][MAXP + 1][MAXP + 1];  // D[m][a][i] = l_i^{(m)}(xi_a)
  float B[2][MAXP + 1];               // B[0][i] = l_i(-1), B[1][i] = l_i(+1)
  float L[MAXP + 1][MAXP + 1];        // L[m][i] = l_i^{(m)}(-1)
  // float64 copies for the smoothness-sensor derivatives (high derivatives of
  // smooth data cancel: table rounding must not multiply the full data)
  double Dd[MAXP + 1][MAXP + 1][MAXP + 1];
  double Ld[MAXP + 1][MAXP + 1];
  double Cd[MAXP + 1][MAXP + 1];      // Cd[m][i] = l_i^{(m)}(0) (cell centre)
  double wd[MAXP + 1];                // float64 copy of w
};

// Per-lane table record of the DG quadrilateral cell kernel: one 16-lane row
// per cell, node (a, b) on lane q = a + 4 b.  Row rotations by 4 s lanes bring
// the value of row (b - s) mod 4; the "rotated" entries are pre-permuted so.
struct alignas(16) LaneRec {
  float CX1[4];      // l_i'(xi_a)
  float CY1[4];      // l'_{(b-s)&3}(xi_b)
  float TX[4];       // l_a'(xi_c)
  float TY[4];       // l_b'(xi_{(b-s)&3})
  float BY0[4];      // l_{(b-s)&3}(-1)
  float BY1[4];      // l_{(b-s)&3}(+1)
  float misc[8];     // l_a(-1), l_a(+1), l_b(-1), l_b(+1), w_a, w_b, xi_a, xi_b
  double DX[3][4];   // l_i^{(m)}(xi_a), m = 1..3
  double DY[3][4];   // l^{(m)}_{(b-s)&3}(xi_b), m = 1..3
  // p = 3 interface step, one face quadrature point per lane: x-faces on the
  // columns a = 0 (W) and 3 (E) at point b; y-faces on the rows b = 0 (S) and
  // 3 (N) for the columns 1, 2; the S / N points of the corner columns 0 / 3
  // on the inner lanes (1, 1), (2, 1) / (1, 2), (2, 2).  Zero for p < 3.
  float OX[4];       // own x-side trace: l_i(-1) on a = 0, l_i(+1) otherwise
  float OY[4];       // own y-side trace, rotated: l_{(b-s)&3}(-1) in rows 0, 1, (+1) in rows 2, 3
  float FB[4];       // neighbour trace along its normal line (its side facing this cell)
  float fwx, fwy;    // face weight: w * h / 2 = fwx * hy + fwy * hx
  float nx, ny;      // outward unit normal of the lane's face point
  int slot;          // neighbour slot (S 0, E 1, N 2, W 3)
  int noff, nstep;   // neighbour node index of the normal line's first node, and its stride
  int srcS, srcN;    // lanes of the row that hold the S / N flux of column a
  float BX0[4], BX1[4];   // l_i(-1), l_i(+1) (x-side traces of p < 3; zero beyond p)
  int pad_[7];       // record stride 116 dwords: 8 consecutive lanes read distinct LDS banks
};

// Per-lane record of the degree-1 DG quadrilateral cell kernel, which packs
// four cells into a 16-lane row: node (a, b) = (l & 1, l >> 1) on lane l of
// the cell's quad.  Each lane takes one point of an x face (side a, point b)
// and one of a y face (side b, point a).  The four records are stored at the
// start of the mesh's lane-table array (which holds 16 LaneRec).
struct alignas(16) LaneRec1 {
  float CX1[2], CY1[2];    // l_i'(xi_a), l_j'(xi_b)
  float TX[2], TY[2];      // l_a'(xi_c), l_b'(xi_d)
  float OX[2], OY[2];      // own traces on the sides a and b: l_i(-1 or +1), l_j(-1 or +1)
  float FX[2], FY[2];      // the neighbours' traces across those faces (their facing sides)
  float lift[4];           // l_a(-1), l_a(+1), l_b(-1), l_b(+1)
  float wa, wb, xq, yq;    // Gauss weights and reference coordinates of the node
  float nx, ny;            // outward normals of the x face (side a) and the y face (side b)
  int slotx, sloty;        // their neighbour slots (S 0, E 1, N 2, W 3)
  double DX[2], DY[2];     // float64 l_i'(xi_a), l_j'(xi_b)
};
static_assert(4 * sizeof(LaneRec1) <= 16 * sizeof(LaneRec), "degree-1 lane records fit the lane-table array");

// Reference tables of a tensor-product CG element (Gauss-Lobatto nodes) of
// degree p <= 2 for the bilinear-map path: Gauss volume rule (p+1 points),
// Gauss semi-norm rule (p+2 points), derivatives up to order 2.
struct CGTables {
  float xn[MAXP + 1];                      // 1D nodes
  float xv[MAXP + 1], wv[MAXP + 1];        // volume rule
  float xs[MAXP + 2], ws[MAXP + 2];        // semi-norm rule
  float Dv[3][MAXP + 1][MAXP + 1];         // Dv[m][q][i] = l_i^{(m)}(xv_q)
  float Ds[3][MAXP + 2][MAXP + 1];         // Ds[m][q][i] = l_i^{(m)}(xs_q)
  float Dn[MAXP + 1][MAXP + 1];            // Dn[a][i] = l_i'(xn_a)
  float Lm[3][MAXP + 1];                   // l_i^{(m)}(-1)
  float Lp[3][MAXP + 1];                   // l_i^{(m)}(+1)
  double Dsd[3][MAXP + 2][MAXP + 1];       // float64 copies for the sensor path
  double Dvd[3][MAXP + 1][MAXP + 1];
  double Lmd[3][MAXP + 1];
  double Lpd[3][MAXP + 1];
};

// Reference tables of a 1D element (float64).
struct SegTables {
  double xn[MAXP + 1];                     // nodes (Gauss-Lobatto for CG, Gauss for DG)
  double xq[MAXP + 1], wq[MAXP + 1];       // (p+1)-point Gauss rule
  double D[MAXP + 1][MAXP + 1][MAXP + 1];  // D[m][q][i] = l_i^{(m)}(xq_q)
  double Dn[MAXP + 1][MAXP + 1];           // Dn[a][i] = l_i'(xn_a)
  double Lv[2][MAXP + 1][MAXP + 1];        // Lv[s][m][i] = l_i^{(m)}(-1) (s = 0), (+1) (s = 1)
};

// Reference tables of the P_p Lagrange triangle (equispaced nodes on the
// reference triangle (0,0), (1,0), (0,1)) with the (p+1)^2-point Stroud
// conical-product rule and (p+1)-point Gauss rules on the edges.  Filled on
// the host; the cell kernel reads them with uniform indices.
constexpr int TRI_NLOC = (MAXP + 1) * (MAXP + 2) / 2;
constexpr int TRI_NQ = (MAXP + 1) * (MAXP + 1);
constexpr int TRI_NK = (MAXP + 1) * (MAXP + 2) / 2 - 1;
struct TriTables {
  float B[TRI_NQ][TRI_NLOC];               // phi_j(xi_q)
  float Gx[TRI_NQ][TRI_NLOC];              // d phi_j / d xi at xi_q
  float Gy[TRI_NQ][TRI_NLOC];              // d phi_j / d eta at xi_q
  float xq[TRI_NQ], yq[TRI_NQ], wq[TRI_NQ];  // Stroud points and weights (reference area 1/2)
  float Bf[3][MAXP + 1][TRI_NLOC];         // phi_j at the Gauss points of edge f (vertex f -> f+1)
  float xf[3][MAXP + 1], yf[3][MAXP + 1];  // reference coordinates of those points
  float wf[MAXP + 1];                      // Gauss weights on [-1, 1]
  float Minv[TRI_NLOC][TRI_NLOC];          // inverse reference mass matrix
  float mvec[TRI_NLOC];                    // int phi_j over the reference triangle
  double xqd[TRI_NQ], yqd[TRI_NQ], wqd[TRI_NQ];
  double TV[3][TRI_NK][TRI_NLOC];          // reference derivatives D^m phi_j at reference vertex l (|m| >= 1)
  // float64 copies for the positivity limiter: phi_j at the volume and edge
  // points, and the cell average as weights of the nodal values
  double Bd[TRI_NQ][TRI_NLOC];
  double Bfd[3][MAXP + 1][TRI_NLOC];
  double mwd[TRI_NLOC];
};

// tables of the 3D cells (cvw_cells3d.h)
struct HexTables;
struct TetTables;

// Scalars of the method in the precision of the kernels.
struct MethodScalars {
  float eps_v, eps_c, r, q_sensor, q_beta, lin_w, c_gamma, lam_g;
  float fp[4];                        // flux parameters
  int sc_on, fast_exp, sensor_kind;   // fast_exp: r == 2 and q == 1
  float fixed_gamma;
  // float64 copies for the float64 sensor paths
  double eps_vd, eps_cd, lin_wd, c_gammad, lam_gd, fixed_gammad, fpd[4];
  // 2D DG boundary faces: kind and exterior state of boundary face b, which
  // the neighbour tables hold as -(b + 1)
  const int32_t* bck;
  const float* bcs;
};

// Learned sensor network 48 -> 64 -> 64 -> 1.  Packed float32 parameters:
// W1 [48][64] (input, hidden), b1 [64], W2 [64][64] (hidden 1, hidden 2),
// b2 [64], w3 [64], b3.
constexpr int MLP_IN = 48, MLP_HID = 64;
constexpr int MLP_OFF_W1 = 0, MLP_OFF_B1 = MLP_IN * MLP_HID, MLP_OFF_W2 = MLP_OFF_B1 + MLP_HID;
constexpr int MLP_OFF_B2 = MLP_OFF_W2 + MLP_HID * MLP_HID, MLP_OFF_W3 = MLP_OFF_B2 + MLP_HID;
constexpr int MLP_OFF_B3 = MLP_OFF_W3 + MLP_HID, MLP_NPARAM = MLP_OFF_B3 + 1;
// device compute copies: bfloat16 W1^T [64][48], W2^T [64][64], W2 [64][64],
// w3 [64]; float32 biases
struct MlpDev {
  const uint16_t* W1t;
  const uint16_t* W2t;
  const uint16_t* W2r;
  const uint16_t* w3;
  const float* b1;
  const float* b2;
  const float* b3;
};
// Guard of the learned sensor's inference (lo null: no guard): the
// network's validity box of the 48 features, the workspace status words (the
// hand-over count and the audit latch among them), per-tile flags of the
// structured grid (nx cells per row, tiles_x 16 x 16 tiles per tile row)
struct MlpGuard {
  const float* lo;
  const float* hi;
  uint32_t* status;        // workspace words: status bits, hand-over count, audit latch
  uint8_t* tile_flag;
  int64_t nx;
  int64_t tiles_x;
};
struct MlpDevMut {
  uint16_t* W1t;
  uint16_t* W2t;
  uint16_t* W2r;
  uint16_t* w3;
  float* b1;
  float* b2;
  float* b3;
};

// Uniform geometry factors of a DG quadrilateral mesh for the cell pass,
// formed once on the host (the device has no scalar floating-point unit, so
// every uniform product computed in a kernel costs a vector instruction).
struct CellGeo {
  float hx, hy, he;        // cell sizes, h_e
  float sx, sy;            // 2 / hx, 2 / hy
  float he2;               // h_e^2
  float mx2, my2;          // hx^2 / 12, hy^2 / 12 (cell mean of X^2, Y^2 about the centre)
  float qx4, qy4;          // hx^4 / 720, hy^4 / 720
  float area4;             // hx hy / 4 (quadrature weight factor)
  float hhx, hhy;          // hx / 2, hy / 2
  float nuf;               // h_e / (2 p): nu_e = lambda_e nuf
};
// Float64 1D Gauss nodes and weights of the DG quadrilateral element (the
// limiter evaluates its reconstruction there)
struct LimitNodes {
  double xi[MAXP + 1];
  double w[MAXP + 1];
};

// Float64 tables of the DG quadrilateral vertex pass for one mesh: L[m][i] =
// l_i^{(m)}(-1), and per multi-index k (in the order of the derivative set)
// sk[t] = h_e^{|k|} (2 / h_x)^{kx} (2 / h_y)^{ky}, which turns reference
// derivatives at the corner into h_e^{|k|} D^k u_h, and hinv[n] = h_e^{-n}.
struct VertexTables {
  double L[MAXP + 1][MAXP + 1];
  double sk[(MAXP + 1) * (MAXP + 2) / 2 - 1];
  double hinv[MAXP + 1];
};
inline VertexTables make_vertex_tables(const TensorTables& t, double hx, double hy, double he, int p) {
  VertexTables v{};
  for (int m = 0; m <= MAXP; ++m)
    for (int i = 0; i <= MAXP; ++i) v.L[m][i] = t.Ld[m][i];
  auto pw = [](double x, int n) { double r = 1.0; for (int i = 0; i < n; ++i) r *= x; return r; };
  int k = 0;
  for (int n = 1; n <= p && n <= MAXP; ++n)       // the derivative set's order: |k| = n, kx = n - j, ky = j
    for (int j = 0; j <= n; ++j) v.sk[k++] = pw(he, n) * pw(2.0 / hx, n - j) * pw(2.0 / hy, j);
  for (int n = 0; n <= MAXP; ++n) v.hinv[n] = 1.0 / pw(he, n);
  return v;
}

inline CellGeo make_cell_geo(double hx, double hy, double he, int p) {
  CellGeo g;
  g.hx = static_cast<float>(hx);
  g.hy = static_cast<float>(hy);
  g.he = static_cast<float>(he);
  g.sx = static_cast<float>(2.0 / hx);
  g.sy = static_cast<float>(2.0 / hy);
  g.he2 = static_cast<float>(he * he);
  g.mx2 = static_cast<float>(hx * hx / 12.0);
  g.my2 = static_cast<float>(hy * hy / 12.0);
  g.qx4 = static_cast<float>(hx * hx * hx * hx / 720.0);
  g.qy4 = static_cast<float>(hy * hy * hy * hy / 720.0);
  g.area4 = static_cast<float>(0.25 * hx * hy);
  g.hhx = static_cast<float>(0.5 * hx);
  g.hhy = static_cast<float>(0.5 * hy);
  g.nuf = static_cast<float>(he / (2.0 * p));
  return g;
}

// Arguments of the fused DG quadrilateral sensor pass (structured periodic
// grid, cells numbered e = i + nx j; 16 x 16 cells per block)
struct SensorTileArgs {
  double T[MAXP + 1][MAXP + 1];   // T[m][i] = (2m + 1) / 2 w_i P_m(xi_i): Legendre coefficients from Gauss-node values
  float sk[(MAXP + 1) * (MAXP + 2) / 2 - 1];   // h_e^{|k|} (2/hx)^kx (2/hy)^ky: reference -> scaled physical derivatives
  float Sk[(MAXP + 1) * (MAXP + 2) / 2 - 1];   // (hx hy / 4) h_e^{2|k|-2} (2/hx)^{2kx} (2/hy)^{2ky}: eq. snorm weights
  int nx, ny, tiles_x, tiles_y;
  int64_t ntiles;
};

// Per-instance descriptor of a batch of independent DG quadrilateral meshes
// (device memory, written by the host before a batch step).  The Runge-Kutta
// stage s reads state in[s] and writes out[s]: u -> st1 -> st2 -> u.
struct alignas(16) BatchInst {
  const float* u_in[3];
  float* u_out[3];
  float* u;                         // u_n (the caller's state)
  float* cand;
  const int32_t* cell_vtx;
  const int32_t* nbr;
  const int32_t* vptr;
  const int32_t* vent;
  int64_t E, Nv;
  VertexTables vt;                  // vertex pass tables of the mesh
  CellGeo g;
  float dt;
  int P, flux;
  uint32_t* status;
  MethodScalars ms;
  float* gam;                       // fused sensor pass: gamma of the stage [E] (null: vertex candidates)
  SensorTileArgs sa;                // its tile arguments
};


// One-dimensional elements of any degree 1 <= p <= HP_MAXP (float64): the
// reference operators of the Lagrange basis at the mesh's nodes, built on the
// host, in one array of doubles with these offsets:
//   xq[n1], wq[n1]                  (p+1)-point Gauss rule on [-1, 1]
//   DQ[m][j][q] = l_j^{(m)}(xq_q)   m = 0..p (lanes over q read consecutively)
//   DV[v][j][m] = l_j^{(m)}(-1 / +1) v = 0 / 1
//   DN[a][j]    = l_j'(x_a)         at the nodes
constexpr int HP_MAXP = 32;
struct HPOff {
  int xq, wq, DQ, DV, DN, size;
};
__host__ __device__ inline HPOff hp_off(int p) {
  const int n1 = p + 1;
  HPOff o;
  o.xq = 0;
  o.wq = n1;
  o.DQ = 2 * n1;
  o.DV = o.DQ + n1 * n1 * n1;
  o.DN = o.DV + 2 * n1 * n1;
  o.size = o.DN + n1 * n1;
  return o;
}

// Arguments of the 1D kernels of any degree: the mesh, the method and the
// boundary data of the two ends of a line (index 0: the end at the left
// vertex of its cell, 1: the right one).
struct SegHPArgs {
  const double* tab;                // hp_off(p) layout
  const int32_t* cell_dof;          // CG [E][p+1]
  const int32_t* cell_vtx;          // [E][2]
  const int32_t* nbr;               // DG [E][2] face neighbours
  const double* hcell;              // [E] cell lengths
  const int32_t* vptr;              // vertex patches (CSR, entries cell * 4 + local vertex)
  const int32_t* vent;
  const int32_t* dptr;              // CG: DOF patches (CSR, entries cell * (p+1) + local node)
  const int32_t* dent;
  int64_t E, Nv, ndof;
  int p, nv, flux, cg;
  int bc[2];
  double bcs[2][4];
  MethodScalars ms;
};

}  // namespace cvw

struct cvw_mesh {
  int dim = 0, cell = 0, degree = 0, space = 0;
  int64_t E = 0, Nv = 0, ndof = 0, nnz = 0;
  int nloc = 0, nk = 0, nq = 0, ve = 0, nf = 0;
  int uniform = 0;
  int closed = 0;                    // DG: every face has a neighbour
  int open_ends = 0;                 // segments: vertices used by one cell only (the ends of a line)
  int64_t n_bfaces = 0;              // DG: faces without a neighbour; device tables hold -(b + 1)
  int64_t grid_nx = 0, grid_ny = 0;  // DG quadrilaterals: structured periodic grid e = i + nx j (0: not)
  double hx = 0, hy = 0, he = 0;
  int device = 0;
  int eval_grid = 0;                 // DG quad cell pass: blocks per launch (0 = default)
  int external = 0;                  // device arrays in a caller-provided buffer (not freed here)
  // host copies
  std::vector<int32_t> h_vtx_ptr, h_vtx_cell, h_vtx_lv, h_cell_vtx, h_nbr, h_nbr_face, h_cell_dof;
  std::vector<int32_t> h_bface;      // DG: [n_bfaces][2] (cell, local face), ascending
  std::vector<double> h_coords;      // [E][ve][dim]
  std::vector<double> h_he;          // [E]
  cvw::TensorTables tens{};
  // device arrays (owned)
  int32_t* d_vtx_ptr = nullptr;      // [Nv + 1]
  int32_t* d_vtx_ent = nullptr;      // [nnz] packed cell * 4 + lv (hexahedra: cell * 8 + lv)
  int32_t* d_cell_vtx = nullptr;     // [E][ve]
  int32_t* d_nbr = nullptr;          // [E][nf]
  cvw::TensorTables* d_tens = nullptr;
  cvw::LaneRec* d_lanes = nullptr;   // [16] DG quadrilateral lane tables
  // CG
  int32_t* d_cell_dof = nullptr;     // [E][nloc]
  int32_t* d_dof_ptr = nullptr;      // [ndof + 1] CSR of the DOF patches
  int32_t* d_dof_ent = nullptr;      // [E * nloc] cell * nloc + local node, ascending (cell, node)
  float* d_geo = nullptr;            // [E][8] vertex 0 and the other vertices relative to it
  float* d_he = nullptr;             // [E] diam K_e
  cvw::CGTables cgt{};
  cvw::CGTables* d_cgt = nullptr;
  // 1D
  double* d_hcell = nullptr;          // [E] cell length
  cvw::SegTables* d_segt = nullptr;
  double* d_hp = nullptr;             // reference operators of any degree (hp_off layout)
  // time stepping: inverse of the lumped CG mass (PCG preconditioner) or of
  // the exact diagonal 1D DG mass, in both precisions
  // triangles
  cvw::TriTables* d_trit = nullptr;
  double* d_geot = nullptr;           // [E][8] x0, y0, x1-x0, y1-y0, x2-x0, y2-y0, diam, 0
  float* d_geov = nullptr;            // [E][8] vertex pass: inverse Jacobian A00, A01, A10, A11, diam, 0, 0, 0
  int32_t* d_nbrf = nullptr;          // [E][3] neighbour cell * 4 + its face
  // hexahedra
  double hz = 0;
  cvw::HexTables* d_hext = nullptr;
  // tetrahedra
  cvw::TetTables* d_tett = nullptr;
  double* d_geoth = nullptr;          // [E][16] vertex 0, J (row-major, J[a][b] = dx_a / dxi_b), diam, padding
  int32_t* d_nbrt = nullptr;          // [E][4] neighbour cell * 32 + its face * 8 + face permutation
  float* d_dinv_f = nullptr;          // [n_mass]
  double* d_dinv_d = nullptr;         // [n_mass]
  int64_t n_mass = 0;
};

namespace cvw {

void set_error(const std::string& msg);
MethodScalars make_scalars(const cvw_params* prm);
int n_var(const cvw_mesh* m, int flux);   // conserved variables: 1, or dim + 2 for the Euler equations

// kernel launchers (cvw_dgquad.hip)
cvw_status dgquad_candidates(const cvw_mesh* m, const cvw_params* prm, const float* u, float* cand,
                             hipStream_t s, const uint32_t* vcount = nullptr, const int32_t* vlist = nullptr);
cvw_status dgquad_eval(const cvw_mesh* m, const cvw_params* prm, int mode, const float* u, const float* u0,
                       float* out, float* gamma, float* alpha, const float* cand, uint32_t* status,
                       float dt, float a0, float b0, hipStream_t s, const float* gamma_in = nullptr);
// HWENO limiter on DG quadrilaterals (cvw_dgquad.hip): cand holds the vertex
// candidates of every variable, [n_var][Nv][n_k], variable 0 already
// computed; gamma the sensor values; count (two words), list (E entries),
// vflag (Nv bytes) and vlist (Nv entries) are scratch for the selected cells
// and their vertices
cvw_status dgquad_limit(const cvw_mesh* m, const cvw_params* prm, const float* u, float* out, float* cand,
                        const float* gamma, const LimitNodes& ln, double threshold, uint32_t* count,
                        int32_t* list, uint8_t* vflag, int32_t* vlist, hipStream_t s);
// fused sensor pass of a structured periodic DG quadrilateral grid: gamma_e
// of every cell from the sensor field (variable 0 of u) (cvw_dgsensor.hip)
cvw_status dgquad_sensor_tile(const cvw_mesh* m, const cvw_params* prm, const float* u, float* gamma, hipStream_t s,
                              int mode = TILE_ALL, uint8_t* tile_flag = nullptr, const float* g_ref = nullptr,
                              double* part = nullptr);
int64_t sensor_tiles(const cvw_mesh* m);   // 16 x 16 tiles of the fused pass (0: no structured grid)
// audit of the learned sensor: the block partials of the TILE_AUDIT pass in a
// fixed order; out (device, 2 doubles) = mean and largest deviation
cvw_status dgquad_audit_finalize(const cvw_mesh* m, const double* part, double tol, uint32_t* status, double* out,
                                 hipStream_t s);
// learned-sensor features of every cell, bfloat16 [E][48] (cvw_dgquad.hip)
cvw_status dgquad_features(const cvw_mesh* m, const float* u, const float* cand, double sigma_ref, uint16_t* feat,
                           hipStream_t s);
// kernel launchers (cvw_cgquad.hip)
cvw_status cgquad_candidates(const cvw_mesh* m, const cvw_params* prm, const float* u, float* cand, hipStream_t s);
cvw_status cgquad_eval(const cvw_mesh* m, const cvw_params* prm, int mode, const float* u, const float* cand,
                       float* pg, float* rcell, float* R, float* gamma, float* alpha, uint32_t* status,
                       hipStream_t s);
// kernel launchers (cvw_seg.hip)
cvw_status seg_candidates(const cvw_mesh* m, const cvw_params* prm, const void* u, void* cand, hipStream_t s);
cvw_status seg_eval(const cvw_mesh* m, const cvw_params* prm, int mode, const void* u, const void* cand, void* pg,
                    void* rcell, void* R, void* gamma, void* alpha, uint32_t* status, hipStream_t s);
// 1D elements of any degree in float64, systems and lines with ends
// (cvw_seghp.hip): the candidates of the sensor variable [Nv][p] and the
// evaluation (modes as seg_eval; pg [nv][ndof] and rcell [nv][E][p+1] are CG
// scratch)
bool seg_hp(const cvw_mesh* m, const cvw_params* prm);
SegHPArgs seghp_args(const cvw_mesh* m, const cvw_params* prm);
cvw_status seghp_candidates(const cvw_mesh* m, const cvw_params* prm, const double* u, double* cand, hipStream_t s);
cvw_status seghp_eval(const cvw_mesh* m, const cvw_params* prm, int mode, const double* u, const double* cand,
                      double* pg, double* rcell, double* R, double* gamma, double* alpha, uint32_t* status,
                      hipStream_t s);
// batched fused sensor pass over (instance, tile) items of degree P
// (cvw_dgsensor.hip), and the tile arguments of a mesh
cvw_status batch_sensor_pass(int P, const BatchInst* inst, const int2* items, int n_items, int stage, int grid,
                             hipStream_t s);
SensorTileArgs make_sensor_tile_args(const cvw_mesh* m);
// batched DG quadrilateral stage over many meshes (cvw_dgquad.hip): the
// vertex pass is launched once per degree P, the cell pass once per (P, flux);
// items are (instance, logical block) pairs of the instances of that class,
// processed by a grid-stride loop
cvw_status batch_vertex_pass(int P, const BatchInst* inst, const int2* items, int n_items, const TensorTables* tabs,
                             int stage, int grid, hipStream_t s);
cvw_status batch_eval_pass(int P, int flux, const BatchInst* inst, const int2* items, int n_items,
                           const TensorTables* tabs, const LaneRec* lanes, int stage, int grid, hipStream_t s);
// learned-sensor network (cvw_mlp.hip)
cvw_status mlp_infer(const MlpDev& W, const uint16_t* feat, int64_t n, float* gamma, hipStream_t s,
                     const MlpGuard* guard = nullptr);
cvw_status mlp_train(const MlpDev& W, const uint16_t* feat, const float* target, const int32_t* idx, int batch,
                     float* part, hipStream_t s);
cvw_status mlp_update(const float* part, int nblk, float* master, float* m1, float* m2, float lr, double beta1,
                      double beta2, float eps, double bc1, double bc2, float* grad_out, const MlpDevMut& W,
                      hipStream_t s);
// kernel launchers (cvw_tri.hip)
cvw_status tri_candidates(const cvw_mesh* m, const cvw_params* prm, const float* u, float* cand, hipStream_t s);
cvw_status tri_eval(const cvw_mesh* m, const cvw_params* prm, int mode, const float* u, const float* u0, float* out,
                    float* gamma, float* alpha, const float* cand, uint32_t* status, float dt, float a0, float b0,
                    hipStream_t s);
cvw_status tri_totals(const cvw_mesh* m, int nvar, const float* u, double* partial, double* out_dev, hipStream_t s);

// time stepping (cvw_cgstep.hip)
size_t pcg_partials(int64_t n);
// M x = b for every variable: lines solve all nvar variables at once (vectors
// [nvar][ndof], ycell [nvar][E][n_loc]); quadrilaterals one variable (nvar 1)
template <typename Real>
cvw_status cg_mass_solve(const cvw_mesh* m, const Real* b, Real* x, Real* r, Real* z, Real* p, Real* Ap,
                         Real* ycell, double* part, double* S, const Real* dinv, double tol, int maxit,
                         uint32_t* status, hipStream_t s, int nvar = 1);
// dinv (a diagonal mass of nm entries, shared by the variables) or null
template <typename Real>
cvw_status stage_update(const Real* us, const Real* un, const Real* x, const Real* dinv, Real* uo, double a0,
                        double b0, double dt, int64_t n, hipStream_t s, int64_t nm = 0);
cvw_status totals_f32(const cvw_mesh* m, int nvar, const float* u, double* partial, double* out_dev,
                      hipStream_t s);

}  // namespace cvw
