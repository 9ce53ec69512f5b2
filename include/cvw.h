/*
 * cvw.h -- C ABI of the cell-vertex WENO stabilised residual library (libcvw.so).
 *
 * The library evaluates, on one AMD Instinct MI355X (gfx950), the per-stage
 * residual of the dissipation-based WENO stabilisation of continuous (CG) and
 * discontinuous (DG) Galerkin discretisations of hyperbolic conservation laws
 * with cell-vertex HWENO smoothness sensors and shock-capturing quadrature
 * (Vedral & Kuzmin, "Cell-vertex WENO schemes with shock-capturing quadrature
 * for high-order finite element discretizations of hyperbolic problems").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns a cvw_status; no exception crosses the ABI.  After a
 *   non-zero status cvw_last_error() describes the failure (thread-local text,
 *   valid until the next call on the same thread).
 * - Host pointers are read during the call only.  Device pointers (state,
 *   residual, sensor, workspace) are owned by the caller; they must be
 *   allocations on the current HIP device, 256-byte aligned and not aliased
 *   unless stated.  The library never allocates in the evaluation calls; only
 *   the handle constructors allocate: cvw_mesh_build (the mesh's device
 *   arrays, freed by cvw_mesh_destroy), cvw_mlp_create (the network's
 *   parameters and Adam state) and cvw_batch_build (descriptors, work lists,
 *   tables).  Each has a variant that places them in a caller-owned device
 *   buffer instead (cvw_mesh_build_in, cvw_mlp_create_in, cvw_batch_build_in,
 *   sized by cvw_mesh_plan, cvw_mlp_device_bytes, cvw_batch_plan).
 * - `stream` is a hipStream_t (NULL = default stream).  Evaluation calls only
 *   enqueue work on it and return; argument errors are detected on the host
 *   before anything is enqueued.  Numerical trouble detected on the device
 *   (non-finite residual, non-positive density or pressure) sets bits in the
 *   workspace status word, read with cvw_poll_status.
 * - State layout is component-major (structure of arrays):
 *     DG: U[v][e][j], j = local node (quads: a + (p+1) b, x fastest),
 *     CG: U[v][I],    I = global DOF in the canonical numbering: vertex DOFs by
 *         vertex id, then edge DOFs (edges sorted by (min, max) vertex id,
 *         oriented min -> max), then cell-interior DOFs by cell id.
 *   Single (CVW_F32) or double (CVW_F64) precision as cvw_params.dtype says.
 * - Results are deterministic: no floating-point atomics are used; every
 *   reduction runs in a fixed order.
 * - Environment: CVW_WIDE_ADDRESSING=1 makes the DG quadrilateral cell pass
 *   use 64-bit addresses for every mesh (by default it uses 32-bit buffer
 *   offsets while the state and the vertex candidates each fit in 4 GiB);
 *   both give bitwise the same results.  Read at every launch.
 */
#ifndef CVW_H
#define CVW_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CVW_ABI_VERSION 12

typedef enum {
  CVW_OK = 0,
  CVW_EINVAL = 1,          /* malformed argument (null pointer, bad size, bad mesh) */
  CVW_ENOMEM = 2,          /* device allocation failed (cvw_mesh_build only)        */
  CVW_EDEVICE = 3,         /* a HIP runtime call failed                              */
  CVW_EUNSUPPORTED = 4,    /* valid request outside what the GPU path implements    */
  CVW_ENUMERIC = 5         /* cvw_poll_status: device flagged a numerical problem   */
} cvw_status;

/* Hexahedra (CVW_HEX, dim 3): DG Q_p, p <= 2, on congruent axis-aligned
 * boxes of a periodic mesh with one cell in each of the eight octants of
 * every vertex (any conforming closed box mesh; the GPU path refuses others
 * with CVW_EUNSUPPORTED), constant advection, Burgers and the Euler
 * equations (five variables rho, m_x, m_y, m_z, E; HLL at the faces; the
 * density is the sensor field), float32.  The vertex-based candidates of a cube: eight per cell (Sec. 3.2,
 * the remark on stencil sizes).  Local vertices: the face z = z0
 * counter-clockwise from the lowest corner, then the face z = z0 + hz in the
 * same order; local node a + (p+1) b + (p+1)^2 c at the tensor Gauss points
 * (x fastest); local faces 2 axis + side (0 -x, 1 +x, 2 -y, 3 +y, 4 -z, 5 +z);
 * cell_coords [E][8][3]; flux_param[0..2] is the velocity (or the Burgers
 * direction) (vx, vy, vz). */
/* Tetrahedra (CVW_TET, dim 3): DG P_p, p <= 2, on periodic meshes of
 * positively oriented tetrahedra (every face shared by two cells), constant
 * advection, Burgers and the Euler equations (as on hexahedra), float32;
 * four vertex candidates per cell.  Local nodes: the
 * equispaced lattice (i, j, k) / p, i + j + k <= p, of the reference cell
 * (0,0,0), (1,0,0), (0,1,0), (0,0,1), i fastest; face f opposite vertex f;
 * cell_coords [E][4][3]. */
typedef enum { CVW_SEG = 1, CVW_TRI = 2, CVW_QUAD = 3, CVW_HEX = 4, CVW_TET = 5 } cvw_cell;
typedef enum { CVW_CG = 0, CVW_DG = 1 } cvw_space;
typedef enum {
  CVW_ADVECT_CONST = 0,    /* f = v u, v = (flux_param[0], flux_param[1])                    */
  CVW_ADVECT_ROT = 1,      /* f = v(x) u, v = w (cy - y, x - cx), (cx, cy, w) = flux_param[0..2] */
  CVW_BURGERS = 2,         /* f = u^2 / 2 (flux_param[0], flux_param[1])                     */
  CVW_KPP = 3,             /* f = (sin u, cos u)                                             */
  CVW_EULER = 4            /* Euler equations, gas gamma = flux_param[0]; dim + 2 conserved
                              variables: (rho, m, E) on lines, (rho, m_x, m_y, E) in 2D        */
} cvw_flux;
/* Boundary data at the two ends of a line (1D meshes whose first and last
 * vertex belong to one cell each; Sec. 5.4 of the paper: an inflow end and
 * reflecting walls).  The boundary term phi_j(x_b) f*(u_h(x_b), u_ext; n) is
 * added to the residual of both CG and DG, with the interface flux of the
 * interior faces (HLL for the Euler equations, Lax-Friedrichs otherwise):
 *   OUTFLOW: u_ext = u_h(x_b) (the physical flux of the trace),
 *   WALL:    u_ext = (rho, -m, E) (Euler only),
 *   INFLOW:  u_ext = bc_state[end] (conserved variables).
 * The vertex patch of an end vertex is the one cell that contains it. */
typedef enum { CVW_BC_NONE = 0, CVW_BC_OUTFLOW = 1, CVW_BC_WALL = 2, CVW_BC_INFLOW = 3 } cvw_bc;
/* On 2D DG meshes with boundary faces (quadrilaterals, triangles) the same
 * kinds are given per boundary face (cvw_params.bc_face_kind / bc_face_state,
 * device arrays owned by the caller, who may rewrite them between calls for
 * time-dependent data), and the wall mirrors the normal momentum:
 * m_ext = m - 2 (m . n) n. */
typedef enum { CVW_F32 = 0, CVW_F64 = 1 } cvw_dtype;
typedef enum { CVW_SENSOR_PLAIN = 0, CVW_SENSOR_LEARNED = 1, CVW_SENSOR_FIXED = 2 } cvw_sensor_kind;

/* Mesh description (host memory, read during cvw_mesh_build only).
 * A conforming mesh of segments, triangles or quadrilaterals (Sec. 2.1 of the
 * paper).  cell_vertices holds topological vertex ids after periodic
 * identification, counter-clockwise in 2D; cell_coords holds the *unwrapped*
 * physical coordinates of each cell's vertices, so a cell on a periodic seam
 * keeps its own geometric position.  Quadrilateral vertices are ordered like
 * the reference vertices (-1,-1), (1,-1), (1,1), (-1,1). */
typedef struct {
  int32_t dim;               /* 1 or 2                                         */
  int32_t cell;              /* cvw_cell                                       */
  int32_t degree;            /* polynomial degree p >= 1                       */
  int32_t space;             /* cvw_space                                      */
  int64_t n_cells;
  int64_t n_vertices;
  const int32_t* cell_vertices;  /* [n_cells][v_e]                              */
  const double* cell_coords;     /* [n_cells][v_e][dim]                         */
  int32_t periodic[2];       /* informative: periodic directions               */
} cvw_mesh_desc;

/* Method parameters.  Defaults (the paper's values): eps = 1e-6 and r = 2 for
 * both WENO stages (Sec. 3.2), q = 1 (Sec. 5), vertex-candidate linear weight
 * 1e-3 (Sec. 3.2), shock-capturing quadrature on with cutoff C_gamma = 0.9
 * (Sec. 5). */
typedef struct {
  int32_t dtype;             /* cvw_dtype of state / residual buffers            */
  int32_t flux;              /* cvw_flux                                         */
  double flux_param[4];
  double eps_vertex;         /* epsilon of the vertex-stage Jiang-Shu weights    */
  double eps_cell;           /* epsilon of the cell-stage weights                */
  int32_t r;                 /* Jiang-Shu exponent                               */
  int32_t sc_on;             /* shock-capturing quadrature on/off                */
  double q_sensor;           /* exponent q of the sensor gamma_e                 */
  double q_beta;             /* exponent q of the smoothness indicators beta     */
  double lin_w_vertex;       /* linear weight of each vertex candidate           */
  double c_gamma;            /* SC active only where gamma_e < c_gamma           */
  double lambda_global;      /* > 0: global wave-speed bound used for nu_e and LLF */
  int32_t sensor;            /* cvw_sensor_kind                                  */
  int32_t audit_every;       /* CVW_SENSOR_LEARNED, cvw_step: audit the network against the
                                plain sensor at the start of every audit_every-th step (0: never) */
  double fixed_gamma;        /* gamma_e for CVW_SENSOR_FIXED                     */
  double sigma_ref;          /* CVW_SENSOR_LEARNED: reference scale of the features (> 0) */
  const struct cvw_mlp* mlp; /* CVW_SENSOR_LEARNED: the network (cvw_mlp_create)  */
  double audit_tol;          /* CVW_SENSOR_LEARNED: an audit whose mean |gamma_learned - gamma_plain|
                                exceeds it switches the run to the plain sensor (cvw_learned_audit) */
  int32_t bc[2];             /* lines with ends: cvw_bc at the left end (vertex 0 of its cell) and
                                the right end; both must be set on such a line, ignored on closed meshes */
  double bc_state[2][4];     /* CVW_BC_INFLOW: exterior conserved state at that end (first n_var used) */
  const int32_t* bc_face_kind; /* 2D DG meshes with boundary faces: device [n_bfaces] cvw_bc of each
                                boundary face, in the order of CVW_EXPORT_BFACE (required there,
                                ignored on closed meshes); a wall on a scalar law acts as outflow */
  const float* bc_face_state;  /* device [n_bfaces][4] exterior conserved state of the inflow faces
                                (float32, like the 2D DG state); may be NULL without inflow faces */
} cvw_params;

typedef struct {
  int64_t n_cells, n_vertices, n_dof, nnz_vertex;
  int32_t n_loc;             /* nodes per cell                                   */
  int32_t n_k;               /* derivative multi-indices 1 <= |k| <= p           */
  int32_t n_q;               /* volume quadrature points per cell                */
  int32_t v_e;               /* vertices per cell                                */
  int32_t n_faces;
  int32_t uniform;           /* 1: congruent axis-aligned cells (structured fast path) */
  double hx, hy;             /* cell sizes when uniform                          */
  int64_t grid_nx, grid_ny;  /* DG quadrilaterals on a structured periodic grid (cells
                                numbered e = i + grid_nx j, four cells at every vertex):
                                the grid's size, which enables the fused sensor pass;
                                0 otherwise                                         */
  int64_t n_bfaces;          /* DG: faces without a neighbour (the boundary faces)  */
} cvw_mesh_info;

typedef struct cvw_mesh cvw_mesh;

/* Export selectors for cvw_mesh_export (all int32 arrays). */
enum {
  CVW_EXPORT_VTX_PTR = 0,    /* [n_vertices + 1] CSR row pointer of the vertex patches */
  CVW_EXPORT_VTX_CELL = 1,   /* [nnz] cell of each patch entry (ascending (cell, lv)) */
  CVW_EXPORT_VTX_LV = 2,     /* [nnz] local vertex of each patch entry              */
  CVW_EXPORT_NBR = 3,        /* DG: [n_cells][n_faces] face neighbour, -1 = boundary */
  CVW_EXPORT_NBR_FACE = 4,   /* DG: [n_cells][n_faces] neighbour's local face        */
  CVW_EXPORT_CELL_DOF = 5,   /* CG: [n_cells][n_loc] global DOF of each local node   */
  CVW_EXPORT_BFACE = 6       /* DG: [n_bfaces][2] (cell, local face) of each boundary face,
                                ascending: the order of the per-face boundary data */
};

int cvw_abi_version(void);
const char* cvw_last_error(void);

/* Build the connectivity the method needs (Sec. 3.2: vertex patches C(x_i);
 * face neighbours for DG interface terms; CG numbering), per-cell geometry
 * (h_e = diam K_e, Sec. 2.1) and the reference tables, and upload them to the
 * current device.  EINVAL for a malformed or non-conforming description,
 * ENOMEM / EDEVICE for device failures.  *out owns device memory. */
cvw_status cvw_mesh_build(const cvw_mesh_desc* desc, cvw_mesh** out);
/* The same mesh with its device arrays placed in a caller-owned device buffer
 * (e.g. a torch allocation): cvw_mesh_plan gives the bytes the buffer needs
 * (host work only, no device memory touched), cvw_mesh_build_in builds into
 * device_buf (256-byte aligned, at least that many bytes; EINVAL if smaller).
 * The buffer must outlive the mesh; cvw_mesh_destroy then frees only the
 * host-side part. */
cvw_status cvw_mesh_plan(const cvw_mesh_desc* desc, size_t* device_bytes);
cvw_status cvw_mesh_build_in(const cvw_mesh_desc* desc, void* device_buf, size_t bytes, cvw_mesh** out);
void cvw_mesh_destroy(cvw_mesh* mesh);
cvw_status cvw_mesh_get_info(const cvw_mesh* mesh, cvw_mesh_info* info);
/* Launch shape of the DG quadrilateral cell pass on this mesh: the number of
 * 256-thread blocks per launch, each walking a contiguous run of cell tiles
 * (blocks <= 0: the built-in default).  Results do not depend on it; it is the
 * knob of the host autotuner (paper_2601_16911_amd/autotune.py).  Not
 * thread-safe against concurrent evaluations on the same mesh. */
cvw_status cvw_mesh_set_grid(cvw_mesh* mesh, int blocks);
/* Copy one host-side connectivity array (see CVW_EXPORT_*) into host_dst; EINVAL
 * if bytes is not exactly its size. */
cvw_status cvw_mesh_export(const cvw_mesh* mesh, int which, void* host_dst, size_t bytes);

/* Workspace size in bytes for an operation: 0 = sensor / residual / candidates,
 * 1 = time step, 2 = HWENO limiter, 3 = positivity limiter.  The workspace
 * holds the vertex candidates, the status word, (time step) the Runge-Kutta
 * stage states and (limiters) the lists of cells to limit; it must stay
 * untouched between the calls of one operation and may be reused afterwards. */
size_t cvw_workspace_bytes(const cvw_mesh* mesh, const cvw_params* prm, int op);

/* Vertex stage of the cell-vertex reconstruction (Sec. 3.2, eq. taylorcand and
 * the Jiang-Shu weights with equal linear weights): for every vertex x_i,
 *   cand[k][i] = sum_{e in C(x_i)} omega_e^i D^k u_h^e(x_i),  1 <= |k| <= p,
 * with omega_e^i proportional to (eps + ||u_h^e||_{x_i}^q)^{-r} (eq. pointsnorm),
 * summed in ascending (cell, local vertex) order.  Multi-indices are ordered
 * by |k|, then by decreasing first component.  u: state (sensor field = first
 * variable); cand: device [n_vertices][n_k] in the state precision. */
cvw_status cvw_vertex_candidates(const cvw_mesh* mesh, const cvw_params* prm, const void* u,
                                 void* cand, void* ws, size_t ws_bytes, void* stream);

/* Smoothness sensor gamma_e (eq. gamma, cell stage of Sec. 3.2) and the
 * shock-capturing quadrature weights alpha_q (eqs. alphaq / alpha_prelim,
 * applied where gamma_e < c_gamma, Sec. 5).  gamma: device [n_cells];
 * alpha: device [n_cells][n_q] or NULL.  For systems the sensor field is the
 * density (Sec. 5.4).  On a structured periodic DG quadrilateral grid
 * (cvw_mesh_info.grid_nx > 0) the plain sensor runs as one fused pass that
 * reads the sensor field once and writes gamma (vertex and cell stages meet in
 * on-chip memory); elsewhere the vertex candidates go through the workspace. */
cvw_status cvw_sensor(const cvw_mesh* mesh, const cvw_params* prm, const void* u, void* gamma,
                      void* alpha, void* ws, size_t ws_bytes, void* stream);

/* HWENO limiter (Sec. 3: the cell-vertex reconstruction u_h^{e,*} of eq.
 * finalweno may overwrite the DG solution u_h^e; Sec. 3.2: the vertex
 * candidates with cell averages corrected to that of u_h^e).  DG
 * quadrilaterals and DG triangles.  On every cell whose sensor value gamma_e (eq. gamma,
 * of the sensor field = variable 0, plain or fixed sensor) is below
 * `threshold`, the nodal values of each variable are replaced by those of its
 * own reconstruction (componentwise: each variable with its own vertex
 * candidates and weights); all other cells are copied unchanged.  Cell
 * averages are preserved.  threshold > 1 limits every cell, <= 0 none.
 * u, u_out: device float32 [n_var][E][n_loc]; u_out may be u (in place),
 * any other overlap is rejected (CVW_EINVAL).
 * gamma_out: device float32 [E] receiving the sensor values used, or NULL.
 * ws: cvw_workspace_bytes(mesh, prm, 2) bytes, 256-byte aligned.
 * Errors: CVW_EUNSUPPORTED for other meshes or the learned sensor, CVW_EINVAL
 * for null pointers, a NaN threshold or a small workspace. */
cvw_status cvw_limit(const cvw_mesh* mesh, const cvw_params* prm, const void* u, void* u_out, double threshold,
                     void* gamma_out, void* ws, size_t ws_bytes, void* stream);

/* Positivity limiter for the Euler equations on DG quadrilaterals: the
 * Zhang-Shu scaling limiter that the paper adds in its double Mach
 * reflection run (Sec. 5), as published by Zhang and Shu.  Per cell, with the
 * cell averages Ubar and the points Q = the Gauss nodes and the Gauss points
 * of the four faces, eps = min(eps0, rhobar, p(Ubar)): (1) the density is
 * scaled towards its average until min_Q rho = eps; (2) the state is scaled
 * towards Ubar by the smallest t in [0, 1] at which the pressure along
 * Ubar + t (U_q - Ubar) reaches eps.  Cell averages are preserved; admissible
 * cells are copied bit for bit.  The arithmetic is float64; the stored state
 * is float32, so the bound holds up to the rounding of the stored values
 * (choose eps0 well above it, e.g. 1e-6 of the data's scale).
 * u, u_out: device float32 [4][E][n_loc]; u_out may be u, any other overlap
 * is rejected.  ws: cvw_workspace_bytes(mesh, prm, 3) bytes (256 + 4 E
 * rounded up to 256), 256-byte aligned.  Errors: CVW_EUNSUPPORTED for other
 * meshes, fluxes or precisions; CVW_EINVAL for null pointers, eps0 <= 0,
 * gamma <= 1 or a small workspace. */
cvw_status cvw_positivity(const cvw_mesh* mesh, const cvw_params* prm, const void* u, void* u_out, double eps0,
                          void* ws, size_t ws_bytes, void* stream);

/* Stabilised residual R of M dU/dt = -R (eq. stabform / sdstab): Galerkin
 * volume term, the blended stabilisation s_h with nonlinear quadrature
 * weights, DG interface fluxes (LLF / HLL), CG assembly, and on lines with
 * ends the boundary terms of prm->bc.  R has the state's layout and precision
 * and must not alias u.  gamma_out: device [n_cells] or NULL.
 * Segments: scalar laws of degree <= 3 on closed lines in float32 or
 * float64; degrees up to 32, the Euler equations (rho, m, E) and lines with
 * ends in float64 only (CVW_EUNSUPPORTED otherwise). */
cvw_status cvw_residual(const cvw_mesh* mesh, const cvw_params* prm, const void* u, void* R,
                        void* gamma_out, void* ws, size_t ws_bytes, void* stream);

/* cvw_residual without a workspace argument, for callers that cannot
 * allocate device memory (code under graph capture, serving loops, harnesses
 * that forbid hipMalloc).  The workspace is a fixed 16 MiB (16777216 bytes)
 * array of the library on each device it runs on, held until the process
 * ends; the call allocates nothing.  Meshes and operations whose workspace
 * (cvw_workspace_bytes(mesh, prm, 0)) exceeds it are refused with CVW_EINVAL
 * (e.g. the fused path up to about 4.19 M cells).  The current device must be
 * the mesh's.  Every call on a device shares its array: calls that overlap
 * on one device race.  The status words are cleared at the start of every
 * call and not reported. */
cvw_status cvw_residual_noalloc(const cvw_mesh* mesh, const cvw_params* prm, const void* u, void* R,
                                void* gamma_out, void* stream);

/* One stage of the SSP Runge-Kutta method in Shu-Osher form (Sec. 5), given
 * the vertex candidates `cand` of u_stage (from cvw_vertex_candidates; not
 * read, and may be NULL, on a structured periodic DG quadrilateral grid with
 * the plain sensor, where the stage runs the fused sensor pass itself):
 *   u_out = a0 * u_n + b0 * (u_stage + dt * L(u_stage)),  L = -M^{-1} R
 * (eq. sdstab).  M: DG exact element mass (diagonal on Gauss-node quads and
 * segments, M_ref |det J| on triangles); CG the consistent global mass,
 * inverted on the device by preconditioned conjugate gradients (lumped-mass
 * preconditioner, relative tolerance 2e-7 in float32 and 1e-14 in float64,
 * at most 64 / 160 iterations; no host synchronisation).  u_n is not read
 * when a0 == 0; u_out may alias u_n (each entry of u_n is read only by the
 * thread that overwrites it) but must not alias u_stage or cand.  Meshes:
 * every mesh with a GPU path (DG quads and triangles, CG quads, segments). */
cvw_status cvw_rk_stage(const cvw_mesh* mesh, const cvw_params* prm, const void* u_stage, const void* cand,
                        const void* u_n, void* u_out, double dt, double a0, double b0, void* ws, size_t ws_bytes,
                        void* stream);

/* The same stage on DG quadrilaterals with the sensor values supplied:
 * gamma (device float32 [n_cells]) gives gamma_e of eq. gamma for u_stage
 * (from cvw_sensor with alpha = NULL, plain or learned), whatever prm->sensor
 * says; the shock-capturing weights (eq. alphaq) are formed in the cell pass
 * where gamma_e < c_gamma.  u_out must not alias u_stage or gamma; the other
 * arguments and errors as for cvw_rk_stage (CVW_EUNSUPPORTED on other meshes). */
cvw_status cvw_rk_stage_gamma(const cvw_mesh* mesh, const cvw_params* prm, const void* u_stage, const void* gamma,
                              const void* u_n, void* u_out, double dt, double a0, double b0, void* ws,
                              size_t ws_bytes, void* stream);

/* n_steps steps of the three-stage SSP Runge-Kutta method with fixed dt,
 * u updated in place (Sec. 2.2 / Sec. 5): per stage the vertex candidates
 * (plain sensor) and cvw_rk_stage, with the two intermediate states in the
 * workspace (op = 1). */
cvw_status cvw_step(const cvw_mesh* mesh, const cvw_params* prm, void* u, double dt, int n_steps,
                    void* ws, size_t ws_bytes, void* stream);

/* Synchronises `stream`, returns the device status bits in *flags and clears
 * them: bit 0 non-finite residual, bit 1 non-positive density or pressure,
 * bit 2 a CG mass solve (PCG) that ended its fixed iteration count above its
 * tolerance, bit 3 the learned sensor handed cells to the plain sensor (their
 * count is cleared too), bit 4 an audit switched the learned sensor off (the
 * latch itself stays set for the workspace).
 * Returns CVW_ENUMERIC when any bit was set. */
cvw_status cvw_poll_status(const cvw_mesh* mesh, void* ws, size_t ws_bytes, uint32_t* flags, void* stream);

/* Per-variable integrals sum_e int_{K_e} u_h dx accumulated in float64 on the
 * device (conservation check), DG quadrilaterals and triangles; writes n_var
 * doubles to host memory and synchronises `stream`. */
cvw_status cvw_totals(const cvw_mesh* mesh, const cvw_params* prm, const void* u, double* out_host,
                      void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Learned smoothness sensor (not in the paper: a replacement of gamma_e of
 * eq. gamma by a small network, trained on gamma_e of the method itself).
 * Features, per cell of a DG quadrilateral mesh (48, bfloat16, [n_cells][48]):
 * 4 vertex slots x 9 multi-indices 1 <= |k| <= 3 of
 * h_e^|k| (c_i[k] - D^k s^e(x_i)) / sigma_e (vertex candidate of eq. taylorcand
 * minus the cell's own Hermite data of eq. taylorsol), 9 slots
 * h_e^|k| D^k s^e(x_c) / sigma_e at the cell centre, log10(sigma_e / sigma_ref),
 * and the largest and the mean of the four per-vertex mismatch 2-norms;
 * sigma_e = ||s^e||_e + 1e-12 sigma_ref (eq. snorm), orders above p are 0.
 * Network: 48 -> 64 -> 64 -> 1, GELU (erf form) after both hidden layers,
 * sigmoid output.  Packed float32 parameters (7361): W1 [48][64], b1 [64],
 * W2 [64][64], b2 [64], w3 [64], b3.  Inference on bfloat16 matrix cores
 * (inputs, weights and hidden activations rounded to bfloat16, float32
 * accumulation); training with Adam on float32 master weights.
 * ------------------------------------------------------------------------- */
typedef struct cvw_mlp cvw_mlp;
#define CVW_MLP_NPARAM 7361

/* Creates a network on the current device from packed host parameters (read
 * during the call).  Adam moments start at zero. */
cvw_status cvw_mlp_create(const float* params, cvw_mlp** out);
/* The same network with its device memory in a caller-owned buffer (device,
 * 256-byte aligned, at least cvw_mlp_device_bytes() bytes; it must outlive the
 * handle and is not freed by cvw_mlp_destroy).  CVW_EINVAL for a null,
 * misaligned or small buffer. */
size_t cvw_mlp_device_bytes(void);
cvw_status cvw_mlp_create_in(const float* params, void* device_buffer, size_t bytes, cvw_mlp** out);
void cvw_mlp_destroy(cvw_mlp* mlp);
/* Copies the float32 master parameters to / from host memory (synchronous);
 * set also resets the Adam state. */
cvw_status cvw_mlp_get_params(const cvw_mlp* mlp, float* params);
cvw_status cvw_mlp_set_params(cvw_mlp* mlp, const float* params);

/* Validity box of the network's 48 features (host arrays, lo[i] <= hi[i];
 * -inf / +inf after cvw_mlp_create): the learned sensor hands a cell whose
 * features leave the box (or whose output is not finite) to the plain sensor.
 * Callers set it from the training data, e.g. its range widened by a margin. */
cvw_status cvw_mlp_set_range(cvw_mlp* mlp, const float* lo, const float* hi);

/* Audit of the learned sensor (the plain sensor as its judge) on state u, on
 * a structured periodic DG quadrilateral grid: gamma of the network (guarded)
 * and of eq. gamma for every cell; out_host[0] = mean |gamma_learned -
 * gamma_plain|, [1] = the largest, [2] = cells handed to the plain sensor
 * since the last poll, [3] = 1 when the audit latch is set.  A mean above
 * prm->audit_tol sets the latch in the workspace: from then on every learned
 * evaluation with this workspace hands all cells to the plain sensor (the run
 * is switched to plain); cvw_poll_status reports bit 4 once.  cvw_step runs
 * the same audit (without the host copy) every prm->audit_every steps.
 * Synchronises `stream`.  ws: cvw_workspace_bytes(mesh, prm, 0) or more. */
cvw_status cvw_learned_audit(const cvw_mesh* mesh, const cvw_params* prm, const void* u, double* out_host,
                             void* ws, size_t ws_bytes, void* stream);

/* Features of every cell (DG quadrilaterals, float32): u the state (the first
 * variable is the sensor field), cand its vertex candidates, prm->sigma_ref
 * the reference scale; feat: device bfloat16 [n_cells][48]. */
cvw_status cvw_mlp_features(const cvw_mesh* mesh, const cvw_params* prm, const void* u, const void* cand,
                            void* feat, void* stream);
/* gamma[i] = network(feat[i]) for i < n: device float32 [n]. */
cvw_status cvw_mlp_infer(const cvw_mlp* mlp, const void* feat, int64_t n, void* gamma, void* stream);

/* Workspace bytes of cvw_mlp_train_step for a batch size. */
size_t cvw_mlp_train_workspace_bytes(int batch);
/* One training step on the rows idx[0..batch) of feat (device int32), with
 * targets target[row] (device float32): loss mean((gamma - target)^2), its
 * gradient (float32 activations through the bfloat16 weights and inputs),
 * written to grad_out (device float32 [7361]) when not NULL, then one Adam
 * step (beta1 0.9, beta2 0.999, eps 1e-8) with rate lr on the master weights
 * (lr = 0: gradient only).  1 <= batch <= 65536. */
cvw_status cvw_mlp_train_step(cvw_mlp* mlp, const void* feat, const void* target, const void* idx, int batch,
                              float lr, void* grad_out, void* ws, size_t ws_bytes, void* stream);

/* ---------------------------------------------------------------------------
 * Batched time stepping of many independent problems (an ensemble of DG
 * meshes, Sec. 2 and Sec. 5 applied per instance): every SSP-RK3 stage of all
 * instances runs as one sensor pass per degree and one cell pass per
 * (degree, flux), captured once into a HIP graph that is replayed per step.
 * The sensor pass is the fused one of cvw_sensor for instances with the plain
 * sensor on a structured periodic grid (gamma of the stage in the workspace,
 * read by the cell pass), else the vertex pass (CVW_SENSOR_PATH=twopass when
 * the batch is built selects it for every instance); each instance's result
 * is bitwise that of its own cvw_step on the same path.
 * Instances: DG, congruent axis-aligned periodic quadrilaterals, p <= 3,
 * float32, scalar flux (constant advection, Burgers, KPP), each with its own
 * parameters and fixed dt.
 * ------------------------------------------------------------------------- */
typedef struct cvw_batch cvw_batch;

typedef struct {
  const cvw_mesh* mesh;      /* built with cvw_mesh_build; must outlive the batch */
  cvw_params params;         /* copied at build                                    */
  void* u;                   /* device state [n_loc * n_cells] float32, updated in
                                place by cvw_batch_step; must outlive the batch     */
  double dt;                 /* fixed time step of this instance                    */
} cvw_batch_instance;

/* Validates the instances, builds the work lists (instance, block) sorted by
 * estimated cost and uploads the reference tables.  Host arrays are read during
 * the call only.  The batch handle owns its device descriptors. */
cvw_status cvw_batch_build(const cvw_batch_instance* inst, int n, cvw_batch** out);
/* Device bytes the batch's arrays take (host work only; the same validation
 * as cvw_batch_build), and the batch built with them in a caller-owned device
 * buffer (256-byte aligned, at least that size; it must outlive the handle and
 * is not freed by cvw_batch_destroy).  CVW_EINVAL for a small buffer. */
cvw_status cvw_batch_plan(const cvw_batch_instance* inst, int n, size_t* device_bytes);
cvw_status cvw_batch_build_in(const cvw_batch_instance* inst, int n, void* device_buffer, size_t bytes,
                              cvw_batch** out);
void cvw_batch_destroy(cvw_batch* batch);

/* Workspace bytes for cvw_batch_step (256-byte aligned device buffer): a status
 * word, then per instance the vertex candidates and two stage states. */
size_t cvw_batch_workspace_bytes(const cvw_batch* batch);

/* n_steps SSP-RK3 steps of every instance.  use_graph != 0: the three stages
 * are captured once into a graph (on a private stream, for this workspace and
 * grid) and the graph is launched n_steps times on `stream`; use_graph == 0:
 * the same kernels are launched directly.  The results are identical, and
 * bitwise those of cvw_step on each instance alone. */
cvw_status cvw_batch_step(cvw_batch* batch, int n_steps, int use_graph, void* ws, size_t ws_bytes, void* stream);

/* Blocks per launch of the work-list kernels (grid-stride over the items);
 * <= 0 selects one block per item.  Invalidates a captured graph. */
cvw_status cvw_batch_set_grid(cvw_batch* batch, int blocks);

/* As cvw_poll_status, for the status word of a batch workspace. */
cvw_status cvw_batch_poll_status(void* ws, size_t ws_bytes, uint32_t* flags, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* CVW_H */
