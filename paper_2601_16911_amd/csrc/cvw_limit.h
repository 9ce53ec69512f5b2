// Launchers of the limiter kernels that are not part of the residual path
// (cvw_limit.hip).
#pragma once

#include "cvw_internal.h"

namespace cvw {

// the cells with gamma_e < threshold appended to list[0 .. count[0]) (any
// order); count[1] is cleared as well
cvw_status limit_select(const float* gamma, int64_t E, double threshold, uint32_t* count, int32_t* list,
                        hipStream_t s);

// HWENO limiter on DG triangles (cvw_tri.hip): cand holds every variable's
// vertex candidates [n_var][Nv][n_k]; list == nullptr: every cell
cvw_status tri_limit(const cvw_mesh* m, const cvw_params* prm, const float* u, float* out, const float* cand,
                     const uint32_t* count, const int32_t* list, hipStream_t s);

// Zhang-Shu positivity limiter, Euler on DG quadrilaterals; count: 256 bytes,
// list: [E] (the cells the float64 stage takes)
cvw_status dgquad_positivity(const cvw_mesh* m, const float* u, float* out, const LimitNodes& ln, double gam,
                             double eps0, uint32_t* count, int32_t* list, hipStream_t s);

// Zhang-Shu positivity limiter, Euler on DG triangles: one float64 thread per
// cell over the points of the volume rule and the edge Gauss points (every
// cell written when out != u)
cvw_status tri_positivity(const cvw_mesh* m, const float* u, float* out, double gam, double eps0, hipStream_t s);

}  // namespace cvw
