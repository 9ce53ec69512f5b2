// Launchers of the limiter kernels that are not part of the residual path
// (cvw_limit.hip).
#pragma once

#include "cvw_internal.h"

namespace cvw {

// Zhang-Shu positivity limiter, Euler on DG quadrilaterals
cvw_status dgquad_positivity(const cvw_mesh* m, const float* u, float* out, const LimitNodes& ln, double gam,
                             double eps0, hipStream_t s);

}  // namespace cvw
