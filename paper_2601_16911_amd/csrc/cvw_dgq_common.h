// Shared by the DG quadrilateral kernels (cell pass, vertex pass, limiter):
// the multi-index set 1 <= |k| <= P in the order of the candidate data (by
// |k|, then by decreasing first component) and an integer power.
#pragma once

#include <cstdint>

namespace cvw {

template <int P>
struct KSet {
  static constexpr int NK = (P + 1) * (P + 2) / 2 - 1;
  int x[NK], y[NK];
  constexpr KSet() : x{}, y{} {
    int t = 0;
    for (int n = 1; n <= P; ++n)
      for (int j = 0; j <= n; ++j) {
        x[t] = n - j;
        y[t] = j;
        ++t;
      }
  }
};
template <int P>
inline constexpr KSet<P> kset{};

__device__ __forceinline__ double dpow(double x, int n) {
  double r = 1.0;
  for (int i = 0; i < n; ++i) r *= x;
  return r;
}

}  // namespace cvw
