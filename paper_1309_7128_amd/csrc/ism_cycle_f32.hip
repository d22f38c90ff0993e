// The fused cycle kernel for FP32 fine grids, nu = 1 .. 5.
#include "ism_cycle.h"

namespace ism {

template <>
hipError_t launch_cycle_fused<float>(const Geo& g, const float* rhs, const float* ein, float* eout,
                                     const double* E, double* rc, double* psq, int nu, int zero_e,
                                     hipStream_t s, const double* stop, int maxmode) {
  if (maxmode && nu != 1) return hipErrorInvalidValue;  // the maxima exist for nu = 1 only
  return launch_cycle_upto<float, 5>(g, rhs, ein, eout, E, rc, psq, nu, zero_e, s, stop, maxmode);
}

template <>
int fused_max_nu<float>() {
  return 5;
}

}  // namespace ism
