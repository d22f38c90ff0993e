// The fused cycle kernel for FP64 fine grids, nu = 1 .. 4.
#include "ism_cycle.h"

namespace ism {

template <>
hipError_t launch_cycle_fused<double>(const Geo& g, const double* rhs, const double* ein, double* eout,
                                      const double* E, double* rc, double* psq, int nu, int zero_e,
                                      hipStream_t s, const double* stop, int maxmode) {
  if (maxmode && nu != 1) return hipErrorInvalidValue;  // the maxima exist for nu = 1 only
  return launch_cycle_upto<double, 4>(g, rhs, ein, eout, E, rc, psq, nu, zero_e, s, stop, maxmode);
}

template <>
int fused_max_nu<double>() {
  return 4;
}

}  // namespace ism
