// Instantiations of the lean sweep kernel for one mode (KM_WFAIL), compiled on
// their own so that the modes build in parallel.
#include "kp_ell_impl.h"

template <>
hipError_t kp_launch_ell_mode<KM_WFAIL>(const SweepArgs &a, const EllGeom &g, size_t lds, int grid, int D,
                                   hipStream_t stream) {
  if (D == 1) return launch_ell_m<1, KM_WFAIL>(a, g, lds, grid, stream);
  return launch_ell_m<2, KM_WFAIL>(a, g, lds, grid, stream);
}
