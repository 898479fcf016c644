// Instantiations of the lean sweep kernel for one mode (KM_FIX), compiled on
// their own so that the modes build in parallel.
#include "kp_ell_impl.h"

template <>
hipError_t kp_launch_ell_mode<KM_FIX>(const SweepArgs &a, const EllGeom &g, size_t lds, int grid, int D,
                                   hipStream_t stream, int *used) {
  if (D == 1) return launch_ell_m<1, KM_FIX>(a, g, lds, grid, stream, used);
  return launch_ell_m<2, KM_FIX>(a, g, lds, grid, stream, used);
}

template <>
int kp_ell_resident_mode<KM_FIX>(int D, int M, size_t lds, int waves) {
  return D == 1 ? resident_blocks_m<1, KM_FIX>(M, lds, waves) : resident_blocks_m<2, KM_FIX>(M, lds, waves);
}
