// Spatial cascade kernels with 5 boxcar passes per axis (see sc_spatial.h).
#include "sc_spatial.h"

namespace sc {
template hipError_t launch_strip<1, 5>(const StripArgs &, int, bool, hipStream_t);
template hipError_t launch_strip<2, 5>(const StripArgs &, int, bool, hipStream_t);
template hipError_t launch_strip<3, 5>(const StripArgs &, int, bool, hipStream_t);
}  // namespace sc
