// Spatial cascade kernels with 6 boxcar passes per axis (see sc_spatial.h).
#include "sc_spatial.h"

namespace sc {
template hipError_t launch_strip<1, 6>(const StripArgs &, int, bool, hipStream_t);
template hipError_t launch_strip<2, 6>(const StripArgs &, int, bool, hipStream_t);
}  // namespace sc
