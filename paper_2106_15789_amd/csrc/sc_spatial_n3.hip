// Spatial cascade kernels with 3 boxcar passes per axis (see sc_spatial.h).
#include "sc_spatial.h"

namespace sc {
template hipError_t launch_strip<1, 3>(const StripArgs &, int, bool, hipStream_t);
template hipError_t launch_strip<2, 3>(const StripArgs &, int, bool, hipStream_t);
template hipError_t launch_strip<3, 3>(const StripArgs &, int, bool, hipStream_t);
template hipError_t launch_strip<4, 3>(const StripArgs &, int, bool, hipStream_t);
template hipError_t launch_strip<5, 3>(const StripArgs &, int, bool, hipStream_t);
}  // namespace sc
