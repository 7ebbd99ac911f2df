// Spatial cascade kernels with 4 boxcar passes per axis (see sc_spatial.h).
#include "sc_spatial.h"

namespace sc {
template hipError_t launch_strip<1, 4>(const StripArgs &, int, bool, hipStream_t);
template hipError_t launch_strip<2, 4>(const StripArgs &, int, bool, hipStream_t);
template hipError_t launch_strip<3, 4>(const StripArgs &, int, bool, hipStream_t);
template hipError_t launch_strip<4, 4>(const StripArgs &, int, bool, hipStream_t);
}  // namespace sc
