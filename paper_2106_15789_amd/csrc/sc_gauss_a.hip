// Sampled-Gaussian spatial kernels of radius 1..8 (see sc_gauss.h).
#include "sc_gauss.h"

namespace sc {
template hipError_t launch_gauss_r<1>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<2>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<3>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<4>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<5>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<6>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<7>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<8>(const GaussArgs &, int, bool, hipStream_t);
}  // namespace sc
