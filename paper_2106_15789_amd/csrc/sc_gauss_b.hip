// Sampled-Gaussian spatial kernels of radius 9..16 (see sc_gauss.h).
#include "sc_gauss.h"

namespace sc {
template hipError_t launch_gauss_r<9>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<10>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<11>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<12>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<13>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<14>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<15>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<16>(const GaussArgs &, int, bool, hipStream_t);
}  // namespace sc
