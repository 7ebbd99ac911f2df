// Sampled-Gaussian spatial kernels of radius 17..24 (see sc_gauss.h).
#include "sc_gauss.h"

namespace sc {
template hipError_t launch_gauss_r<17>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<18>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<19>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<20>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<21>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<22>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<23>(const GaussArgs &, int, bool, hipStream_t);
template hipError_t launch_gauss_r<24>(const GaussArgs &, int, bool, hipStream_t);
}  // namespace sc
