// Instantiations of the column kernel for OP_SELCLIP (selection pass with the
// clip of every voxel outside the threshold window).
#include "sc_column.h"

namespace sc {

template hipError_t launch_column_op<OP_SELCLIP>(int src, bool spec,
                                                const ColArgs &a, int nb, hipStream_t s);

}  // namespace sc
