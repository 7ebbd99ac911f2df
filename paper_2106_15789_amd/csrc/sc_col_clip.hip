// Instantiations of the column kernel for OP_CLIP.
#include "sc_column.h"

namespace sc {

template hipError_t launch_column_op<OP_CLIP>(int src, bool spec,
                                               const ColArgs &a, int nb, hipStream_t s);

}  // namespace sc
