// Instantiations of the column kernel for OP_HIST1, OP_HIST2.
#include "sc_column.h"

namespace sc {

template hipError_t launch_column_op<OP_HIST1>(int src, bool spec,
                                               const ColArgs &a, int nb, hipStream_t s);
template hipError_t launch_column_op<OP_HIST2>(int src, bool spec,
                                               const ColArgs &a, int nb, hipStream_t s);

}  // namespace sc
