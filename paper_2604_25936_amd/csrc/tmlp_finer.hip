// The fused T-MLP kernels for FINER-backbone models (SAND-FINER, Sec. 4.1):
// h = sin(omega (|z| + 1) z).
#include "tmlp_kernels.h"

namespace sand {
template hipError_t launch_tmlp_act<ACT_FINER>(int, int, int, const QueryArgs*, const BatchArgs*,
                                               int, hipStream_t);
}  // namespace sand
