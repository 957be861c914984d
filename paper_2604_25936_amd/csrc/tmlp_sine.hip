// The fused T-MLP kernels for SIREN-backbone models: h = sin(omega z).
#include "tmlp_kernels.h"

namespace sand {
template hipError_t launch_tmlp_act<ACT_SINE>(int, int, int, const QueryArgs*, const BatchArgs*,
                                              int, hipStream_t);
}  // namespace sand
