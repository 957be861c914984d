// The input-gradient kernel for SIREN-backbone models: h = sin(omega z).
#include "adjoint_kernels.h"

namespace sand {
template hipError_t launch_adjoint_act<ACT_SINE>(int, const AdjointArgs&, int, hipStream_t);
}  // namespace sand
