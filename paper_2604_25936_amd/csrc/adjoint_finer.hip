// The input-gradient kernel for FINER-backbone models (SAND-FINER, Sec. 4.1):
// h = sin(omega (|z| + 1) z).
#include "adjoint_kernels.h"

namespace sand {
template hipError_t launch_adjoint_act<ACT_FINER>(int, const AdjointArgs&, int, hipStream_t);
}  // namespace sand
