// Host-side entry points of the input-gradient kernel: dispatch on the
// model's activation to the kernel built for it (adjoint_sine.hip,
// adjoint_finer.hip), and the stash and tile geometry.

#include "mfma_common.h"

namespace sand {

size_t adjoint_stash_bytes_per_wg(int prec, int WP, int L) {
  const int BM = prec == PREC_FP32 ? 16 : 32;
  const int lane_bytes = prec == PREC_FP32 ? 16 : 32;
  return (size_t)8 * L * (WP / BM) * 64 * lane_bytes;
}

hipError_t launch_adjoint(int prec, const AdjointArgs& a, int grid, hipStream_t s) {
  if (a.q.m.act == ACT_SINE) return launch_adjoint_act<ACT_SINE>(prec, a, grid, s);
  if (a.q.m.act == ACT_FINER) return launch_adjoint_act<ACT_FINER>(prec, a, grid, s);
  return hipErrorInvalidValue;
}

int adjoint_tile_points(int prec) {
  return prec == PREC_FP32 ? mfma::Cfg<PREC_FP32, 64>::Q : mfma::Cfg<PREC_BF16, 64>::Q;
}

}  // namespace sand
