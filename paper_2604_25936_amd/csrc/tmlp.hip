// Host-side entry points of the fused T-MLP kernels: dispatch on the
// model's activation to the kernels built for it (tmlp_sine.hip,
// tmlp_finer.hip), plus the small helpers that need no T-MLP arithmetic.

#include <type_traits>

#include "mfma_common.h"

namespace sand {

namespace {

using namespace mfma;

// Points xyz[i * stride], i < n, gathered into out (a sample of a query).
__global__ void k_gather_points(const float* __restrict__ xyz, int64_t stride, int64_t n,
                                float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float* p = xyz + 3 * (i * stride);
  out[3 * i] = p[0];
  out[3 * i + 1] = p[1];
  out[3 * i + 2] = p[2];
}

hipError_t dispatch(int what, int act, int prec, int WP, const QueryArgs* q, const BatchArgs* b,
                    int num_cu, hipStream_t s) {
  if (act == ACT_SINE) return launch_tmlp_act<ACT_SINE>(what, prec, WP, q, b, num_cu, s);
  if (act == ACT_FINER) return launch_tmlp_act<ACT_FINER>(what, prec, WP, q, b, num_cu, s);
  return hipErrorInvalidValue;
}

}  // namespace

int tmlp_tile_points(int prec, int WP) {
  const int nq = prec == PREC_FP32 ? 16 : 32;
  return (WP > 256 ? 8 : SAND_FWD_WAVES) * nq;
}

hipError_t launch_tmlp(int prec, const QueryArgs& a, int num_cu, hipStream_t s) {
  return dispatch(0, a.m.act, prec, a.m.WP, &a, nullptr, num_cu, s);
}

hipError_t launch_tmlp_resume(int prec, const QueryArgs& a, int num_cu, hipStream_t s) {
  return dispatch(1, a.m.act, prec, a.m.WP, &a, nullptr, num_cu, s);
}

hipError_t launch_tmlp_batch(int prec, int WP, int act, const BatchArgs& a, int num_cu,
                             hipStream_t s) {
  return dispatch(2, act, prec, WP, nullptr, &a, num_cu, s);
}

int dyn_record_bytes(int prec, int WP) {
  auto pick = [&](auto tag) -> int {
    constexpr int P = decltype(tag)::value;
    switch (WP) {
      case 64: return Cfg<P, 64>::REC;
      case 128: return Cfg<P, 128>::REC;
      case 256: return Cfg<P, 256>::REC;
      default: return Cfg<P, 352>::REC;
    }
  };
  if (prec == PREC_FP32) return pick(std::integral_constant<int, PREC_FP32>{});
  if (prec == PREC_BF16) return pick(std::integral_constant<int, PREC_BF16>{});
  return pick(std::integral_constant<int, PREC_FP16>{});
}

hipError_t launch_gather_points(const float* xyz, int64_t stride, int64_t n, float* out,
                                hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_points, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, xyz,
                     stride, n, out);
  return hipGetLastError();
}

}  // namespace sand
