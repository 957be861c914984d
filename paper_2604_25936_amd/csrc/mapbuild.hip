// Building a network-depth map on the GPU (Sec. 3.2, Eq. 5-7).
//
// For a dense R^3 grid over [-1, 1]^3 and a caller-supplied near-surface
// mask: the near voxels are listed, each is sampled at the s^3 centres of
// its sub-cells, the T-MLP runs every sample to full depth writing all
// accumulated outputs y_1..y_L (the forward kernel's y_all output), and
// each sample's required depth
//     d(x) = min { i : |y_L - y_i| < r and sign(y_i) = sign(y_L) }   (Eq. 5)
// is max-pooled into its voxel (Eq. 6). Far voxels keep depth 0 and store
// the caller's SDF at their centre (Eq. 7).

#include "sand_internal.h"

namespace sand {

namespace {

constexpr int kThreads = 256;

int grid_for(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

// Near voxels into `list` in unspecified order (the map is a maximum over
// each voxel's samples, so it does not depend on it). One atomic per
// wavefront: lanes holding a near voxel take consecutive slots.
__global__ __launch_bounds__(kThreads) void k_map_list(const uint8_t* __restrict__ near,
                                                       int64_t cells, int32_t* __restrict__ list,
                                                       uint32_t* __restrict__ count) {
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t v0 = (int64_t)blockIdx.x * kThreads; v0 < cells; v0 += stride) {
    const int64_t v = v0 + threadIdx.x;
    const bool hit = v < cells && near[v] != 0;
    const uint64_t mask = __ballot(hit);
    if (mask == 0) continue;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(count, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (hit) {
      const uint64_t below = lane == 0 ? 0 : (mask & ((~0ull) >> (64 - lane)));
      list[base + __popcll(below)] = (int32_t)v;
    }
  }
}

// Samples first .. first+nsamp-1: sample t is sub-cell t % s^3 (C order
// kx, ky, kz) of voxel list[t / s^3], at -1 + (2/R)(i + (k + 1/2)/s) per
// axis (computed in FP64; exact in FP32 for power-of-two R and s).
__global__ __launch_bounds__(kThreads) void k_map_samples(const int32_t* __restrict__ list,
                                                          int64_t first, int64_t nsamp, int R,
                                                          int sps, float* __restrict__ xyz) {
  const int64_t s3 = (int64_t)sps * sps * sps;
  const double h = 2.0 / R;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nsamp;
       i += (int64_t)gridDim.x * kThreads) {
    const int64_t t = first + i;
    const int64_t v = list[t / s3];
    const int k = (int)(t % s3);
    const int64_t ix = v / ((int64_t)R * R), iy = (v / R) % R, iz = v % R;
    const int kx = k / (sps * sps), ky = (k / sps) % sps, kz = k % sps;
    xyz[3 * i + 0] = (float)(-1.0 + h * ((double)ix + (kx + 0.5) / sps));
    xyz[3 * i + 1] = (float)(-1.0 + h * ((double)iy + (ky + 0.5) / sps));
    xyz[3 * i + 2] = (float)(-1.0 + h * ((double)iz + (kz + 0.5) / sps));
  }
}

__device__ __forceinline__ int sign3(float v) { return (v > 0.0f) - (v < 0.0f); }

// Eq. 5 for each sample of the chunk, max-pooled into its voxel (Eq. 6).
__global__ __launch_bounds__(kThreads) void k_map_pool(const float* __restrict__ y_all, int L,
                                                       const int32_t* __restrict__ list,
                                                       int64_t first, int64_t nsamp, int sps,
                                                       float r, uint32_t* __restrict__ depth32) {
  const int64_t s3 = (int64_t)sps * sps * sps;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nsamp;
       i += (int64_t)gridDim.x * kThreads) {
    const float* y = y_all + i * L;
    const float yL = y[L - 1];
    const int sL = sign3(yL);
    int d = L;
    for (int j = 0; j < L - 1; ++j)
      if (fabsf(yL - y[j]) < r && sign3(y[j]) == sL) {
        d = j + 1;
        break;
      }
    atomicMax(&depth32[list[(first + i) / s3]], (uint32_t)d);
  }
}

// Eq. 7: near voxels keep the pooled depth (far value 0); far voxels depth
// 0 and the SDF at their centre.
__global__ __launch_bounds__(kThreads) void k_map_finish(const uint8_t* __restrict__ near,
                                                         const float* __restrict__ center_sdf,
                                                         const uint32_t* __restrict__ depth32,
                                                         int64_t cells, uint8_t* __restrict__ depth,
                                                         float* __restrict__ far) {
  for (int64_t v = (int64_t)blockIdx.x * kThreads + threadIdx.x; v < cells;
       v += (int64_t)gridDim.x * kThreads) {
    const bool nr = near[v] != 0;
    depth[v] = nr ? (uint8_t)depth32[v] : 0;
    far[v] = nr ? 0.0f : center_sdf[v];
  }
}

}  // namespace

hipError_t launch_map_list(const uint8_t* near, int64_t cells, int32_t* list, uint32_t* count,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_map_list, dim3(grid_for(cells)), dim3(kThreads), 0, s, near, cells, list,
                     count);
  return hipGetLastError();
}

hipError_t launch_map_samples(const int32_t* list, int64_t first, int64_t nsamp, int R, int sps,
                              float* xyz, hipStream_t s) {
  hipLaunchKernelGGL(k_map_samples, dim3(grid_for(nsamp)), dim3(kThreads), 0, s, list, first,
                     nsamp, R, sps, xyz);
  return hipGetLastError();
}

hipError_t launch_map_pool(const float* y_all, int L, const int32_t* list, int64_t first,
                           int64_t nsamp, int sps, float r, uint32_t* depth32, hipStream_t s) {
  hipLaunchKernelGGL(k_map_pool, dim3(grid_for(nsamp)), dim3(kThreads), 0, s, y_all, L, list,
                     first, nsamp, sps, r, depth32);
  return hipGetLastError();
}

hipError_t launch_map_finish(const uint8_t* near, const float* center_sdf, const uint32_t* depth32,
                             int64_t cells, uint8_t* depth, float* far, hipStream_t s) {
  hipLaunchKernelGGL(k_map_finish, dim3(grid_for(cells)), dim3(kThreads), 0, s, near, center_sdf,
                     depth32, cells, depth, far);
  return hipGetLastError();
}

}  // namespace sand
