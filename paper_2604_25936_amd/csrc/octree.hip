// Building the sparse network-depth octree on the GPU (Sec. 3.2, Eq. 5-7).
//
// Top-down, one level at a time: the candidates of level l are the eight
// children of every internal node of level l-1 (child slot 8 rank + child,
// in Morton order of the parents). The T-MLP evaluates y_L at every
// candidate's centre; a candidate intersects the shape the network
// represents when |y_L| is at most half its diagonal, sqrt(3) 2^-l (the
// paper's centre-distance test). Intersecting candidates above level D
// become internal (a bit in the level's Morton bitmask); those at level D
// are near leaves, whose depth is the maximum of Eq. 5 over sub-cell
// samples (the map builder's pooling kernel); every other candidate is a
// far leaf storing y_L at its centre (Eq. 7). Each level's bitmask gets an
// exclusive popcount prefix per 64-bit word (its rank array) and the list
// of its internal codes in Morton order (the next level's parents).

#include "sand_internal.h"

namespace sand {

namespace {

constexpr int kThreads = 256;
constexpr int kRankThreads = 1024;

int grid_for(int64_t n) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return (int)(b < 4096 ? (b > 0 ? b : 1) : 4096);
}

// Cell coordinates of Morton code m at `level` (bit b of i is bit 3b+2 of m,
// of j bit 3b+1, of k bit 3b).
__device__ __forceinline__ void morton_cell(uint64_t m, int level, int64_t& i, int64_t& j,
                                            int64_t& k) {
  i = j = k = 0;
  for (int b = 0; b < level; ++b) {
    i |= (int64_t)((m >> (3 * b + 2)) & 1ull) << b;
    j |= (int64_t)((m >> (3 * b + 1)) & 1ull) << b;
    k |= (int64_t)((m >> (3 * b)) & 1ull) << b;
  }
}

__device__ __forceinline__ uint64_t child_code(const uint64_t* parents, int64_t slot) {
  return 8ull * parents[slot >> 3] + (uint64_t)(slot & 7);
}

__global__ __launch_bounds__(kThreads) void k_oct_centres(const uint64_t* __restrict__ parents,
                                                          int64_t first, int64_t n, int level,
                                                          float* __restrict__ xyz) {
  const double side = 2.0 / (double)(1ll << level);
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * kThreads) {
    int64_t i, j, k;
    morton_cell(child_code(parents, first + t), level, i, j, k);
    xyz[3 * t + 0] = (float)(-1.0 + ((double)i + 0.5) * side);
    xyz[3 * t + 1] = (float)(-1.0 + ((double)j + 0.5) * side);
    xyz[3 * t + 2] = (float)(-1.0 + ((double)k + 0.5) * side);
  }
}

__global__ __launch_bounds__(kThreads) void k_oct_classify(
    const uint64_t* __restrict__ parents, const float* __restrict__ y, int64_t first, int64_t n,
    int level, int D, float h, uint64_t* __restrict__ bits, uint8_t* __restrict__ depth,
    float* __restrict__ value, int32_t* __restrict__ near_slots, uint32_t* __restrict__ near_count) {
  const int lane = threadIdx.x & 63;
  const int64_t stride = (int64_t)gridDim.x * kThreads;
  for (int64_t t0 = (int64_t)blockIdx.x * kThreads; t0 < n; t0 += stride) {
    const int64_t t = t0 + threadIdx.x;
    const bool valid = t < n;
    bool near = false;
    if (valid) {
      const int64_t slot = first + t;
      const float yy = y[t];
      const bool hit = fabsf(yy) <= h;
      if (hit && level < D) {
        const uint64_t m = child_code(parents, slot);
        atomicOr((unsigned long long*)&bits[m >> 6], 1ull << (m & 63));
        depth[slot] = 255;
        value[slot] = 0.0f;
      } else if (hit) {
        near = true;
        depth[slot] = 0;          // set by the pooled required depth
        value[slot] = 0.0f;
      } else {
        depth[slot] = 0;
        value[slot] = yy;
      }
    }
    // near leaves into near_slots, one atomic per wavefront
    const uint64_t mask = __ballot(near);
    if (mask == 0) continue;
    const int leader = __ffsll((unsigned long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(near_count, (uint32_t)__popcll(mask));
    base = __shfl(base, leader);
    if (near) {
      const uint64_t below = lane == 0 ? 0ull : (mask & (~0ull >> (64 - lane)));
      near_slots[base + __popcll(below)] = (int32_t)(first + t);
    }
  }
}

// One workgroup: rank[w] = number of set bits in words 0..w-1; *total = all.
__global__ __launch_bounds__(kRankThreads) void k_oct_rank(const uint64_t* __restrict__ bits,
                                                           int64_t words,
                                                           uint32_t* __restrict__ rank,
                                                           int64_t* __restrict__ total) {
  __shared__ uint32_t part[kRankThreads];
  const int t = threadIdx.x;
  const int64_t per = (words + kRankThreads - 1) / kRankThreads;
  const int64_t w0 = t * per, w1 = w0 + per < words ? w0 + per : words;
  uint32_t sum = 0;
  for (int64_t w = w0; w < w1; ++w) sum += (uint32_t)__popcll(bits[w]);
  part[t] = sum;
  __syncthreads();
  if (t == 0) {
    uint32_t run = 0;
    for (int k = 0; k < kRankThreads; ++k) {
      const uint32_t v = part[k];
      part[k] = run;
      run += v;
    }
    *total = run;
  }
  __syncthreads();
  uint32_t run = part[t];
  for (int64_t w = w0; w < w1; ++w) {
    rank[w] = run;
    run += (uint32_t)__popcll(bits[w]);
  }
}

// Internal codes of a level in Morton order (positions from the rank array).
__global__ __launch_bounds__(kThreads) void k_oct_list(const uint64_t* __restrict__ bits,
                                                       const uint32_t* __restrict__ rank,
                                                       int64_t words, uint64_t* __restrict__ list) {
  for (int64_t w = (int64_t)blockIdx.x * kThreads + threadIdx.x; w < words;
       w += (int64_t)gridDim.x * kThreads) {
    uint64_t b = bits[w];
    uint32_t at = rank[w];
    while (b) {
      const int i = __ffsll((unsigned long long)b) - 1;
      list[at++] = 64ull * (uint64_t)w + (uint64_t)i;
      b &= b - 1ull;
    }
  }
}

// Sample t of the chunk: sub-cell (t % s^3) of near leaf near_slots[t / s^3].
__global__ __launch_bounds__(kThreads) void k_oct_samples(const int32_t* __restrict__ near_slots,
                                                          const uint64_t* __restrict__ parents,
                                                          int64_t first, int64_t nsamp, int D,
                                                          int sps, float* __restrict__ xyz) {
  const int64_t s3 = (int64_t)sps * sps * sps;
  const double side = 2.0 / (double)(1ll << D);
  for (int64_t q = (int64_t)blockIdx.x * kThreads + threadIdx.x; q < nsamp;
       q += (int64_t)gridDim.x * kThreads) {
    const int64_t t = first + q;
    int64_t i, j, k;
    morton_cell(child_code(parents, near_slots[t / s3]), D, i, j, k);
    const int sub = (int)(t % s3);
    const int kx = sub / (sps * sps), ky = (sub / sps) % sps, kz = sub % sps;
    xyz[3 * q + 0] = (float)(-1.0 + side * ((double)i + (kx + 0.5) / sps));
    xyz[3 * q + 1] = (float)(-1.0 + side * ((double)j + (ky + 0.5) / sps));
    xyz[3 * q + 2] = (float)(-1.0 + side * ((double)k + (kz + 0.5) / sps));
  }
}

__global__ __launch_bounds__(kThreads) void k_oct_finish(const int32_t* __restrict__ near_slots,
                                                         int64_t nnear,
                                                         const uint32_t* __restrict__ depth32,
                                                         uint8_t* __restrict__ depth) {
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nnear;
       i += (int64_t)gridDim.x * kThreads) {
    const int32_t slot = near_slots[i];
    depth[slot] = (uint8_t)depth32[slot];
  }
}

}  // namespace

hipError_t launch_oct_centres(const uint64_t* parents, int64_t first, int64_t nslots, int level,
                              float* xyz, hipStream_t s) {
  hipLaunchKernelGGL(k_oct_centres, dim3(grid_for(nslots)), dim3(kThreads), 0, s, parents, first,
                     nslots, level, xyz);
  return hipGetLastError();
}

hipError_t launch_oct_classify(const uint64_t* parents, const float* y, int64_t first,
                               int64_t nslots, int level, int D, float h, uint64_t* bits,
                               uint8_t* depth, float* value, int32_t* near_slots,
                               uint32_t* near_count, hipStream_t s) {
  hipLaunchKernelGGL(k_oct_classify, dim3(grid_for(nslots)), dim3(kThreads), 0, s, parents, y,
                     first, nslots, level, D, h, bits, depth, value, near_slots, near_count);
  return hipGetLastError();
}

hipError_t launch_oct_rank(const uint64_t* bits, int64_t words, uint32_t* rank, int64_t* total,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_oct_rank, dim3(1), dim3(kRankThreads), 0, s, bits, words, rank, total);
  return hipGetLastError();
}

hipError_t launch_oct_list(const uint64_t* bits, const uint32_t* rank, int64_t words,
                           uint64_t* list, hipStream_t s) {
  hipLaunchKernelGGL(k_oct_list, dim3(grid_for(words)), dim3(kThreads), 0, s, bits, rank, words,
                     list);
  return hipGetLastError();
}

hipError_t launch_oct_samples(const int32_t* near_slots, const uint64_t* parents, int64_t first,
                              int64_t nsamp, int D, int sps, float* xyz, hipStream_t s) {
  hipLaunchKernelGGL(k_oct_samples, dim3(grid_for(nsamp)), dim3(kThreads), 0, s, near_slots,
                     parents, first, nsamp, D, sps, xyz);
  return hipGetLastError();
}

hipError_t launch_oct_finish(const int32_t* near_slots, int64_t nnear, const uint32_t* depth32,
                             uint8_t* depth, hipStream_t s) {
  hipLaunchKernelGGL(k_oct_finish, dim3(grid_for(nnear)), dim3(kThreads), 0, s, near_slots, nnear,
                     depth32, depth);
  return hipGetLastError();
}

namespace {

// One thread per level-K cell (Morton code c): the cell's child index at
// level l is the l-th octal digit of c from the top; descend from the root as
// the lookup does and record the leaf holding the cell, or that the cell is
// an internal node.
__global__ __launch_bounds__(kThreads) void k_oct_top(OctreeArgs o, int K, uint2* __restrict__ top) {
  const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= ((int64_t)1 << (3 * K))) return;
  uint64_t p = 0;
  uint64_t w = o.bits[0][0];
  for (int l = 1; l <= K; ++l) {
    const uint64_t child = (uint64_t)(c >> (3 * (K - l))) & 7u;
    const uint64_t m = 8u * p + child;
    const uint64_t r = o.rank[l - 1][p >> 6] + (uint64_t)__popcll(w & ((1ull << (p & 63)) - 1ull));
    const uint64_t slot = 8u * r + child;
    const uint64_t wn = l < o.D ? o.bits[l][m >> 6] : 0ull;
    if ((wn >> (m & 63)) & 1ull) {
      if (l == K) {
        top[c] = make_uint2(kOctInternal, 0u);
        return;
      }
      p = m;
      w = wn;
    } else {
      top[c] = make_uint2((uint32_t)o.depth[l][slot], __float_as_uint(o.value[l][slot]));
      return;
    }
  }
}

}  // namespace

hipError_t launch_oct_top(const OctreeArgs& oa, int K, uint2* top, hipStream_t s) {
  const int64_t cells = (int64_t)1 << (3 * K);
  hipLaunchKernelGGL(k_oct_top, dim3((unsigned)((cells + kThreads - 1) / kThreads)),
                     dim3(kThreads), 0, s, oa, K, top);
  return hipGetLastError();
}

}  // namespace sand
