// Depth lookup and stable bucketing of query points by exit depth.
//
// Inference first reads every point's exit depth from the network-depth map
// and answers far-field points (depth 0) from the stored value (Sec. 3.4,
// Eq. 7); the remaining points are evaluated to their own depth. To run
// points of equal depth together, three launches build a permutation that
// groups point indices by depth, stable within each group:
//   1. k_lookup_count: per 4096-point chunk, depth per point (written as
//      uint8), far values written straight to the output, and a per-chunk
//      histogram built from wavefront ballots;
//   2. k_scan: one workgroup turns the per-chunk histograms into per-chunk
//      output offsets and writes the tile plan (deepest bucket first);
//   3. k_scatter: per chunk again, each point's rank among equal depths
//      (ballot + popcount below the lane) gives its slot in the permutation.
// Point coordinates are read through LDS so that every global load of a
// wavefront covers 256 contiguous bytes. Batched variants run the same
// bodies for several queries in one launch (each lookup block belongs to
// one query; one scan workgroup per query).

#include "sand_internal.h"

namespace sand {

namespace {

constexpr int kRounds = kLookupChunk / kLookupThreads;

__device__ __forceinline__ int cell_index(float x, float s, int half) {
  // x * s is exact (s a power of two); clamp before the float->int step so
  // that out-of-cube points and NaN land in a border cell (NaN -> cell 0).
  float v = x * s;
  if (!(v >= -s)) v = -s;
  if (v > s - 1.0f) v = s - 1.0f;
  return (int)floorf(v) + half;
}

// Leaf of the octree holding a point: its stored depth d and far value v.
// The point's cell at level D follows from the exact cell rule; its cell at
// every coarser level is that index shifted right. The descent follows
// internal nodes from the root; a node's child slot is 8 rank(parent) +
// child, rank counting the internal nodes before it at its level.
__device__ __forceinline__ void octree_leaf(const OctreeArgs& o, float x, float y, float z,
                                            int& d, float& v) {
  if (o.root_leaf) {
    d = 0;
    v = o.root_value;
    return;
  }
  const int D = o.D, half = 1 << (D - 1);
  const float s = (float)half;
  const int ix = cell_index(x, s, half), iy = cell_index(y, s, half), iz = cell_index(z, s, half);
  uint64_t p = 0;   // code of the internal node at level l-1 holding the point
  for (int l = 1; l <= D; ++l) {
    const int sh = D - l;
    const int child = (((ix >> sh) & 1) << 2) | (((iy >> sh) & 1) << 1) | ((iz >> sh) & 1);
    const uint64_t w = o.bits[l - 1][p >> 6];
    const uint64_t rk = o.rank[l - 1][p >> 6] + __popcll(w & ((1ull << (p & 63)) - 1ull));
    const uint64_t slot = 8ull * rk + (uint64_t)child;
    const uint64_t m = 8ull * p + (uint64_t)child;
    if (l < D && ((o.bits[l][m >> 6] >> (m & 63)) & 1ull)) {
      p = m;
      continue;
    }
    d = o.depth[l][slot];
    v = o.value[l][slot];
    return;
  }
  d = 0;                      // not reached: level D has no internal nodes
  v = __builtin_nanf("");
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Add the wavefront's points to hist[depth]: one LDS atomic per distinct
// depth present in the wavefront.
__device__ __forceinline__ void wave_histogram(int d, bool valid, int* hist) {
  uint64_t todo = __ballot(valid);
  const int lane = threadIdx.x & 63;
  while (todo) {
    const int leader = __ffsll((unsigned long long)todo) - 1;
    const int v = __shfl(d, leader);
    const uint64_t m = __ballot(valid && d == v);
    if (lane == leader) atomicAdd(&hist[v], __popcll(m));
    todo &= ~m;
  }
}

// Body of one lookup block: points [blk*4096, blk*4096 + 4096) of one query.
__device__ __forceinline__ void lookup_block(
    int64_t blk, const float* __restrict__ xyz, int64_t n, const uint8_t* __restrict__ map,
    int R, const float* __restrict__ far, const OctreeArgs* __restrict__ oct,
    const uint8_t* __restrict__ forced, int mode, int L, int max_depth,
    uint8_t* __restrict__ depth, float* __restrict__ sdf, float* __restrict__ grad,
    int32_t* __restrict__ counts) {
  __shared__ float sx[3 * kLookupThreads];
  __shared__ int hist[kBuckets];
  const int t = threadIdx.x;
  if (t < kBuckets) hist[t] = 0;
  const int64_t base = blk * kLookupChunk;
  const int half = R >> 1;
  const float s = (float)half;
  for (int r = 0; r < kRounds; ++r) {
    const int64_t q0 = base + (int64_t)r * kLookupThreads;
    if (q0 >= n) break;
    __syncthreads();
    for (int k = 0; k < 3; ++k) {
      const int64_t f = q0 * 3 + k * kLookupThreads + t;
      sx[k * kLookupThreads + t] = f < 3 * n ? xyz[f] : 0.0f;
    }
    __syncthreads();
    const int64_t q = q0 + t;
    const bool valid = q < n;
    int d = 0;
    if (valid) {
      const float x = sx[3 * t], y = sx[3 * t + 1], z = sx[3 * t + 2];
      int cell = -1;
      float farv = __builtin_nanf("");   // octree: the leaf's value; dense: read below
      int od = 0;
      if (oct != nullptr) {
        if (mode != 1) octree_leaf(*oct, x, y, z, od, farv);
      } else if (map != nullptr) {
        const int ix = cell_index(x, s, half), iy = cell_index(y, s, half),
                  iz = cell_index(z, s, half);
        cell = (ix * R + iy) * R + iz;
      }
      if (mode == 1) {
        d = L;
      } else if (mode == 2) {
        d = forced[q];
        if (d > L) d = L;
      } else {
        d = oct != nullptr ? od : map[cell];
      }
      if (max_depth > 0 && d > max_depth) d = max_depth;
      depth[q] = (uint8_t)d;
      if (d == 0) {
        if (oct == nullptr && far != nullptr && cell >= 0) farv = far[cell];
        if (sdf) sdf[q] = farv;
        if (grad) grad[3 * q] = grad[3 * q + 1] = grad[3 * q + 2] = 0.0f;
      }
    }
    wave_histogram(d, valid, hist);
  }
  __syncthreads();
  if (t < kBuckets) counts[blk * kBuckets + t] = hist[t];
}

__global__ __launch_bounds__(kLookupThreads) void k_lookup_count(
    const float* __restrict__ xyz, int64_t n, const uint8_t* __restrict__ map,
    int R, const float* __restrict__ far, const OctreeArgs* __restrict__ oct,
    const uint8_t* __restrict__ forced, int mode, int L, int max_depth,
    uint8_t* __restrict__ depth, float* __restrict__ sdf, float* __restrict__ grad,
    int32_t* __restrict__ counts) {
  lookup_block(blockIdx.x, xyz, n, map, R, far, oct, forced, mode, L, max_depth, depth, sdf,
               grad, counts);
}

constexpr int kScanThreads = 256;

// One workgroup: per-chunk histograms -> per-chunk bucket offsets (in
// place) and the tile plan. Bucket d >= 1 occupies perm slots
// [start[d], start[d] + count[d]); depth-0 points are not in the permutation.
__device__ __forceinline__ void scan_body(int32_t* __restrict__ counts, int64_t nblk, int L,
                                          int tile_q, Plan* __restrict__ plan) {
  __shared__ int64_t part[kScanThreads][kBuckets];
  __shared__ int64_t start[kBuckets];
  const int t = threadIdx.x;
  const int64_t per = (nblk + kScanThreads - 1) / kScanThreads;
  const int64_t b0 = t * per;
  const int64_t b1 = b0 + per < nblk ? b0 + per : nblk;
  int64_t sum[kBuckets];
  for (int d = 0; d < kBuckets; ++d) sum[d] = 0;
  for (int64_t b = b0; b < b1; ++b)
    for (int d = 0; d < kBuckets; ++d) sum[d] += counts[b * kBuckets + d];
  for (int d = 0; d < kBuckets; ++d) part[t][d] = sum[d];
  __syncthreads();
  if (t < kBuckets) {
    // exclusive scan over threads for bucket t
    int64_t run = 0;
    for (int k = 0; k < kScanThreads; ++k) {
      const int64_t v = part[k][t];
      part[k][t] = run;
      run += v;
    }
    plan->count[t] = run;
    start[t] = run;  // temporarily the total
  }
  __syncthreads();
  if (t == 0) {
    int64_t run = 0;
    for (int d = 1; d < kBuckets; ++d) {
      const int64_t tot = start[d];
      start[d] = run;
      run += tot;
    }
    start[0] = -1;
    int64_t tiles = 0;
    plan->tile_end[kBuckets] = 0;
    for (int d = kBuckets - 1; d >= 1; --d) {
      const int64_t cnt = d <= L ? plan->count[d] : 0;
      tiles += (cnt + tile_q - 1) / tile_q;
      plan->tile_end[d] = tiles;
    }
    plan->tile_end[0] = tiles;
    plan->total_tiles = tiles;
    plan->tile_q = tile_q;
    for (int d = 0; d < kBuckets; ++d) plan->start[d] = start[d];
  }
  __syncthreads();
  int64_t run[kBuckets];
  for (int d = 0; d < kBuckets; ++d) run[d] = start[d] + part[t][d];
  for (int64_t b = b0; b < b1; ++b)
    for (int d = 0; d < kBuckets; ++d) {
      const int32_t c = counts[b * kBuckets + d];
      counts[b * kBuckets + d] = (int32_t)run[d];
      run[d] += c;
    }
}

__global__ __launch_bounds__(kScanThreads) void k_scan(int32_t* __restrict__ counts,
                                                      int64_t nblk, int L, int tile_q,
                                                      Plan* __restrict__ plan) {
  scan_body(counts, nblk, L, tile_q, plan);
}

__device__ __forceinline__ void scatter_block(int64_t blk, const uint8_t* __restrict__ depth,
                                              int64_t n, const int32_t* __restrict__ offs,
                                              int32_t* __restrict__ perm) {
  __shared__ int run[kBuckets];
  __shared__ int wcnt[kLookupThreads / 64][kBuckets];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t base = blk * kLookupChunk;
  if (t < kBuckets) run[t] = offs[blk * kBuckets + t];
  for (int r = 0; r < kRounds; ++r) {
    const int64_t q0 = base + (int64_t)r * kLookupThreads;
    if (q0 >= n) break;
    __syncthreads();  // the previous round's update of run[] has read wcnt
    if (t < kBuckets * (kLookupThreads / 64)) wcnt[t / kBuckets][t % kBuckets] = 0;
    __syncthreads();
    const int64_t q = q0 + t;
    const int d = q < n ? depth[q] : 0;
    const bool valid = q < n && d > 0;
    // rank among equal depths within the wavefront
    uint64_t todo = __ballot(valid);
    int rank = 0;
    while (todo) {
      const int leader = __ffsll((unsigned long long)todo) - 1;
      const int v = __shfl(d, leader);
      const uint64_t m = __ballot(valid && d == v);
      if (valid && d == v) rank = __popcll(m & lanemask_lt());
      if (lane == leader) wcnt[w][v] = __popcll(m);
      todo &= ~m;
    }
    __syncthreads();
    if (valid) {
      int pos = run[d] + rank;
      for (int k = 0; k < w; ++k) pos += wcnt[k][d];
      perm[pos] = (int32_t)q;
    }
    __syncthreads();
    if (t < kBuckets) {
      int add = 0;
      for (int k = 0; k < kLookupThreads / 64; ++k) add += wcnt[k][t];
      run[t] += add;
    }
  }
}

__global__ __launch_bounds__(kLookupThreads) void k_scatter(
    const uint8_t* __restrict__ depth, int64_t n, const int32_t* __restrict__ offs,
    int32_t* __restrict__ perm) {
  scatter_block(blockIdx.x, depth, n, offs, perm);
}

// ---- batched variants: one launch covers several queries (server) ----

// Request owning lookup block b: the last r with reqs[r].blk0 <= b.
__device__ __forceinline__ int find_request(const BatchReq* reqs, int nreq, int64_t b) {
  int lo = 0, hi = nreq - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (reqs[mid].blk0 <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(kLookupThreads) void k_lookup_batch(const BatchReq* __restrict__ reqs,
                                                                 int nreq, int max_depth) {
  const int r = find_request(reqs, nreq, blockIdx.x);
  const BatchReq& q = reqs[r];
  lookup_block((int64_t)blockIdx.x - q.blk0, q.xyz, q.n, q.map, q.R, q.far, q.oct, nullptr, 0,
               q.L, max_depth, q.depth, q.sdf, nullptr, q.counts);
}

__global__ __launch_bounds__(kScanThreads) void k_scan_batch(BatchReq* __restrict__ reqs,
                                                            int tile_q) {
  BatchReq& q = reqs[blockIdx.x];
  scan_body(q.counts, (q.n + kLookupChunk - 1) / kLookupChunk, q.L, tile_q, &q.plan);
}

__global__ __launch_bounds__(kLookupThreads) void k_scatter_batch(const BatchReq* __restrict__ reqs,
                                                                  int nreq) {
  const int r = find_request(reqs, nreq, blockIdx.x);
  const BatchReq& q = reqs[r];
  scatter_block((int64_t)blockIdx.x - q.blk0, q.depth, q.n, q.counts, q.perm);
}

// First tile of every request and the batch's tile count.
__global__ void k_batch_tiles(BatchReq* __restrict__ reqs, int nreq,
                              int64_t* __restrict__ total) {
  if (threadIdx.x != 0) return;
  int64_t run = 0;
  for (int r = 0; r < nreq; ++r) {
    reqs[r].tile0 = run;
    run += reqs[r].plan.total_tiles;
  }
  *total = run;
}

__global__ void k_fill_u8(uint8_t* p, int64_t n, uint8_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

}  // namespace

hipError_t launch_lookup_count(const float* xyz, int64_t n, const uint8_t* map, int R,
                               const float* far, const OctreeArgs* oct, const uint8_t* forced,
                               int mode, int L, int max_depth, uint8_t* depth, float* sdf,
                               float* grad, int32_t* counts, hipStream_t s) {
  const int64_t nblk = (n + kLookupChunk - 1) / kLookupChunk;
  hipLaunchKernelGGL(k_lookup_count, dim3((unsigned)nblk), dim3(kLookupThreads), 0, s, xyz,
                     n, map, R, far, oct, forced, mode, L, max_depth, depth, sdf, grad, counts);
  return hipGetLastError();
}

hipError_t launch_scan(int32_t* counts, int64_t nblk, int L, int tile_q, Plan* plan,
                       hipStream_t s) {
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, counts, nblk, L, tile_q,
                     plan);
  return hipGetLastError();
}

hipError_t launch_scatter(const uint8_t* depth, int64_t n, const int32_t* offs,
                          int32_t* perm, hipStream_t s) {
  const int64_t nblk = (n + kLookupChunk - 1) / kLookupChunk;
  hipLaunchKernelGGL(k_scatter, dim3((unsigned)nblk), dim3(kLookupThreads), 0, s, depth, n,
                     offs, perm);
  return hipGetLastError();
}

hipError_t launch_bucketing_batch(BatchReq* reqs, int nreq, int64_t nblk, int max_depth,
                                  int tile_q, int64_t* total_tiles, hipStream_t s) {
  hipLaunchKernelGGL(k_lookup_batch, dim3((unsigned)nblk), dim3(kLookupThreads), 0, s, reqs, nreq,
                     max_depth);
  hipLaunchKernelGGL(k_scan_batch, dim3((unsigned)nreq), dim3(kScanThreads), 0, s, reqs, tile_q);
  hipLaunchKernelGGL(k_scatter_batch, dim3((unsigned)nblk), dim3(kLookupThreads), 0, s, reqs, nreq);
  hipLaunchKernelGGL(k_batch_tiles, dim3(1), dim3(64), 0, s, reqs, nreq, total_tiles);
  return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)blocks), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace sand
