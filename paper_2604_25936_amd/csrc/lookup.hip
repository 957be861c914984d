// Depth lookup and stable bucketing of query points by exit depth.
//
// Inference first reads every point's exit depth from the network-depth map
// (a dense grid or the sparse octree) and answers far-field points (depth
// 0) from the stored value (Sec. 3.4, Eq. 7); the remaining points are
// evaluated to their own depth. To run points of equal depth together, three
// steps build a permutation that groups point indices by depth, stable
// within each group:
//   1. k_lookup_count: per 4096-point chunk, depth per point (written as
//      uint8), far values written straight to the output, and a per-chunk
//      histogram built from wavefront ballots;
//   2. k_scan: one workgroup turns the per-chunk histograms into per-chunk
//      output offsets and writes the tile plan (deepest bucket first); large
//      queries first sum groups of chunks in parallel (k_group_sums), scan
//      the group sums, and expand them per chunk (k_group_offsets);
//   3. k_scatter: per chunk again, each point's rank among equal depths
//      (ballots + popcounts below the lane) gives its slot in the
//      permutation.
// Every thread takes four consecutive points per round, so a wavefront's
// coordinate loads cover 3 KB of contiguous memory in 16-byte pieces. With
// an octree, the first step resolves points through the tree's dense index
// only and queues the rest per chunk; k_oct_deferred descends those (one
// wavefront per chunk) and adds them to the chunk histograms before the
// scan, so no resolved point waits on another point's descent.
// Batched variants run the same bodies for several queries in one launch
// (each lookup block belongs to one query; one scan workgroup per query).

#include "sand_internal.h"

namespace sand {

namespace {


__device__ __forceinline__ int cell_index(float x, float s, int half) {
  // x * s is exact (s a power of two); clamp before the float->int step so
  // that out-of-cube points and NaN land in a border cell (NaN -> cell 0).
  float v = x * s;
  if (!(v >= -s)) v = -s;
  if (v > s - 1.0f) v = s - 1.0f;
  return (int)floorf(v) + half;
}

// Leaves of the octree holding P points: stored depth d and far value v
// of each. A point's cell at level D follows from the exact cell rule; its
// cell at every coarser level is that index shifted right. The descents run
// level by level together so that their loads overlap. At level l the word
// holding the parent's bit (level l-1) is already in hand; the parent's
// rank word and the word holding the child's bit are loaded together: the
// child's slot is 8 rank(parent) + child, and the child is internal when its
// bit is set (only below level D). A leaf's depth and value are loaded last.
// DEFER: points whose level-K cell is internal are not descended; their
// depth is set to kDeferred for a second pass (k_oct_deferred).
constexpr int kDeferred = 255;

// Bit i of v (v < 2^10) moved to bit 3i.
__device__ __forceinline__ uint32_t spread3(uint32_t v) {
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  return (v | (v << 2)) & 0x09249249u;
}

template <int P, bool DEFER = false>
__device__ __forceinline__ void octree_leaves(const OctreeArgs& o, const float (&x)[P],
                                              const float (&y)[P], const float (&z)[P],
                                              int (&d)[P], float (&v)[P]) {
  if (o.root_leaf) {
#pragma unroll
    for (int i = 0; i < P; ++i) {
      d[i] = 0;
      v[i] = o.root_value;
    }
    return;
  }
  const int D = o.D, half = 1 << (D - 1);
  const float s = (float)half;
  int ix[P], iy[P], iz[P];
  uint32_t p[P];      // code of the internal node holding the point (level l-1)
  uint64_t w[P];      // the bitmask word holding p's bit
  bool live[P];
  const int K = o.top_level;
#pragma unroll
  for (int i = 0; i < P; ++i) {
    ix[i] = cell_index(x[i], s, half);
    iy[i] = cell_index(y[i], s, half);
    iz[i] = cell_index(z[i], s, half);
    d[i] = 0;
    v[i] = __builtin_nanf("");
  }
  if (K > 0) {
    // the dense index of level K: the Morton code of the point's level-K cell
    // (the top K bits of each cell index, interleaved x, y, z from the top)
    uint2 e[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const int sh = D - K;
      const uint32_t code = (spread3((uint32_t)ix[i] >> sh) << 2) |
                            (spread3((uint32_t)iy[i] >> sh) << 1) | spread3((uint32_t)iz[i] >> sh);
      p[i] = code;
      e[i] = o.top[code];
    }
    const uint64_t* bitsK = o.bits[K];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      live[i] = e[i].x == kOctInternal;
      w[i] = 0;
      if (live[i]) {
        if constexpr (DEFER) d[i] = kDeferred;
        else w[i] = bitsK[p[i] >> 6];
      } else {
        d[i] = (int)e[i].x;
        v[i] = __uint_as_float(e[i].y);
      }
    }
    if constexpr (DEFER) return;
  } else {
    const uint64_t w0 = o.bits[0][0];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      p[i] = 0;
      w[i] = w0;
      live[i] = true;
    }
  }
  for (int l = K + 1; l <= D; ++l) {
    bool any = false;
#pragma unroll
    for (int i = 0; i < P; ++i) any |= live[i];
    if (!any) break;
    const int sh = D - l;
    const uint32_t* rank = o.rank[l - 1];
    const uint64_t* bits = l < D ? o.bits[l] : nullptr;
    uint32_t rk[P];
    uint64_t wn[P];
    uint32_t m[P];
#pragma unroll
    for (int i = 0; i < P; ++i) {
      const uint32_t child = (((ix[i] >> sh) & 1) << 2) | (((iy[i] >> sh) & 1) << 1) |
                             ((iz[i] >> sh) & 1);
      m[i] = 8u * p[i] + child;
      rk[i] = 0;
      wn[i] = 0;
      if (live[i]) {
        rk[i] = rank[p[i] >> 6];
        if (bits) wn[i] = bits[m[i] >> 6];
      }
    }
#pragma unroll
    for (int i = 0; i < P; ++i) {
      if (!live[i]) continue;
      const uint32_t r = rk[i] + (uint32_t)__popcll(w[i] & ((1ull << (p[i] & 63)) - 1ull));
      const uint32_t slot = 8u * r + (m[i] & 7u);
      if ((wn[i] >> (m[i] & 63)) & 1ull) {
        p[i] = m[i];
        w[i] = wn[i];
      } else {
        d[i] = o.depth[l][slot];
        v[i] = o.value[l][slot];
        live[i] = false;
      }
    }
  }
}

__device__ __forceinline__ uint64_t lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Add the wavefront's points (P per lane) to hist[depth]: one LDS atomic per
// distinct depth present in the wavefront, whatever slot it occurs in.
template <int P>
__device__ __forceinline__ void wave_histogram_n(const int (&d)[P], const bool (&valid)[P],
                                                 int* hist) {
  const int lane = threadIdx.x & 63;
  bool todo[P];
#pragma unroll
  for (int j = 0; j < P; ++j) todo[j] = valid[j];
  for (;;) {
    bool mine_any = false;
    int mine = 0;
#pragma unroll
    for (int j = P - 1; j >= 0; --j)
      if (todo[j]) {
        mine_any = true;
        mine = d[j];
      }
    const uint64_t any = __ballot(mine_any);
    if (!any) break;
    const int leader = __ffsll((unsigned long long)any) - 1;
    const int v = __shfl(mine, leader);
    int total = 0;
#pragma unroll
    for (int j = 0; j < P; ++j) {
      const bool hit = valid[j] && d[j] == v;
      total += __popcll(__ballot(hit));
      if (hit) todo[j] = false;
    }
    if (lane == leader) atomicAdd(&hist[v], total);
  }
}

// Body of one lookup block: points [blk*4096, blk*4096 + 4096) of one query.
// Each thread takes kPP consecutive points per round, kQuadRounds rounds; a
// wavefront's round covers 3 KB of contiguous coordinates, read with 16-byte
// loads (all rounds' loads are issued before any point is looked up).
constexpr int kPP = 4;
constexpr int kQuadRounds = kLookupChunk / (kLookupThreads * kPP);

// OCT = false: a dense map only (oct is ignored), so the octree descent's
// registers do not limit the occupancy of the dense-map lookup.
template <bool DEFER, bool OCT = true>
__device__ __forceinline__ void lookup_block(
    int64_t blk, const float* __restrict__ xyz, int64_t n, const uint8_t* __restrict__ map,
    int R, const float* __restrict__ far, const OctreeArgs* __restrict__ oct,
    const uint8_t* __restrict__ forced, int mode, int L, int max_depth,
    uint8_t* __restrict__ depth, float* __restrict__ sdf, float* __restrict__ grad,
    int32_t* __restrict__ counts, int32_t* __restrict__ queue, int32_t* __restrict__ qcount) {
  __shared__ int hist[kBuckets];
  __shared__ int nq;
  const int t = threadIdx.x;
  if (t < kBuckets) hist[t] = 0;
  if (t == 0) nq = 0;
  const int64_t base = blk * kLookupChunk;
  const int half = R >> 1;
  const float s = (float)half;
  const bool vec_in = ((uintptr_t)xyz & 15) == 0;
  const bool vec_depth = ((uintptr_t)depth & 3) == 0;
  const bool vec_sdf = ((uintptr_t)sdf & 15) == 0;
  // coordinates of PIPE rounds in flight: all of them with an octree; two
  // for a dense map, the next but one loaded as each round is taken (fewer
  // registers, more wavefronts per SIMD)
  constexpr int PIPE = OCT ? kQuadRounds : 2;
  float pt[PIPE][3 * kPP];
  auto load_round = [&](int r, float (&dst)[3 * kPP]) {
    const int64_t q0 = base + ((int64_t)r * kLookupThreads + t) * kPP;
    if (vec_in && q0 + kPP <= n) {
      const float4* src = (const float4*)(xyz + 3 * q0);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float4 f = src[k];
        dst[4 * k] = f.x;
        dst[4 * k + 1] = f.y;
        dst[4 * k + 2] = f.z;
        dst[4 * k + 3] = f.w;
      }
    } else {
#pragma unroll
      for (int k = 0; k < 3 * kPP; ++k) dst[k] = 3 * q0 + k < 3 * n ? xyz[3 * q0 + k] : 0.0f;
    }
  };
#pragma unroll
  for (int r = 0; r < PIPE; ++r) load_round(r, pt[r]);
  __syncthreads();   // hist cleared
#pragma unroll
  for (int r = 0; r < kQuadRounds; ++r) {
    const int64_t q0 = base + ((int64_t)r * kLookupThreads + t) * kPP;
    float x[kPP], y[kPP], z[kPP], farv[kPP];
    int d[kPP], cell[kPP];
#pragma unroll
    for (int i = 0; i < kPP; ++i) {
      x[i] = pt[r % PIPE][3 * i];
      y[i] = pt[r % PIPE][3 * i + 1];
      z[i] = pt[r % PIPE][3 * i + 2];
      cell[i] = -1;
      farv[i] = __builtin_nanf("");
      d[i] = 0;
    }
    if (r + PIPE < kQuadRounds) load_round(r + PIPE, pt[r % PIPE]);
    // the map's depth (and, for an octree, the leaf's value) of every point;
    // FORCED mode keeps the map's far value for points forced to depth 0
    if (OCT && oct != nullptr) {
      if (DEFER)
        octree_leaves<kPP, true>(*oct, x, y, z, d, farv);
      else if (mode != 1)
        octree_leaves<kPP>(*oct, x, y, z, d, farv);
    } else if (map != nullptr) {
#pragma unroll
      for (int i = 0; i < kPP; ++i)
        cell[i] = (cell_index(x[i], s, half) * R + cell_index(y[i], s, half)) * R +
                  cell_index(z[i], s, half);
      if (mode == 0) {
#pragma unroll
        for (int i = 0; i < kPP; ++i) d[i] = map[cell[i]];
      }
    }
    if (mode == 1) {
#pragma unroll
      for (int i = 0; i < kPP; ++i) d[i] = L;
    } else if (mode == 2) {
#pragma unroll
      for (int i = 0; i < kPP; ++i) {
        const int dd = q0 + i < n ? forced[q0 + i] : 0;
        d[i] = dd > L ? L : dd;
      }
    }
    // points left for the octree's second pass: queued, kept out of this
    // pass's histogram, their depth byte written there
    bool deferred[kPP];
#pragma unroll
    for (int i = 0; i < kPP; ++i) deferred[i] = DEFER && d[i] == kDeferred && q0 + i < n;
    if constexpr (DEFER) {
      const int lane = t & 63;
      uint64_t m[kPP];
      int tot = 0;
#pragma unroll
      for (int i = 0; i < kPP; ++i) {
        m[i] = __ballot(deferred[i]);
        tot += __popcll(m[i]);
      }
      if (tot > 0) {
        // the chunk's own stretch of the queue: no global atomics
        int qb = 0;
        if (lane == 0) qb = atomicAdd(&nq, tot);
        qb = __shfl(qb, 0);
        const uint64_t below = lane == 0 ? 0ull : (~0ull >> (64 - lane));
        int32_t* cq = queue + base;
#pragma unroll
        for (int i = 0; i < kPP; ++i) {
          if (deferred[i]) cq[qb + __popcll(m[i] & below)] = (int32_t)(q0 + i);
          qb += __popcll(m[i]);
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kPP; ++i) {
      if (!deferred[i] && max_depth > 0 && d[i] > max_depth) d[i] = max_depth;
      if (q0 + i >= n) d[i] = 0;
      if (d[i] == 0 && oct == nullptr && far != nullptr && cell[i] >= 0) farv[i] = far[cell[i]];
    }
    // whole quads are written with one store each where the pointers allow
    const bool full = q0 + kPP <= n;
    if (full && vec_depth) {
      *(uint32_t*)(depth + q0) = (uint32_t)d[0] | ((uint32_t)d[1] << 8) |
                                 ((uint32_t)d[2] << 16) | ((uint32_t)d[3] << 24);
    } else {
#pragma unroll
      for (int i = 0; i < kPP; ++i)
        if (q0 + i < n) depth[q0 + i] = (uint8_t)d[i];
    }
    if (sdf) {
      if (full && vec_sdf && d[0] == 0 && d[1] == 0 && d[2] == 0 && d[3] == 0) {
        *(float4*)(sdf + q0) = make_float4(farv[0], farv[1], farv[2], farv[3]);
      } else {
#pragma unroll
        for (int i = 0; i < kPP; ++i)
          if (q0 + i < n && d[i] == 0) sdf[q0 + i] = farv[i];
      }
    }
    bool valid[kPP];
#pragma unroll
    for (int i = 0; i < kPP; ++i) {
      const int64_t q = q0 + i;
      valid[i] = q < n && !deferred[i];
      if (valid[i] && d[i] == 0 && grad) grad[3 * q] = grad[3 * q + 1] = grad[3 * q + 2] = 0.0f;
    }
    wave_histogram_n<kPP>(d, valid, hist);
  }
  __syncthreads();
  if (t < kBuckets) counts[blk * kBuckets + t] = hist[t];
  if (DEFER && t == 0) qcount[blk] = nq;
}

// DEFER: the octree's two-pass adaptive lookup (first pass)
template <bool DEFER, bool OCT>
__global__ __launch_bounds__(kLookupThreads) void k_lookup_count(
    const float* __restrict__ xyz, int64_t n, const uint8_t* __restrict__ map,
    int R, const float* __restrict__ far, const OctreeArgs* __restrict__ oct,
    const uint8_t* __restrict__ forced, int mode, int L, int max_depth,
    uint8_t* __restrict__ depth, float* __restrict__ sdf, float* __restrict__ grad,
    int32_t* __restrict__ counts, int32_t* __restrict__ queue, int32_t* __restrict__ qcount) {
  lookup_block<DEFER, OCT>(blockIdx.x, xyz, n, map, R, far, oct, forced, mode, L, max_depth, depth,
                      sdf, grad, counts, queue, qcount);
}

constexpr int kScanThreads = 1024;

// One workgroup: per-chunk histograms -> per-chunk bucket offsets (in
// place) and the tile plan. Bucket d >= 1 occupies perm slots
// [start[d], start[d] + count[d]); depth-0 points are not in the permutation.
// Thread t owns a contiguous range of chunks: it sums them, the per-bucket
// exclusive prefix over threads comes from a wavefront scan (shuffles) and a
// scan of the sixteen wavefront totals, and the thread then rewrites its
// chunks' counts as running offsets.
__device__ __forceinline__ void scan_body(int32_t* __restrict__ counts, int64_t nblk, int L,
                                          int tile_q, Plan* __restrict__ plan) {
  constexpr int NWAVE = kScanThreads / 64;
  __shared__ int64_t wtot[NWAVE][kBuckets];
  __shared__ int64_t start[kBuckets];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t per = (nblk + kScanThreads - 1) / kScanThreads;
  const int64_t b0 = t * per < nblk ? t * per : nblk;
  const int64_t b1 = b0 + per < nblk ? b0 + per : nblk;
  int64_t sum[kBuckets];
#pragma unroll
  for (int d = 0; d < kBuckets; ++d) sum[d] = 0;
  int64_t b = b0;
  for (; b + 4 <= b1; b += 4) {
    int32_t c[4][kBuckets];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int d = 0; d < kBuckets; ++d) c[k][d] = counts[(b + k) * kBuckets + d];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
      for (int d = 0; d < kBuckets; ++d) sum[d] += c[k][d];
  }
  for (; b < b1; ++b)
#pragma unroll
    for (int d = 0; d < kBuckets; ++d) sum[d] += counts[b * kBuckets + d];
  // inclusive scan over the wavefront's lanes, bucket by bucket
  int64_t incl[kBuckets];
#pragma unroll
  for (int d = 0; d < kBuckets; ++d) {
    int64_t v = sum[d];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const int64_t u = __shfl_up(v, off);
      if (lane >= off) v += u;
    }
    incl[d] = v;
  }
  if (lane == 63)
#pragma unroll
    for (int d = 0; d < kBuckets; ++d) wtot[w][d] = incl[d];
  __syncthreads();
  if (t < kBuckets) {
    int64_t run = 0;
    for (int k = 0; k < NWAVE; ++k) {
      const int64_t v = wtot[k][t];
      wtot[k][t] = run;
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
#pragma unroll
  for (int d = 0; d < kBuckets; ++d) run[d] = start[d] + wtot[w][d] + incl[d] - sum[d];
  // bucket 0 is not in the permutation: its entry keeps the chunk's count of
  // far-field points, which lets the scatter skip chunks without others
  for (b = b0; b < b1; ++b)
#pragma unroll
    for (int d = 1; d < kBuckets; ++d) {
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

// Large queries scan in three launches: per-group sums of kScanGroup
// chunks (many workgroups), the scan of the group sums (one workgroup, as
// above), then each group's chunk offsets from its group offset.
__global__ __launch_bounds__(64) void k_group_sums(const int32_t* __restrict__ counts,
                                                   int64_t nblk, int32_t* __restrict__ groups) {
  const int d = threadIdx.x;
  if (d >= kBuckets) return;
  const int64_t b0 = (int64_t)blockIdx.x * kScanGroup;
  const int64_t b1 = b0 + kScanGroup < nblk ? b0 + kScanGroup : nblk;
  int32_t sum = 0;
  for (int64_t b = b0; b < b1; ++b) sum += counts[b * kBuckets + d];
  groups[(int64_t)blockIdx.x * kBuckets + d] = sum;
}

__global__ __launch_bounds__(64) void k_group_offsets(int32_t* __restrict__ counts, int64_t nblk,
                                                      const int32_t* __restrict__ groups) {
  const int d = threadIdx.x;
  if (d < 1 || d >= kBuckets) return;   // bucket 0 keeps the far-field counts
  const int64_t b0 = (int64_t)blockIdx.x * kScanGroup;
  const int64_t b1 = b0 + kScanGroup < nblk ? b0 + kScanGroup : nblk;
  int32_t c[kScanGroup];
#pragma unroll
  for (int k = 0; k < kScanGroup; ++k) c[k] = b0 + k < b1 ? counts[(b0 + k) * kBuckets + d] : 0;
  int32_t run = groups[(int64_t)blockIdx.x * kBuckets + d];
#pragma unroll
  for (int k = 0; k < kScanGroup; ++k)
    if (b0 + k < b1) {
      counts[(b0 + k) * kBuckets + d] = run;
      run += c[k];
    }
}

// Scatter of one lookup block's points into the permutation, stable within
// each depth bucket. A thread takes kPP consecutive points per round. Within
// a wavefront a point's rank among equal depths is the count of such points
// in lower lanes (one ballot per slot) plus those in its own lane's earlier
// slots; the per-(round, wavefront) bucket counts are then turned into
// offsets by one pass over the block, in point order.
__device__ __forceinline__ void scatter_block(int64_t blk, const uint8_t* __restrict__ depth,
                                              int64_t n, const int32_t* __restrict__ offs,
                                              int32_t* __restrict__ perm) {
  constexpr int NWV = kLookupThreads / 64;
  __shared__ int wcnt[kQuadRounds][NWV][kBuckets];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t base = blk * kLookupChunk;
  // offs[.][0] holds the chunk's far-field count: nothing to place if all are far
  const int64_t in_chunk = n - base < kLookupChunk ? n - base : kLookupChunk;
  if (offs[blk * kBuckets] >= in_chunk) return;
  for (int i = t; i < kQuadRounds * NWV * kBuckets; i += kLookupThreads) (&wcnt[0][0][0])[i] = 0;
  const bool vec = ((uintptr_t)depth & 3) == 0;
  int d[kQuadRounds][kPP], rank[kQuadRounds][kPP];
#pragma unroll
  for (int r = 0; r < kQuadRounds; ++r) {
    const int64_t q0 = base + ((int64_t)r * kLookupThreads + t) * kPP;
    if (vec && q0 + kPP <= n) {
      const uint32_t v = *(const uint32_t*)(depth + q0);
#pragma unroll
      for (int j = 0; j < kPP; ++j) d[r][j] = (v >> (8 * j)) & 0xff;
    } else {
#pragma unroll
      for (int j = 0; j < kPP; ++j) d[r][j] = q0 + j < n ? depth[q0 + j] : 0;
    }
  }
  __syncthreads();   // wcnt cleared
  const uint64_t lt = lanemask_lt();
#pragma unroll
  for (int r = 0; r < kQuadRounds; ++r) {
    bool todo[kPP];
#pragma unroll
    for (int j = 0; j < kPP; ++j) {
      todo[j] = d[r][j] > 0;   // invalid points read as depth 0
      rank[r][j] = 0;
    }
    for (;;) {
      bool mine_any = false;
      int mine = 0;
#pragma unroll
      for (int j = kPP - 1; j >= 0; --j)
        if (todo[j]) {
          mine_any = true;
          mine = d[r][j];
        }
      const uint64_t any = __ballot(mine_any);
      if (!any) break;
      const int leader = __ffsll((unsigned long long)any) - 1;
      const int v = __shfl(mine, leader);
      int below = 0, total = 0, own = 0;
#pragma unroll
      for (int j = 0; j < kPP; ++j) {
        const uint64_t m = __ballot(d[r][j] == v);
        below += __popcll(m & lt);
        total += __popcll(m);
      }
#pragma unroll
      for (int j = 0; j < kPP; ++j)
        if (d[r][j] == v) {
          rank[r][j] = below + own;
          ++own;
          todo[j] = false;
        }
      if (lane == leader) wcnt[r][w][v] = total;
    }
  }
  __syncthreads();
  if (t < kBuckets) {
    int run = offs[blk * kBuckets + t];
    for (int r = 0; r < kQuadRounds; ++r)
      for (int k = 0; k < NWV; ++k) {
        const int c = wcnt[r][k][t];
        wcnt[r][k][t] = run;
        run += c;
      }
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kQuadRounds; ++r) {
    const int64_t q0 = base + ((int64_t)r * kLookupThreads + t) * kPP;
#pragma unroll
    for (int j = 0; j < kPP; ++j)
      if (d[r][j] > 0) perm[wcnt[r][w][d[r][j]] + rank[r][j]] = (int32_t)(q0 + j);
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
  lookup_block<false>((int64_t)blockIdx.x - q.blk0, q.xyz, q.n, q.map, q.R, q.far, q.oct, nullptr, 0,
               q.L, max_depth, q.depth, q.sdf, nullptr, q.counts, nullptr, nullptr);
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

// Second pass of an octree lookup: the points whose level-K cell is
// internal, queued per 4096-point chunk (qcount[c] of them at queue + 4096 c),
// one thread each, descend from the root (no resolved point waits for
// them); one wavefront per chunk. Writes their depth, far value and zero
// gradient, and adds them to their chunk's histogram with one atomic per
// distinct depth of a wavefront.
__global__ __launch_bounds__(64) void k_oct_deferred(
    const float* __restrict__ xyz, const OctreeArgs* __restrict__ oct, int max_depth,
    const int32_t* __restrict__ queue, const int32_t* __restrict__ qcount,
    uint8_t* __restrict__ depth, float* __restrict__ sdf, float* __restrict__ grad,
    int32_t* __restrict__ counts) {
  const int lane = threadIdx.x;
  const int64_t c = blockIdx.x;
  const int cnt = qcount[c];
  for (int b0 = 0; b0 < cnt; b0 += 64) {
    const int idx = b0 + (int)threadIdx.x;
    const bool active = idx < cnt;
    int d1 = -1;
    if (active) {
      const int64_t q = queue[c * kLookupChunk + idx];
      float x[1] = {xyz[3 * q]}, y[1] = {xyz[3 * q + 1]}, z[1] = {xyz[3 * q + 2]}, v[1];
      int d[1];
      octree_leaves<1>(*oct, x, y, z, d, v);
      if (max_depth > 0 && d[0] > max_depth) d[0] = max_depth;
      depth[q] = (uint8_t)d[0];
      if (d[0] == 0) {
        if (sdf) sdf[q] = v[0];
        if (grad) grad[3 * q] = grad[3 * q + 1] = grad[3 * q + 2] = 0.0f;
      }
      d1 = d[0];
    }
    uint64_t todo = __ballot(active);
    while (todo) {
      const int lead = __ffsll((long long)todo) - 1;
      const int ld = __shfl(d1, lead);
      const uint64_t same = __ballot(active && d1 == ld);
      if (lane == lead) atomicAdd(&counts[c * kBuckets + ld], __popcll(same));
      todo &= ~same;
    }
  }
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
                               float* grad, int32_t* counts, int32_t* queue, int32_t* qcount,
                               hipStream_t s) {
  const int64_t nblk = (n + kLookupChunk - 1) / kLookupChunk;
  const bool two_pass = oct != nullptr && mode == 0 && queue != nullptr && qcount != nullptr;
  if (two_pass)
    hipLaunchKernelGGL((k_lookup_count<true, true>), dim3((unsigned)nblk), dim3(kLookupThreads), 0,
                       s, xyz, n, map, R, far, oct, forced, mode, L, max_depth, depth, sdf, grad,
                       counts, queue, qcount);
  else if (oct != nullptr)
    hipLaunchKernelGGL((k_lookup_count<false, true>), dim3((unsigned)nblk), dim3(kLookupThreads), 0,
                       s, xyz, n, map, R, far, oct, forced, mode, L, max_depth, depth, sdf, grad,
                       counts, nullptr, nullptr);
  else
    hipLaunchKernelGGL((k_lookup_count<false, false>), dim3((unsigned)nblk), dim3(kLookupThreads),
                       0, s, xyz, n, map, R, far, nullptr, forced, mode, L, max_depth, depth, sdf,
                       grad, counts, nullptr, nullptr);
  if (two_pass) {
    hipLaunchKernelGGL(k_oct_deferred, dim3((unsigned)nblk), dim3(64), 0, s, xyz, oct,
                       max_depth, queue, qcount, depth, sdf, grad, counts);
  }
  return hipGetLastError();
}

hipError_t launch_scan(int32_t* counts, int64_t nblk, int L, int tile_q, Plan* plan,
                       int32_t* groups, hipStream_t s) {
  if (nblk <= kScanThreads) {
    hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, counts, nblk, L, tile_q,
                       plan);
    return hipGetLastError();
  }
  const int64_t ngrp = (nblk + kScanGroup - 1) / kScanGroup;
  hipLaunchKernelGGL(k_group_sums, dim3((unsigned)ngrp), dim3(64), 0, s, counts, nblk, groups);
  hipLaunchKernelGGL(k_scan, dim3(1), dim3(kScanThreads), 0, s, groups, ngrp, L, tile_q, plan);
  hipLaunchKernelGGL(k_group_offsets, dim3((unsigned)ngrp), dim3(64), 0, s, counts, nblk,
                     groups);
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
