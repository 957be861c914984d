// Internal declarations shared by the host library and the gfx950 kernels.
//
// Packed model layout on the device (built once by sand_load_model):
//
//   The hidden width W is padded to WP (64, 128, 256 or 352) with zero rows
//   and columns, and the output units of every layer are cut into blocks of
//   BM units (BM = 16 for FP32, 32 for BF16/FP16). Each (layer, block) pair
//   is one "chunk": the MFMA A-operand tiles of that block in exactly the
//   per-lane order the kernel reads them, followed by the block's FP32 tail
//   weights: a0[BM], a1[BM] in unit order for FP32 (128 B); for BF16/FP16
//   a0[64], a1[64] indexed by lane, lane l holding the weight of the unit in
//   its accumulator register l & 15 (row 8 ((l & 15) / 4) + 4 (l / 32) +
//   l % 4 of the block), 512 B:
//
//     layer 1, FP32 path (16x16x4 FP32 MFMA, K = 4 = x, y, z, bias):
//        float A[1 step][64 lanes], then tails             256 + 128 B
//     layer 1, BF16/FP16 path (32x32x16 BF16 MFMA, 2 K steps, on three-way
//     BF16 splits of the weights and coordinates: lane half h of step s
//     holds the six products of coordinate 2s + h and bias parts):
//        u16 A[2 steps][64 lanes][8], then tails          2048 + 512 B
//     layer j >= 2, FP32 (16x16x4 MFMA, WP/4 K steps + 1 bias step):
//        float A[WP/4 + 1][64 lanes], then tails
//     layer j >= 2, BF16/FP16 (32x32x16 MFMA, WP/16 K steps + 1 bias step):
//        u16   A[WP/16 + 1][64 lanes][8], then tails
//
//   Weights and biases are pre-multiplied by omega_j / (2 pi) so that one
//   hardware sine in revolutions gives sin(omega_j (W h + b)). The K order of
//   layer j's weights is permuted so that the accumulator registers of
//   layer j-1 are, as they stand, the B operand of layer j (activations
//   never leave registers). A linear tail is stored as a0 = a, a1 = 0 with
//   c0 = c, c1 = 1, so every tail is evaluated as (a0.h + c0)(a1.h + c1).
#pragma once

#include <stdint.h>
#include <hip/hip_runtime.h>

namespace sand {

constexpr int kMaxLayers = 16;
constexpr int kMaxWidth = 352;
constexpr int kBuckets = kMaxLayers + 1;   // exit depths 0..16
constexpr int kLookupThreads = 256;
constexpr int kLookupChunk = 4096;         // points per lookup block
constexpr int kScanGroup = 32;             // lookup blocks per group of the large-query scan
constexpr double kTwoPi = 6.283185307179586476925286766559;

enum Prec { PREC_FP32 = 0, PREC_BF16 = 1, PREC_FP16 = 2 };

// Activation of the hidden layers (the model blob's header byte 48): the
// SIREN sine sin(omega z) or the FINER variable-periodic sine
// sin(omega (|z| + 1) z), z = W h + b (the two backbones of Sec. 4.1).
enum Act { ACT_SINE = 0, ACT_FINER = 1 };

// Padded widths the kernels are built for.
inline int padded_width(int W) {
  if (W <= 64) return 64;
  if (W <= 128) return 128;
  if (W <= 256) return 256;
  return 352;
}


// Device-side description of a packed model for one precision.
struct ModelArgs {
  const char* chunks;      // layer-1 chunks, then hidden chunks (layer-major)
  int L;                   // hidden layers
  int WP;                  // padded width
  size_t chunk_bytes;      // bytes of one hidden chunk
  float c0[kMaxLayers];    // tail bias of the first factor
  float c1[kMaxLayers];    // tail bias of the second factor (1 for linear)
  uint32_t lin_mask;       // bit j: tail j+1 is linear (second factor a1 = 0, c1 = 1)
  int act;                 // Act
  float kf[2];             // 2 pi / omega of layer 1 and of layers 2..L (FINER's |z| = |u| kf
                           // for the omega / (2 pi)-scaled accumulator u)
};

// Sparse network-depth octree (Sec. 3.2), pointer-free. Node codes are
// Morton codes (x, y, z bits interleaved, x most significant per level);
// the children of internal node p are 8p + (a << 2 | b << 1 | c). Level l
// (0..D-1) keeps a bitmask of its internal nodes over all 8^l codes and the
// exclusive popcount prefix of each 64-bit word; child slot
// 8 rank_l(p) + child of level l+1 holds that child's leaf payload:
// depth 0 with the stored far value, 1..L for a near leaf (level D only),
// 255 for an internal child.
constexpr int kMaxOctDepth = 10;
struct OctreeArgs {
  int D;
  int root_leaf;                            // 1: the root is the only leaf
  float root_value;                         // its far value
  int pad;
  const uint64_t* bits[kMaxOctDepth];       // level l = 0..D-1
  const uint32_t* rank[kMaxOctDepth];
  const uint8_t* depth[kMaxOctDepth + 1];   // level l = 1..D, per child slot
  const float* value[kMaxOctDepth + 1];
  // Dense index of level top_level (< D), Morton order: per cell the depth
  // and value bits of the leaf holding it when that leaf is at a level <=
  // top_level, else x = kOctInternal (descend on from top_level + 1).
  int top_level;                            // 0: no index
  int pad2;
  const uint2* top;
};
constexpr uint32_t kOctInternal = 0xffffffffu;

// Bucketed work plan written on the device by the scan kernel.
struct Plan {
  int64_t start[kBuckets];      // first perm slot of depth bucket d
  int64_t count[kBuckets];      // points in bucket d
  int64_t tile_end[kBuckets + 1];  // tiles of depths >= d (tile_end[L+1] = 0):
                                   // depth d owns [tile_end[d+1], tile_end[d])
  int64_t total_tiles;
  int32_t tile_q;               // points per tile the plan was cut for
  int32_t pad;
};

// Compaction of map-free dynamic exit: points still running after layer
// `layer` leave their tile as records (point index, y, the packed layer
// output) in `arena`, and a second launch runs them on from layer + 1 in
// full tiles. Record r occupies dyn_record_bytes() bytes at arena + r * that.
struct DynSpill {
  char* arena;
  int* count;              // records written by the spilling launch
  int64_t cap;             // records the arena holds
  int layer;               // 0: no compaction
};

// Everything one forward launch needs.
struct QueryArgs {
  ModelArgs m;
  const float* xyz;        // [n][3]
  float* sdf;              // [n]
  const int32_t* perm;     // bucketed point order, or null (FULL mode)
  const Plan* plan;        // device plan, or null (FULL mode)
  int64_t n;
  int full_depth;          // FULL mode: the depth every point runs to
  float* y_all;            // [n][L] every accumulated output y_1..y_d, or null
  float dyn_r;             // > 0: map-free early exit on |t_j| < dyn_r (j >= 2)
  uint8_t* depth_out;      // [n] exit depths (written when dyn_r > 0), or null
  DynSpill spill;          // dynamic mode: spill after spill.layer (0: none)
};

// One query of a batched launch (server). Pointers are device memory; the
// lookup/scan kernels fill plan and tile0.
struct BatchReq {
  const float* xyz;        // [n][3]
  float* sdf;              // [n]
  uint8_t* depth;          // [n] scratch
  int32_t* perm;           // [n] scratch
  int32_t* counts;         // [ceil(n/4096)][kBuckets] scratch
  const uint8_t* map;      // R^3 depth map, or null for an octree map
  const float* far;        // R^3 far values or null
  const OctreeArgs* oct;   // octree map (device), or null
  const ModelArgs* model;  // device copy of the model's arguments
  int64_t n;
  int64_t blk0;            // first lookup block of this query in the launch
  int64_t tile0;           // first T-MLP tile of this query (device-filled)
  int R;
  int L;
  Plan plan;               // device-filled
};

// Everything one batched T-MLP launch needs.
struct BatchArgs {
  const BatchReq* reqs;
  int nreq;
  const int64_t* total_tiles;   // device-filled by the bucketing launch
};

// Everything one input-gradient launch needs.
struct AdjointArgs {
  QueryArgs q;             // forward chunks, points, optional sdf out, plan
  const char* bwd;         // transposed-weight chunks of layers 2..L
  const float* w1t;        // [WP][4]: omega_1 * W_1[u][0..2], 0
  const float* tails;      // [L][2][WP]: a0, a1 of every layer
  const float* dy;         // [n] upstream gradient or null (ones)
  float* grad;             // [n][3]
  char* stash;             // per-workgroup cosine stash
  size_t stash_wg;         // stash bytes per workgroup
  uint32_t* next_tile;     // tile counter, zero at launch (tiles are drawn one at a time)
};

// ---- launchers (defined in the .hip files) ----
// queue [n] and qcount [ceil(n / kLookupChunk)]: scratch of the octree's
// two-pass adaptive lookup (points below the dense index are queued per
// chunk and descended in a second kernel), or null
hipError_t launch_lookup_count(const float* xyz, int64_t n, const uint8_t* map,
                               int R, const float* far, const OctreeArgs* oct,
                               const uint8_t* forced,
                               int mode, int L, int max_depth, uint8_t* depth,
                               float* sdf, float* grad, int32_t* counts, int32_t* queue,
                               int32_t* qcount, hipStream_t s);
// groups: scratch of ceil(nblk / kScanGroup) * kBuckets int32, used when
// nblk exceeds one scan workgroup's threads
hipError_t launch_scan(int32_t* counts, int64_t nblk, int L, int tile_q,
                       Plan* plan, int32_t* groups, hipStream_t s);
hipError_t launch_scatter(const uint8_t* depth, int64_t n, const int32_t* offs,
                          int32_t* perm, hipStream_t s);
hipError_t launch_fill_u8(uint8_t* p, int64_t n, uint8_t v, hipStream_t s);
hipError_t launch_bucketing_batch(BatchReq* reqs, int nreq, int64_t nblk, int max_depth,
                                  int tile_q, int64_t* total_tiles, hipStream_t s);
hipError_t launch_tmlp_batch(int prec, int WP, int act, const BatchArgs& a, int num_cu,
                             hipStream_t s);
// The forward kernels of one activation (tmlp_sine.hip, tmlp_finer.hip):
// what = 0 a query (q), 1 the resumed launch of compacted dynamic exit (q),
// 2 a batch (b).
template <int ACT>
hipError_t launch_tmlp_act(int what, int prec, int WP, const QueryArgs* q, const BatchArgs* b,
                           int num_cu, hipStream_t s);

// network-depth map construction (mapbuild.hip)
hipError_t launch_map_list(const uint8_t* near, int64_t cells, int32_t* list, uint32_t* count,
                           hipStream_t s);
hipError_t launch_map_samples(const int32_t* list, int64_t first, int64_t nsamp, int R, int sps,
                              float* xyz, hipStream_t s);
hipError_t launch_map_pool(const float* y_all, int L, const int32_t* list, int64_t first,
                           int64_t nsamp, int sps, float r, uint32_t* depth32, hipStream_t s);
hipError_t launch_map_finish(const uint8_t* near, const float* center_sdf, const uint32_t* depth32,
                             int64_t cells, uint8_t* depth, float* far, hipStream_t s);

// sparse octree construction (octree.hip)
hipError_t launch_oct_centres(const uint64_t* parents, int64_t first, int64_t nslots, int level,
                              float* xyz, hipStream_t s);
hipError_t launch_oct_classify(const uint64_t* parents, const float* y, int64_t first,
                               int64_t nslots, int level, int D, float h, uint64_t* bits,
                               uint8_t* depth, float* value, int32_t* near_slots,
                               uint32_t* near_count, hipStream_t s);
hipError_t launch_oct_rank(const uint64_t* bits, int64_t words, uint32_t* rank, int64_t* total,
                           hipStream_t s);
hipError_t launch_oct_list(const uint64_t* bits, const uint32_t* rank, int64_t words,
                           uint64_t* list, hipStream_t s);
hipError_t launch_oct_samples(const int32_t* near_slots, const uint64_t* parents, int64_t first,
                              int64_t nsamp, int D, int sps, float* xyz, hipStream_t s);
// Fill the dense top index of an octree (8^K cells of level K).
hipError_t launch_oct_top(const OctreeArgs& oa, int K, uint2* top, hipStream_t s);
hipError_t launch_oct_finish(const int32_t* near_slots, int64_t nnear, const uint32_t* depth32,
                             uint8_t* depth, hipStream_t s);

int tmlp_tile_points(int prec, int WP);   // forward tile (the plan's tile_q for sand_query)
int adjoint_tile_points(int prec);   // adjoint tile (the plan's tile_q for sand_query_grad)
size_t adjoint_stash_bytes_per_wg(int prec, int WP, int L);
hipError_t launch_adjoint(int prec, const AdjointArgs& a, int grid, hipStream_t s);
// The input-gradient kernel of one activation (adjoint_sine.hip, adjoint_finer.hip).
template <int ACT>
hipError_t launch_adjoint_act(int prec, const AdjointArgs& a, int grid, hipStream_t s);
hipError_t launch_tmlp(int prec, const QueryArgs& a, int num_cu, hipStream_t s);
// Second launch of compacted dynamic exit: the records of a.spill, from
// layer a.spill.layer + 1 on (a.xyz unused; a.sdf/a.depth_out indexed as in
// the spilling launch).
hipError_t launch_tmlp_resume(int prec, const QueryArgs& a, int num_cu, hipStream_t s);
int dyn_record_bytes(int prec, int WP);
// out[i] = xyz[i * stride] for i < n (float3 points).
hipError_t launch_gather_points(const float* xyz, int64_t stride, int64_t n, float* out,
                                hipStream_t s);

}  // namespace sand
