// Host-side internals shared by the C ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/sand.h"
#include "sand_internal.h"

struct sand_model_s {
  int device = 0;
  int L = 0, W = 0, WP = 0;
  int act = 0;                // sand::Act
  int num_cu = 0;
  char* dev = nullptr;        // one allocation holding the three packed precisions
  size_t bytes = 0;
  sand::ModelArgs args[3];    // indexed by sand_precision
  // input-gradient data (same allocation): transposed chunks per precision,
  // omega_1 W_1 rows and the tail table
  const char* bwd[3] = {nullptr, nullptr, nullptr};
  // device copies of args[] (read per tile by batched launches)
  const sand::ModelArgs* args_dev[3] = {nullptr, nullptr, nullptr};
  const float* w1t = nullptr;
  const float* tails = nullptr;
};

struct sand_depthmap_s {
  sand_model model = nullptr;   // identity only: never dereferenced when freeing
  int device = 0;               // so the map can be freed after its model
  int R = 0;                    // dense: R; octree: 2^D
  uint8_t* depth = nullptr;   // device [R^3] (dense maps)
  float* far = nullptr;       // device [R^3] or null (dense maps)
  sand::OctreeArgs* oct = nullptr;   // device descriptor (octree maps)
  std::vector<void*> owned;          // octree arrays
};

namespace sand {

sand_status fail(sand_status st, const char* fmt, ...);
sand_status device_fail(hipError_t e, const char* what);

// Selects a device for the current thread and restores the previous one.
struct DeviceGuard {
  int prev = -1;
  bool ok = false;
  explicit DeviceGuard(int dev);
  ~DeviceGuard();
};

// Byte offsets of the per-query scratch regions.
struct WorkspaceLayout {
  size_t depth, perm, counts, plan, groups, qcount, total;
  int64_t nblk;
};
WorkspaceLayout workspace_layout(int64_t n);
size_t grad_stash_bytes(sand_model m, int prec);

sand_status check_query(const char* who, sand_model m, sand_depthmap dm, const float* xyz,
                        int64_t n, const void* out, const sand_query_opts& o);
// Lookup, histogram, scan and scatter (ADAPTIVE / FORCED). Far-field points
// get their value in sdf (if non-null) and a zero gradient in grad (if
// non-null). On return perm/plan describe the depth buckets.
sand_status run_bucketing(sand_model m, sand_depthmap dm, const float* xyz, int64_t n, float* sdf,
                          float* grad, const sand_query_opts& o, char* ws, hipStream_t s,
                          int tile_q, hipEvent_t* ev, const int32_t** perm, const Plan** plan);

// Optional HIP events recorded between the forward phases (any may be null):
// ev[0] before the lookup, ev[1] after it, ev[2] after the scan, ev[3] after
// the scatter, ev[4] after the T-MLP.
sand_status run_forward(sand_model m, sand_depthmap dm, const float* xyz, int64_t n, float* sdf,
                        const sand_query_opts& o, char* ws, hipStream_t s,
                        hipEvent_t* ev = nullptr);

}  // namespace sand
