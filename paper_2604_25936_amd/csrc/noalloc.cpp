// sand_query_noalloc: sand_query for callers that cannot allocate device
// memory (code under HIP graph capture, tight serving loops, harnesses that
// forbid hipMalloc). The per-query scratch that sand_query allocates (or
// takes as opts.workspace: exit depths, the bucketed permutation, chunk
// histograms, the tile plan, scan sums and octree queue lengths) lives here
// in one file-scope device array of kScratchBytes, of which every GPU the
// library runs on holds its own copy until the process ends. The kernels are
// sand_query's own.
//
// Every call on a GPU shares that GPU's copy and finds the last call's
// contents in it; the kernels overwrite what they read (no region has to
// start at zero), but two calls that overlap in time on one GPU, on any
// streams, race on it: the caller orders them.

#include <mutex>

#include "sand_host.h"

using namespace sand;

namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;   // 64 MiB: up to 13,373,120 points
constexpr int kMaxDevices = 64;

static __device__ __align__(256) char scratch[kScratchBytes];

std::mutex g_mu;
char* g_scratch[kMaxDevices] = {};

// Device address of `device`'s copy of the scratch array, looked up once per
// device (with that device current). In host code the array's name stands
// for no device address: only this pointer may reach a kernel.
sand_status scratch_of(int device, char** out) {
  if (device < 0 || device >= kMaxDevices)
    return fail(SAND_ERR_UNSUPPORTED, "sand_query_noalloc: device %d beyond %d", device,
                kMaxDevices);
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return device_fail(e, "sand_query_noalloc: scratch address");
    g_scratch[device] = (char*)p;
  }
  *out = g_scratch[device];
  return SAND_OK;
}

}  // namespace

extern "C" sand_status sand_query_noalloc(sand_model m, sand_depthmap dm, const float* xyz,
                                          int64_t n, float* sdf, const sand_query_opts* opts,
                                          void* stream) {
  sand_query_opts o;
  if (opts) o = *opts; else sand_query_opts_init(&o);
  if (o.workspace)
    return fail(SAND_ERR_INVALID, "sand_query_noalloc: takes no workspace (its scratch is the "
                "library's own)");
  sand_status st = check_query("sand_query_noalloc", m, dm, xyz, n, sdf, o);
  if (st != SAND_OK) return st;
  if (o.mode == SAND_DYNAMIC && o.dynamic_checkpoint != -1)
    return fail(SAND_ERR_UNSUPPORTED, "sand_query_noalloc: dynamic mode runs without compaction "
                "only (dynamic_checkpoint = -1): compaction needs a record arena");
  const size_t need = workspace_layout(n).total;
  if (need > kScratchBytes)
    return fail(SAND_ERR_INVALID, "sand_query_noalloc: %lld points need %zu bytes of scratch, "
                "more than its %zu (at most 13,373,120 points)", (long long)n, need,
                kScratchBytes);
  if (n == 0) return SAND_OK;
  DeviceGuard guard(m->device);
  if (!guard.ok) return fail(SAND_ERR_DEVICE, "sand_query_noalloc: cannot select device");
  char* ws = nullptr;
  if ((st = scratch_of(m->device, &ws)) != SAND_OK) return st;
  return run_forward(m, dm, xyz, n, sdf, o, ws, (hipStream_t)stream);
}
