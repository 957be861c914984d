/*
 * sand.h -- C ABI of the SAND query library for AMD Instinct MI355X (gfx950).
 *
 * SAND answers signed-distance queries with a tailed MLP (T-MLP) whose
 * evaluation depth varies per point (Sec. 3, overview figure): a dense
 * network-depth map gives each point its exit depth d(x) (Sec. 3.2), the
 * T-MLP runs hidden layers 1..d(x) only, and the answer is the accumulated
 * tail output y_d = t_1 + ... + t_d (Eq. 2), with tails 2..L optionally the
 * product of two linear heads (Eq. 3). A depth of 0 marks a far-field cell
 * whose stored value is returned without running the network (Eq. 7,
 * Sec. 3.4). Capping the depth gives the level-of-detail control of Sec. 3.4.
 *
 * Conventions for every entry point:
 *  - Pointers documented "device" must point to memory on the model's GPU;
 *    "host" pointers to ordinary CPU memory. The caller owns every buffer it
 *    passes and the library never frees or keeps them past the call (except
 *    where a server entry point says otherwise).
 *  - All argument and format checks happen on the host before anything is
 *    enqueued; a failing check returns a status != SAND_OK and touches
 *    neither the device nor the output buffers. sand_last_error() then holds
 *    a message for the calling thread.
 *  - Query entry points are asynchronous and ordered on the given HIP
 *    stream (a hipStream_t passed as void*, NULL = the null stream). Model
 *    and map handles are immutable after creation and may be used by
 *    several streams and threads at once; free them only after their work
 *    has completed.
 *  - Device-side failures (a failed launch or allocation) surface as
 *    SAND_ERR_DEVICE from the call that observed them.
 */
#ifndef SAND_H_
#define SAND_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sand_model_s* sand_model;
typedef struct sand_depthmap_s* sand_depthmap;
typedef struct sand_server_s* sand_server;

typedef enum {
  SAND_OK = 0,
  SAND_ERR_INVALID = 1,     /* bad argument (null pointer, size, enum value) */
  SAND_ERR_FORMAT = 2,      /* malformed model blob or depth map */
  SAND_ERR_NOMEM = 3,       /* device or host allocation failed */
  SAND_ERR_DEVICE = 4,      /* HIP runtime or launch error */
  SAND_ERR_BUDGET = 5,      /* a server request alone exceeds the HBM budget */
  SAND_ERR_UNSUPPORTED = 6, /* valid input outside what this build supports */
  SAND_ERR_TIMEOUT = 7      /* sand_server_wait gave up before completion */
} sand_status;

/* Arithmetic of the hidden-layer products W_j h_{j-1}, j >= 2. Layer 1
 * (its omega-scaled sine argument), the sines and every tail are FP32 in
 * all three; the hidden products accumulate in FP32. */
typedef enum { SAND_FP32 = 0, SAND_BF16 = 1, SAND_FP16 = 2 } sand_precision;

/* Where the exit depth comes from:
 *  ADAPTIVE: the depth map (Sec. 3.4);
 *  FULL:     every point runs all L layers (the plain full-depth network);
 *  FORCED:   a caller-given depth per point (opts.forced_depth);
 *  DYNAMIC:  no map: a point stops after the first layer i >= 2 whose
 *            residual (tail output t_i, FP32) satisfies |t_i| < opts.dynamic_r,
 *            else runs to L (the map-free strategy of the Sec. 4.4 ablation;
 *            t_1 is the base prediction and is not tested). */
typedef enum { SAND_ADAPTIVE = 0, SAND_FULL = 1, SAND_FORCED = 2, SAND_DYNAMIC = 3 } sand_mode;

typedef struct {
  int32_t precision;            /* sand_precision */
  int32_t mode;                 /* sand_mode */
  int32_t max_depth;            /* > 0: exit depth <- min(depth, max_depth)
                                   (level of detail, Sec. 3.4); 0: no clamp */
  float dynamic_r;              /* DYNAMIC: residual threshold r > 0;
                                   other modes: must be 0 */
  const uint8_t* forced_depth;  /* device [n], FORCED only: values 0..L
                                   (0 needs a map with far-field values) */
  uint8_t* depth_out;           /* device [n] or NULL: receives each
                                   point's exit depth */
  void* workspace;              /* device scratch or NULL (then the library
                                   allocates stream-ordered scratch itself) */
  size_t workspace_bytes;       /* size of workspace; must be at least
                                   sand_query_workspace_size(n) when given */
  int32_t dynamic_checkpoint;   /* DYNAMIC only (else 0): the layer c after
                                   which points still running leave their
                                   tiles and continue, from layer c + 1, in
                                   full tiles of such points (results are
                                   the same for every c). 0: chosen by the
                                   library from the exit depths of a 65536-
                                   point strided sample when n >= 2^22 (one
                                   host synchronisation); -1: never; values
                                   >= the exit-depth bound mean never. The
                                   library allocates the compaction arena
                                   itself (stream-ordered, at most 2 GiB;
                                   larger queries run in slabs). */
} sand_query_opts;

/* Fill opts with the defaults: FP32, ADAPTIVE, no clamp, no buffers. */
void sand_query_opts_init(sand_query_opts* opts);

/* ---- models ------------------------------------------------------------ */

/* Parse a version-1 model blob (host memory, nbytes long) and upload it to
 * GPU `device`, packed for every precision.
 *
 * Blob layout (little-endian): 64-byte header = magic "SANDTMLP", u32
 * version (1), u32 L (1..16 hidden sine layers), u32 W (1..352 hidden
 * width), u32 input dim (3), f32 omega of layer 1, f32 omega of layers
 * 2..L, u8[16] tail kind per layer (0 linear, 1 multiplicative; unused
 * entries 0), 16 zero bytes; then float32 W_1 [W x 3], b_1 [W],
 * (W_j [W x W] row-major out x in, b_j [W]) for j = 2..L, and per tail in
 * layer order a [W], c (linear) or a0 [W], c0, a1 [W], c1 (Eq. 3).
 * Layer j computes h_j = sin(omega_j (W_j h_{j-1} + b_j)).
 *
 * Errors: SAND_ERR_INVALID (null blob/out, bad device), SAND_ERR_FORMAT
 * (magic, version, size or a non-finite parameter), SAND_ERR_UNSUPPORTED
 * (W > 352), SAND_ERR_NOMEM / SAND_ERR_DEVICE. On success *out owns the
 * device copy until sand_free_model. */
sand_status sand_load_model(const void* blob, size_t nbytes, int device,
                            sand_model* out);
void sand_free_model(sand_model model);
/* Number of hidden layers and width of a loaded model. */
sand_status sand_model_info(sand_model model, int32_t* n_layers,
                            int32_t* width);

/* ---- depth maps ---------------------------------------------------------- */

/* Upload a dense R^3 network-depth map (the dense stand-in for the octree
 * of Sec. 3.2) for use with `model`.
 *  depth_host: host uint8 [R][R][R], C order (x slowest, z fastest), values
 *              0..L; cell i along an axis covers [-1 + 2i/R, -1 + 2(i+1)/R).
 *  R:          power of two, 2..1024.
 *  far_host:   host float32 [R][R][R] far-field values (Eq. 7), read for
 *              cells of depth 0; may be NULL only if no cell has depth 0.
 * Points outside [-1, 1]^3 use the border cell; a NaN coordinate uses
 * cell 0 on that axis.
 * Errors: SAND_ERR_INVALID (null pointers, bad R), SAND_ERR_FORMAT (a
 * value > L, depth 0 without far values), SAND_ERR_NOMEM/_DEVICE. */
sand_status sand_build_depthmap(sand_model model, const uint8_t* depth_host,
                                int32_t R, const float* far_host,
                                sand_depthmap* out);
/* Free a map (before or after its model; queries using it must be done). */
void sand_free_depthmap(sand_depthmap map);

/* What sand_construct_depthmap did. */
typedef struct {
  int64_t near_voxels;     /* voxels with near_host != 0 */
  int64_t samples;         /* near_voxels * s^3 points run to full depth */
  int32_t depth_counts[17];/* voxels per stored depth 0..16 */
} sand_map_info;

/* Build a network-depth map from `model` on the GPU (Sec. 3.2: Eq. 5
 * required depth, Eq. 6 max-pooling per voxel, Eq. 7 far voxels).
 *  near_host:  host uint8 [R][R][R] (C order as above): nonzero marks a
 *              voxel that meets the surface (the paper tests whether the
 *              distance from the voxel centre to the shape is at most half
 *              the voxel diagonal); the caller decides.
 *  center_sdf_host: host float32 [R][R][R], the shape's signed distance at
 *              each voxel centre, stored for far voxels (Eq. 7).
 *  R:          power of two, 2..1024.
 *  s:          samples per axis, 1, 2, 4 or 8: each near voxel is sampled at
 *              the s^3 centres of its sub-cells, -1 + (2/R)(i + (k + 1/2)/s)
 *              per axis (exact in float32). With R = 128 and s = 4 these
 *              are the 512^3 grid's cell centres.
 *  r:          error threshold of Eq. 5 (> 0; the paper uses 1.5e-4).
 *  precision:  arithmetic of the full-depth pass (FP32 recommended: the
 *              decisions compare outputs against r).
 * A near voxel stores max over its samples of
 *   d(x) = min { i : |y_L(x) - y_i(x)| < r and sign(y_i(x)) = sign(y_L(x)) }
 * (1..L), with far value 0; a far voxel stores depth 0 and its centre SDF.
 * Blocking: runs on `stream`, waits for it, and returns the map (*out) and,
 * when depth_host / info are not NULL, a host copy [R^3] and the counts.
 * Errors: SAND_ERR_INVALID (null pointers, bad R, s or r, precision),
 * SAND_ERR_NOMEM / SAND_ERR_DEVICE. */
sand_status sand_construct_depthmap(sand_model model, const uint8_t* near_host,
                                    const float* center_sdf_host, int32_t R,
                                    int32_t s, float r, int32_t precision,
                                    void* stream, sand_depthmap* out,
                                    uint8_t* depth_host, sand_map_info* info);

/* What sand_construct_octree built. */
typedef struct {
  int32_t D;                   /* maximum depth */
  int64_t internal_nodes[11];  /* subdivided nodes per level 0..D-1 */
  int64_t leaves[11];          /* leaves per level 0..D */
  int64_t near_leaves;         /* level-D leaves that meet the surface */
  int64_t samples;             /* near_leaves * s^3 points run to full depth */
  size_t bytes;                /* device memory of the octree */
  int32_t depth_counts[17];    /* leaves per stored depth 0..16 */
} sand_octree_info;

/* Build the sparse network-depth octree of Sec. 3.2 from `model` on the GPU
 * and return it as a map for sand_query (ADAPTIVE and FORCED), the
 * gradient and the server.
 *  D:  maximum depth, 1..10 (the paper uses 9: level-9 cells are the
 *      512^3 grid's cells).
 * Levels l = 0..D, node cells of side 2^(1-l) over [-1, 1]^3. From the root
 * down, a node is subdivided when l < D and it meets the shape the network
 * represents: |y_L(centre)| <= sqrt(3) 2^-l, its centre within half its
 * diagonal (the paper's intersection test, Sec. 4.1, with the network's
 * full-depth value as the distance; FP32 comparison). A level-D node that
 * meets the shape is a near leaf storing the maximum of Eq. 5 over its s^3
 * sub-cell centres (threshold r; s in {1, 2, 4, 8}); every other leaf is
 * far: depth 0 and y_L at its centre (Eq. 7). Storage is pointer-free:
 * per level a bitmask of internal nodes in Morton order with popcount
 * ranks, and per child slot of each internal node a depth byte and a far
 * value (see sand_octree_info.bytes). A point is answered by the leaf whose
 * cell contains it, with the dense map's exact cell rule at level D.
 *  precision: arithmetic of the full-depth passes (FP32 recommended).
 * Blocking: runs on `stream` and waits for it.
 * Errors: SAND_ERR_INVALID (null pointers, bad D, s, r or precision),
 * SAND_ERR_NOMEM / SAND_ERR_DEVICE. */
sand_status sand_construct_octree(sand_model model, int32_t D, int32_t s, float r,
                                  int32_t precision, void* stream, sand_depthmap* out,
                                  sand_octree_info* info);

/* ---- queries ------------------------------------------------------------- */

/* Bytes of device scratch a query of n points needs (same for the gradient). */
size_t sand_query_workspace_size(int64_t n);

/* Signed distance of n points (Sec. 3.4 inference).
 *  xyz_dev: device float32 [n][3] (x, y, z per point), 4-byte aligned.
 *  sdf_dev: device float32 [n], written with y_{d(x)} (or the far value).
 *  map:     required for ADAPTIVE and for FORCED depths of 0; ignored by
 *           FULL (may be NULL there).
 *  opts:    NULL = defaults.
 * n = 0 is a no-op. Errors: SAND_ERR_INVALID (null pointers, n < 0 or
 * n > 2^31 - 1, bad enum, map of another model, workspace too small). */
sand_status sand_query(sand_model model, sand_depthmap map,
                       const float* xyz_dev, int64_t n, float* sdf_dev,
                       const sand_query_opts* opts, void* hip_stream);

/* sand_query for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): it
 * calls no hipMalloc, hipFree or allocating library routine. The scratch
 * that sand_query allocates (or takes as opts.workspace) is instead a 64 MiB
 * device array inside the library, one copy per GPU, held until the process
 * ends; the caller still owns xyz_dev, sdf_dev and the opts buffers.
 *  n:    at most 13,373,120 (sand_query_workspace_size(n) <= 64 MiB).
 *  opts: as sand_query, except that opts.workspace must be NULL and DYNAMIC
 *        mode runs only without compaction (dynamic_checkpoint = -1).
 * All calls on one GPU share its array: two calls that overlap in time on
 * one GPU (any streams) race, so the caller orders them. Results are
 * sand_query's, bit for bit (the same kernels).
 * Errors as sand_query, plus SAND_ERR_INVALID for n above the limit or a
 * workspace, SAND_ERR_UNSUPPORTED for dynamic mode with compaction. */
sand_status sand_query_noalloc(sand_model model, sand_depthmap map,
                               const float* xyz_dev, int64_t n, float* sdf_dev,
                               const sand_query_opts* opts, void* hip_stream);

/* sand_query, instrumented: records HIP events on `hip_stream` between the
 * phases, waits for the query to finish, and stores the device time of each
 * phase in phase_ms (host float[5]): [0] depth lookup and histogram, [1]
 * bucket scan, [2] permutation scatter, [3] T-MLP evaluation with the
 * result scatter, [4] the whole query. Phases a mode skips (FULL runs only
 * the T-MLP) read 0. Blocks the calling thread; meant for measurement.
 * Errors as sand_query, plus SAND_ERR_INVALID for a null phase_ms. */
sand_status sand_query_timed(sand_model model, sand_depthmap map,
                             const float* xyz_dev, int64_t n, float* sdf_dev,
                             const sand_query_opts* opts, void* hip_stream,
                             float* phase_ms);

/* Bytes of device scratch sand_query_grad needs for n points at the given
 * precision (the query scratch plus a per-workgroup stash of the forward
 * pass's cosines); 0 for n <= 0, a null model or a bad precision. */
size_t sand_query_grad_workspace_size(sand_model model, int64_t n,
                                      int32_t precision);

/* Input gradient (surface normal direction) of the queried value with each
 * point's exit depth held fixed: grad_dev[i] = dy[i] * d y_{d(x_i)} / d x_i,
 * computed by reverse accumulation from the exit tail back through layers
 * d..1 (derived from Eq. 2-3). Far-field points (depth 0) get 0.
 *  dy_dev:   device float32 [n] upstream gradient, or NULL for all ones.
 *  sdf_dev:  device float32 [n] or NULL; receives the forward values.
 *  grad_dev: device float32 [n][3].
 *  opts.workspace, when given, must hold sand_query_grad_workspace_size.
 * Other arguments and errors as sand_query. */
sand_status sand_query_grad(sand_model model, sand_depthmap map,
                            const float* xyz_dev, int64_t n,
                            const float* dy_dev, float* sdf_dev,
                            float* grad_dev, const sand_query_opts* opts,
                            void* hip_stream);

/* ---- serving --------------------------------------------------------------- */

typedef struct {
  double t_submit;     /* seconds, library monotonic clock */
  double t_admit;      /* admitted under the HBM budget */
  double t_launch;     /* its batch was enqueued */
  double t_done;       /* its results were complete on the device */
  double t_copied;     /* its results were in the caller's host buffer */
  int64_t n;           /* points in the request */
  int32_t batch_size;  /* requests that shared its launches */
  int32_t reserved;
} sand_req_stats;

/* A request loop on one GPU. Requests name a resident model and map and
 * carry a host query set; the server admits them while the bytes they need
 * (points, results, scratch) fit `hbm_budget_bytes`, packs the admitted
 * requests of all models into shared launches (continuous batching: requests
 * arriving while others run join the next launch), overlaps launches on
 * `n_streams` streams and copies results back. Precision as in
 * sand_query_opts (FP32, BF16 or FP16); mode is always ADAPTIVE.
 * The device bytes a request holds (points, results, bucketing scratch:
 * about 21 bytes per point) are reserved from a single arena of
 * `hbm_budget_bytes` allocated at creation; requests are admitted first-in
 * first-out, so a large request is never overtaken. Host buffers may be
 * pageable; pinned buffers let the copies overlap with computation.
 * n_streams: 1..16 concurrent batches.
 * A result is the same whether a request runs alone or batched. */
sand_status sand_server_create(int device, size_t hbm_budget_bytes,
                               int32_t precision, int32_t n_streams,
                               sand_server* out);
/* Queue one request; never blocks. xyz_host: host float32 [n][3]; sdf_host:
 * host float32 [n] that receives the results. Both must stay valid until
 * sand_server_wait returns for this ticket. Errors: SAND_ERR_INVALID,
 * SAND_ERR_BUDGET (the request alone exceeds the budget). */
sand_status sand_server_submit(sand_server server, sand_model model,
                               sand_depthmap map, const float* xyz_host,
                               int64_t n, float* sdf_host, uint64_t* ticket);
/* Block until request `ticket` has completed (timeout_s < 0: no limit).
 * stats may be NULL. Each ticket can be waited for once. */
sand_status sand_server_wait(sand_server server, uint64_t ticket,
                             double timeout_s, sand_req_stats* stats);
typedef struct {
  size_t budget_bytes;         /* the HBM arena size given at creation */
  size_t reserved_bytes;       /* held now by admitted requests */
  size_t peak_reserved_bytes;  /* maximum ever held (never above the budget) */
  uint64_t submitted;          /* requests accepted by sand_server_submit */
  uint64_t completed;          /* requests whose results are in host memory */
  uint64_t batches;            /* batched launches issued */
  int32_t max_batch_requests;  /* most requests that shared one launch */
  int32_t in_flight_batches;   /* batches on the device now */
} sand_server_info;

/* Counters of a running server. Errors: SAND_ERR_INVALID for null args. */
sand_status sand_server_stats(sand_server server, sand_server_info* info);

/* Stop accepting requests, finish everything admitted or queued, and free
 * the server. Tickets not yet waited for become invalid. */
void sand_server_destroy(sand_server server);

/* ---- errors -------------------------------------------------------------- */

const char* sand_status_str(sand_status status);
/* Message describing the calling thread's most recent failure ("" if none). */
const char* sand_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* SAND_H_ */
