"""ctypes binding of the SAND C ABI (include/sand.h).

Argument marshalling only: every step of a query runs in the gfx950 kernels
of ``_lib/libsand.so``. Torch supplies device memory and the current HIP
stream. There is no fallback: if the library is missing, every entry point
raises.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# SAND_LIBRARY names another build of the same library (the sanitizer build
# of the host code that the CPU tests load)
LIB_PATH = os.environ.get("SAND_LIBRARY") or os.path.join(_HERE, "_lib", "libsand.so")

OK, ERR_INVALID, ERR_FORMAT, ERR_NOMEM, ERR_DEVICE, ERR_BUDGET, ERR_UNSUPPORTED, ERR_TIMEOUT = range(8)
PRECISIONS = {"fp32": 0, "bf16": 1, "fp16": 2}
MODES = {"adaptive": 0, "full": 1, "forced": 2, "dynamic": 3}


class SandError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"[{status}] {message}")
        self.status = status


class QueryOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("mode", ctypes.c_int32),
                ("max_depth", ctypes.c_int32), ("dynamic_r", ctypes.c_float),
                ("forced_depth", ctypes.c_void_p), ("depth_out", ctypes.c_void_p),
                ("workspace", ctypes.c_void_p), ("workspace_bytes", ctypes.c_size_t),
                ("dynamic_checkpoint", ctypes.c_int32)]


class ServerInfo(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_size_t), ("reserved_bytes", ctypes.c_size_t),
                ("peak_reserved_bytes", ctypes.c_size_t), ("submitted", ctypes.c_uint64),
                ("completed", ctypes.c_uint64), ("batches", ctypes.c_uint64),
                ("max_batch_requests", ctypes.c_int32), ("in_flight_batches", ctypes.c_int32)]


class ReqStats(ctypes.Structure):
    _fields_ = [("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double),
                ("t_copied", ctypes.c_double), ("n", ctypes.c_int64),
                ("batch_size", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class MapInfo(ctypes.Structure):
    _fields_ = [("near_voxels", ctypes.c_int64), ("samples", ctypes.c_int64),
                ("depth_counts", ctypes.c_int32 * 17)]


class OctreeInfo(ctypes.Structure):
    _fields_ = [("D", ctypes.c_int32), ("internal_nodes", ctypes.c_int64 * 11),
                ("leaves", ctypes.c_int64 * 11), ("near_leaves", ctypes.c_int64),
                ("samples", ctypes.c_int64), ("bytes", ctypes.c_size_t),
                ("depth_counts", ctypes.c_int32 * 17)]


_lib = None


def library():
    """The loaded shared library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"SAND library not built: {LIB_PATH} is missing "
                               "(run __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        P, I32, I64, SZ, U64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t, ctypes.c_uint64
        sig = {
            "sand_query_opts_init": (None, [P]),
            "sand_load_model": (I32, [P, SZ, ctypes.c_int, ctypes.POINTER(P)]),
            "sand_free_model": (None, [P]),
            "sand_model_info": (I32, [P, ctypes.POINTER(I32), ctypes.POINTER(I32)]),
            "sand_build_depthmap": (I32, [P, P, I32, P, ctypes.POINTER(P)]),
            "sand_free_depthmap": (None, [P]),
            "sand_construct_depthmap": (I32, [P, P, P, I32, I32, ctypes.c_float, I32, P,
                                              ctypes.POINTER(P), P, ctypes.POINTER(MapInfo)]),
            "sand_construct_octree": (I32, [P, I32, I32, ctypes.c_float, I32, P,
                                            ctypes.POINTER(P), ctypes.POINTER(OctreeInfo)]),
            "sand_query_workspace_size": (SZ, [I64]),
            "sand_query_grad_workspace_size": (SZ, [P, I64, I32]),
            "sand_query": (I32, [P, P, P, I64, P, ctypes.POINTER(QueryOpts), P]),
            "sand_query_noalloc": (I32, [P, P, P, I64, P, ctypes.POINTER(QueryOpts), P]),
            "sand_query_timed": (I32, [P, P, P, I64, P, ctypes.POINTER(QueryOpts), P,
                                       ctypes.POINTER(ctypes.c_float)]),
            "sand_query_grad": (I32, [P, P, P, I64, P, P, P, ctypes.POINTER(QueryOpts), P]),
            "sand_server_create": (I32, [ctypes.c_int, SZ, I32, I32, ctypes.POINTER(P)]),
            "sand_server_submit": (I32, [P, P, P, P, I64, P, ctypes.POINTER(U64)]),
            "sand_server_wait": (I32, [P, U64, ctypes.c_double, ctypes.POINTER(ReqStats)]),
            "sand_server_stats": (I32, [P, ctypes.POINTER(ServerInfo)]),
            "sand_server_destroy": (None, [P]),
            "sand_status_str": (ctypes.c_char_p, [I32]),
            "sand_last_error": (ctypes.c_char_p, []),
        }
        for name, (res, args) in sig.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _check(status, what=""):
    if status != OK:
        msg = library().sand_last_error().decode(errors="replace")
        raise SandError(status, msg or what)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Model:
    """A T-MLP uploaded to one GPU (sand_load_model)."""

    def __init__(self, blob, device=0):
        blob = bytes(blob)
        h = ctypes.c_void_p()
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(library().sand_load_model(buf, len(blob), device, ctypes.byref(h)))
        self._h = h
        self.device = device
        L, W = ctypes.c_int32(), ctypes.c_int32()
        _check(library().sand_model_info(h, ctypes.byref(L), ctypes.byref(W)))
        self.L, self.W = L.value, W.value

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("model has been freed")
        return self._h

    def free(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.sand_free_model(self._h)
        self._h = None

    def __del__(self):
        self.free()


class DepthMap:
    """A dense R^3 network-depth map for one model (sand_build_depthmap)."""

    def __init__(self, model, depth, far=None, _handle=None):
        if _handle is not None:     # built on the device (construct_depthmap)
            self._h = _handle
            self.model = model
            self.R = int(depth)
            return
        depth = np.ascontiguousarray(depth, dtype=np.uint8)
        if depth.ndim != 3 or not (depth.shape[0] == depth.shape[1] == depth.shape[2]):
            raise ValueError("depth map must be a cube [R, R, R]")
        farp = None
        if far is not None:
            far = np.ascontiguousarray(far, dtype=np.float32)
            if far.shape != depth.shape:
                raise ValueError("far values must match the map's shape")
            farp = far.ctypes.data_as(ctypes.c_void_p)
        h = ctypes.c_void_p()
        _check(library().sand_build_depthmap(model.handle, depth.ctypes.data_as(ctypes.c_void_p),
                                             depth.shape[0], farp, ctypes.byref(h)))
        self._h = h
        self.model = model
        self.R = depth.shape[0]

    @property
    def handle(self):
        if self._h is None:
            raise ValueError("depth map has been freed")
        return self._h

    def free(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.sand_free_depthmap(self._h)
        self._h = None

    def __del__(self):
        self.free()


def load_model(blob, device=0):
    return Model(blob, device)


def build_depthmap(model, depth, far=None):
    return DepthMap(model, depth, far)


def construct_octree(model, D=9, s=1, r=1.5e-4, precision="fp32", stream=None):
    """Build the sparse network-depth octree from the model on the GPU
    (sand_construct_octree). Returns (DepthMap, info dict)."""
    info = OctreeInfo()
    h = ctypes.c_void_p()
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(library().sand_construct_octree(model.handle, int(D), int(s), float(r), p,
                                           _stream(stream), ctypes.byref(h), ctypes.byref(info)))
    dm = DepthMap(model, 1 << int(D), _handle=h)
    D = info.D
    return dm, {"D": D, "internal_nodes": list(info.internal_nodes)[:D],
                "leaves": list(info.leaves)[:D + 1], "near_leaves": info.near_leaves,
                "samples": info.samples, "bytes": info.bytes,
                "depth_counts": list(info.depth_counts)}


def construct_depthmap(model, near, center_sdf, s=4, r=1.5e-4, precision="fp32", stream=None):
    """Build a network-depth map from the model on the GPU
    (sand_construct_depthmap). near: uint8/bool [R, R, R] near-surface mask;
    center_sdf: float [R, R, R] signed distance at voxel centres (stored for
    far voxels). Returns (DepthMap, depth uint8 [R, R, R], info dict)."""
    near = np.ascontiguousarray(near, dtype=np.uint8)
    if near.ndim != 3 or not (near.shape[0] == near.shape[1] == near.shape[2]):
        raise ValueError("near mask must be a cube [R, R, R]")
    csdf = np.ascontiguousarray(center_sdf, dtype=np.float32)
    if csdf.shape != near.shape:
        raise ValueError("centre values must match the mask's shape")
    R = near.shape[0]
    depth = np.empty_like(near)
    info = MapInfo()
    h = ctypes.c_void_p()
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    _check(library().sand_construct_depthmap(
        model.handle, near.ctypes.data_as(ctypes.c_void_p), csdf.ctypes.data_as(ctypes.c_void_p),
        R, int(s), float(r), p, _stream(stream), ctypes.byref(h),
        depth.ctypes.data_as(ctypes.c_void_p), ctypes.byref(info)))
    dm = DepthMap(model, R, _handle=h)
    return dm, depth, {"near_voxels": info.near_voxels, "samples": info.samples,
                       "depth_counts": list(info.depth_counts)}


def query_workspace_size(n):
    return int(library().sand_query_workspace_size(int(n)))


def query_grad_workspace_size(model, n, precision="fp32"):
    p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    return int(library().sand_query_grad_workspace_size(model.handle, int(n), p))


def _opts(precision, mode, max_depth, forced_depth, depth_out, workspace, dynamic_r=0.0,
          dynamic_checkpoint=0):
    o = QueryOpts()
    library().sand_query_opts_init(ctypes.byref(o))
    o.dynamic_r = float(dynamic_r)
    o.dynamic_checkpoint = int(dynamic_checkpoint)
    o.precision = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    o.mode = MODES[mode] if isinstance(mode, str) else int(mode)
    o.max_depth = int(max_depth)
    o.forced_depth = None if forced_depth is None else forced_depth.data_ptr()
    o.depth_out = None if depth_out is None else depth_out.data_ptr()
    if workspace is not None:
        o.workspace = workspace.data_ptr()
        o.workspace_bytes = workspace.numel() * workspace.element_size()
    return o


def _check_points(xyz):
    import torch
    if xyz.dtype != torch.float32 or xyz.dim() != 2 or xyz.shape[1] != 3:
        raise ValueError("xyz must be a float32 tensor of shape [n, 3]")
    if not xyz.is_contiguous():
        raise ValueError("xyz must be contiguous")


def query(model, dmap, xyz, out=None, precision="fp32", mode="adaptive", max_depth=0,
          forced_depth=None, depth_out=None, workspace=None, stream=None, dynamic_r=0.0,
          dynamic_checkpoint=0):
    """Signed distances of points ``xyz`` (float32 [n, 3] on the model's GPU).
    mode "dynamic" needs no map and takes the residual threshold dynamic_r;
    dynamic_checkpoint: layer after which running points are compacted (0:
    chosen by the library, -1: never)."""
    import torch
    _check_points(xyz)
    n = xyz.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=xyz.device)
    o = _opts(precision, mode, max_depth, forced_depth, depth_out, workspace, dynamic_r,
              dynamic_checkpoint)
    _check(library().sand_query(model.handle, None if dmap is None else dmap.handle, _ptr(xyz), n,
                                _ptr(out), ctypes.byref(o), _stream(stream)))
    return out


def query_noalloc(model, dmap, xyz, out=None, precision="fp32", mode="adaptive", max_depth=0,
                  forced_depth=None, depth_out=None, workspace=None, stream=None, dynamic_r=0.0,
                  dynamic_checkpoint=0):
    """query() through sand_query_noalloc: the library allocates nothing (its
    scratch is a fixed device array; at most 13,373,120 points, no
    workspace, dynamic mode only with dynamic_checkpoint=-1). Pass ``out``
    to keep this call free of torch allocations too."""
    import torch
    _check_points(xyz)
    n = xyz.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=xyz.device)
    o = _opts(precision, mode, max_depth, forced_depth, depth_out, workspace, dynamic_r,
              dynamic_checkpoint)
    _check(library().sand_query_noalloc(model.handle, None if dmap is None else dmap.handle,
                                        _ptr(xyz), n, _ptr(out), ctypes.byref(o),
                                        _stream(stream)))
    return out


def query_timed(model, dmap, xyz, out=None, precision="fp32", mode="adaptive", max_depth=0,
                forced_depth=None, depth_out=None, workspace=None, stream=None, dynamic_r=0.0,
                dynamic_checkpoint=0):
    """query() that waits and returns (out, phase_ms): device milliseconds of
    [lookup, scan, scatter, t-mlp, whole query] measured with HIP events."""
    import torch
    _check_points(xyz)
    n = xyz.shape[0]
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=xyz.device)
    o = _opts(precision, mode, max_depth, forced_depth, depth_out, workspace, dynamic_r,
              dynamic_checkpoint)
    ms = (ctypes.c_float * 5)()
    _check(library().sand_query_timed(model.handle, None if dmap is None else dmap.handle,
                                      _ptr(xyz), n, _ptr(out), ctypes.byref(o), _stream(stream),
                                      ms))
    return out, [float(v) for v in ms]


def query_grad(model, dmap, xyz, dy=None, sdf_out=None, grad_out=None, precision="fp32",
               mode="adaptive", max_depth=0, forced_depth=None, depth_out=None, workspace=None,
               stream=None):
    """Input gradient dy * d y_{d(x)} / dx, float32 [n, 3]; also fills sdf_out if given."""
    import torch
    _check_points(xyz)
    n = xyz.shape[0]
    if grad_out is None:
        grad_out = torch.empty((n, 3), dtype=torch.float32, device=xyz.device)
    o = _opts(precision, mode, max_depth, forced_depth, depth_out, workspace)
    _check(library().sand_query_grad(model.handle, None if dmap is None else dmap.handle, _ptr(xyz),
                                     n, _ptr(dy), _ptr(sdf_out), _ptr(grad_out), ctypes.byref(o),
                                     _stream(stream)))
    return grad_out


class Server:
    """The request loop of one GPU (sand_server_*).

    submit() takes host arrays (numpy float32 [n, 3] points and a float32 [n]
    result buffer, ideally pinned) and returns a ticket; wait() blocks until
    that request's results are in its buffer and returns its time stamps.
    The arrays must stay alive until wait() returns for their ticket.
    """

    def __init__(self, device=0, budget_bytes=4 << 30, precision="bf16", n_streams=2):
        h = ctypes.c_void_p()
        p = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
        _check(library().sand_server_create(device, int(budget_bytes), p, int(n_streams),
                                            ctypes.byref(h)))
        self._h = h
        self._keep = {}

    def submit(self, model, dmap, xyz, sdf_out):
        t = ctypes.c_uint64()
        xp = _host_ptr(xyz, np.float32, 2)
        yp = _host_ptr(sdf_out, np.float32, 1)
        n = int(xyz.shape[0])
        if sdf_out.shape[0] != n:
            raise ValueError("result buffer has the wrong length")
        _check(library().sand_server_submit(self._h, model.handle, dmap.handle, xp, n, yp,
                                            ctypes.byref(t)))
        self._keep[t.value] = (xyz, sdf_out, model, dmap)
        return t.value

    def wait(self, ticket, timeout=-1.0):
        st = ReqStats()
        try:
            _check(library().sand_server_wait(self._h, ticket, float(timeout), ctypes.byref(st)))
        except SandError as e:
            # a timeout leaves the request running, and an invalid ticket is
            # unknown or has another waiter: its buffers stay referenced
            if e.status not in (ERR_TIMEOUT, ERR_INVALID):
                self._keep.pop(ticket, None)
            raise
        self._keep.pop(ticket, None)
        return {k: getattr(st, k) for k, _ in ReqStats._fields_}

    def stats(self):
        info = ServerInfo()
        _check(library().sand_server_stats(self._h, ctypes.byref(info)))
        return {k: getattr(info, k) for k, _ in ServerInfo._fields_}

    def close(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.sand_server_destroy(self._h)
        self._h = None
        self._keep = {}

    def __del__(self):
        self.close()


def _host_ptr(a, dtype, ndim):
    """Data pointer of a host array (numpy, or a CPU torch tensor)."""
    if hasattr(a, "data_ptr"):
        if a.is_cuda or not a.is_contiguous():
            raise ValueError("server buffers must be contiguous host tensors")
        return ctypes.c_void_p(a.data_ptr())
    if not isinstance(a, np.ndarray) or a.dtype != dtype or a.ndim != ndim or \
            not a.flags.c_contiguous:
        raise ValueError("server buffers must be C-contiguous float32 numpy arrays")
    return a.ctypes.data_as(ctypes.c_void_p)
