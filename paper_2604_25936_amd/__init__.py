"""SAND query path for AMD Instinct MI355X (gfx950).

Batched signed-distance queries of a tailed sine MLP (T-MLP) whose depth
varies per point through a network-depth map (Sec. 3 of the SAND paper),
served by hand-written HIP kernels behind the C ABI of include/sand.h.
This package is the Python binding of that library.
"""

from .sand import (Model, DepthMap, Server, SandError, load_model, build_depthmap,
                   construct_depthmap, construct_octree, query, query_noalloc,
                   query_timed, query_grad, query_workspace_size,
                   query_grad_workspace_size, library, PRECISIONS, MODES)

__all__ = ["Model", "DepthMap", "Server", "SandError", "load_model", "build_depthmap",
           "construct_depthmap", "construct_octree", "query", "query_noalloc",
           "query_timed", "query_grad", "query_workspace_size",
           "query_grad_workspace_size", "library", "PRECISIONS", "MODES"]
