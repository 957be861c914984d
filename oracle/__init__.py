"""FP64 CPU oracle for the SAND query path. TEST INFRASTRUCTURE ONLY.

This package is the plain, slow, obviously-correct reference that the GPU
library is checked against. Only the test suite, the package smoke check and
the benchmark's CPU-baseline leg may import it; the product path never
does. It shares no code with the GPU library: it has its own model-blob
parser and evaluates everything in float64 with numpy.

Modules:
  blob     -- model-blob parser (independent of the C++ loader)
  tmlp     -- voxel lookup, depth rule, T-MLP forward and input gradient
              (Sec. 3.1 Eq. 2-3, Sec. 3.2 Eq. 7, Sec. 3.4)
  scalar   -- a pure-Python scalar twin for tiny brute-force checks
  depthmap -- building the network-depth map from a model (Sec. 3.2,
              Eq. 5-7): required depth per point, sub-cell samples,
              max-pooling per voxel, far voxels
  dynamic  -- map-free early exit on small residuals (Sec. 4.4 ablation)
  octree   -- the sparse network-depth octree: top-down subdivision, leaf
              depths and far values, point lookup (Sec. 3.2, Eq. 5-7)

Parity status per function (what pins it) is listed in each module header.
"""

from .blob import parse_blob
from .tmlp import (voxel_index, lookup_depth, forward, forward_all_tails,
                   gradient, MODE_ADAPTIVE, MODE_FULL, MODE_FORCED)
from . import depthmap, dynamic, octree

__all__ = ["parse_blob", "voxel_index", "lookup_depth", "forward",
           "forward_all_tails", "gradient", "MODE_ADAPTIVE", "MODE_FULL",
           "MODE_FORCED", "depthmap", "dynamic", "octree"]
