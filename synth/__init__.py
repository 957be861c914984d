"""Seeded synthetic inputs for the SAND query path.

This package draws the inputs that both the FP64 oracle and the GPU library
consume: T-MLP parameter sets serialised as model blobs, analytic surfaces,
dense network-depth maps derived from those surfaces, and query point sets.
It holds none of the method's arithmetic (no T-MLP evaluation, no depth-map
lookup): each generator only draws numbers and lays them out.

Every generator takes an explicit seed and uses numpy's PCG64 with a fixed
draw order, so a (seed, shape) pair always yields the same bytes.
"""

from .blob import (MAGIC, VERSION, HEADER_BYTES, TAIL_LINEAR, TAIL_MULT,
                   write_blob, blob_nbytes)
from .model import siren_tmlp, TailScale
from .surface import sphere_sdf, Primitives, random_primitives
from .depthmap import (voxel_centres, band_map_c1, band_map_c2, far_value_grid,
                       near_surface_mask)
from .queries import (grid_points, grid_points_at, sample_indices,
                      near_surface_points, slab_points, camera_ray_points)

__all__ = [
    "MAGIC", "VERSION", "HEADER_BYTES", "TAIL_LINEAR", "TAIL_MULT",
    "write_blob", "blob_nbytes", "siren_tmlp", "TailScale",
    "sphere_sdf", "Primitives", "random_primitives",
    "voxel_centres", "band_map_c1", "band_map_c2", "far_value_grid", "near_surface_mask",
    "grid_points", "grid_points_at", "sample_indices",
    "near_surface_points", "slab_points", "camera_ray_points",
]
