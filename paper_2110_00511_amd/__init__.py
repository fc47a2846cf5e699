"""MI355X-native (gfx950) spatial hash map after ASH (arXiv 2110.00511).

HashMap / HashSet / voxelize call the C ABI of include/ash.h implemented by
libash.so (hand-written HIP kernels); torch supplies device memory and
streams.  Build the library with `python -m paper_2110_00511_amd.build`.
"""
from .hashmap import HashMap, HashSet, Server, autotune, batched, block_coords, neighbor_offsets, voxelize

__all__ = ["HashMap", "HashSet", "Server", "autotune", "batched", "block_coords", "neighbor_offsets", "voxelize"]
