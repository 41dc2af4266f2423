"""Exact GPU distance maps for real-time collision avoidance on MI355X.

Hot path of "Real Time Collision Avoidance with GPU-Computed Distance Maps":
insert a point cloud and voxelized robot links into occupancy maps, compute
the exact squared Euclidean distance transform with nearest-site indices,
and query it at bounding-sphere centres.  The compute lives in hand-written
HIP kernels behind the C-ABI library ``libedtmi.so`` (declared in
``include/edt.h``); ``paper_2407_02363_amd.edt`` is its thin binding.

Importing this package does not load the library; the binding loads it on
first use and raises if it is missing.
"""
__all__ = ["inputs"]
