"""MI355X-native fragment-history volumes: capture into per-pixel or
per-octant fragment lists, compaction into per-octant arrays and point
splatting into novel views, as hand-written HIP kernels for gfx950 behind a
C ABI (include/fhv.h).

Importing the package loads nothing; ``paper_2211_15460_amd.fhv`` loads the
native library and raises if it is missing.
"""
__all__ = ["scenes"]
