"""MI355X (gfx950) library for the per-timestep hot path of united-atom polyethylene MD.

The computation lives in ``libmd_gfx950.so`` (HIP, C ABI in ``include/md.h``);
``paper_1001_3764_amd.md`` is its ctypes binding.  Importing this package loads nothing.
"""
