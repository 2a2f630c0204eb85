"""MI355X DEM force step (Nakahara & Washizawa, arXiv:1503.03553) behind a C ABI.

The compute path is libdem.so (HIP kernels for gfx950, see include/dem.h);
this package only marshals arguments to it through ctypes.  There is no CPU
fallback: importing works without the library, but creating a simulation
raises if libdem.so is missing or no GPU is present.
"""
from .binding import (DEM_FACE_ID, DemError, Pool, PreparedJob, Sim, lib, library_path,  # noqa: F401
                      status_str, footprint, pool_footprint, make_pool_params, PREC_FP64,
                      PREC_MIXED, FLAG_NO_FORCE_OUTPUT, FLAG_RADIX_SORT, FLAG_FUSED,
                      FLAG_ACTION_REACTION, FLAG_THREAD_SPLIT, FLAG_FULL_DETECT,
                      JOB_RUNNING, JOB_DONE, JOB_FAILED)

__all__ = ["Sim", "Pool", "PreparedJob", "DemError", "lib", "library_path", "status_str", "footprint",
           "pool_footprint", "make_pool_params", "DEM_FACE_ID", "PREC_FP64", "PREC_MIXED",
           "FLAG_NO_FORCE_OUTPUT", "FLAG_RADIX_SORT", "FLAG_FUSED",
           "FLAG_ACTION_REACTION", "FLAG_THREAD_SPLIT", "FLAG_FULL_DETECT",
           "JOB_RUNNING", "JOB_DONE", "JOB_FAILED"]
