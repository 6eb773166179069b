"""TV-Stokes denoising with overlapping Schwarz domain decomposition on AMD
MI355X: Python binding of the HIP library libtvs (see include/tvs.h)."""
from .tvs import (Context, Job, Params, Layout, Iters, Stats, TvsError, job_footprint, make_params,
                  make_layout, make_iters, TVS_EBUSY, TVS_IRV1, TVS_IRV2, TVS_LP_IMAGE, TVS_LP_BLOCKDCT, load)

__all__ = ["Context", "Job", "Params", "Layout", "Iters", "Stats", "TvsError", "job_footprint",
           "make_params", "make_layout", "make_iters", "TVS_EBUSY", "TVS_IRV1", "TVS_IRV2", "TVS_LP_IMAGE",
           "TVS_LP_BLOCKDCT", "load"]
