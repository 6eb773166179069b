"""TV-Stokes denoising with overlapping Schwarz domain decomposition on AMD
MI355X: Python binding of the HIP library libtvs (see include/tvs.h).

Modules: ``tvs`` (the ctypes binding: contexts, one-shot solves, jobs,
checkpoints, quality measures), ``serve`` (continuous batching of requests as
jobs), ``quality`` (the parameter selection of Section 5.2), ``validate``
(the domain-decomposition validation of Section 6.3) and ``build`` (compiles
libtvs.so for gfx950)."""
from .tvs import (Context, Job, Params, Layout, Iters, Stats, TvsError, job_footprint, make_params,
                  make_layout, make_iters, TVS_EINVAL, TVS_ENONFINITE, TVS_EBUSY, TVS_IRV1, TVS_IRV2, TVS_LP_IMAGE, TVS_LP_BLOCKDCT, load)

__all__ = ["Context", "Job", "Params", "Layout", "Iters", "Stats", "TvsError", "job_footprint",
           "make_params", "make_layout", "make_iters", "TVS_EINVAL", "TVS_ENONFINITE", "TVS_EBUSY", "TVS_IRV1", "TVS_IRV2", "TVS_LP_IMAGE",
           "TVS_LP_BLOCKDCT", "load"]
