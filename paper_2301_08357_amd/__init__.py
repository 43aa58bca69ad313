"""MI355X-native matrix-free P1 pressure solver (arXiv 2301.08357, Sec. 3.4).

The compute lives in libpressure.so (include/pressure_cg.h); this package is
its Python binding.  Building: ``paper_2301_08357_amd.build.build()``.
"""

from ._lib import (PM_OK, PM_NOT_CONVERGED, PM_PENDING, PM_EINVAL, PM_EDEGENERATE, PM_ENOMEM,  # noqa: F401
                   PM_EBREAKDOWN, PM_EHIP, PM_ETOOLARGE, PM_ETIMEOUT, PM_NOALLOC_MAX_NODES, PM_NOALLOC_MAX_ITER, PM_FP64, PM_FP32_INNER, PM_MASS_LUMPED, PM_TILE_128, PM_TILE_256, PM_TILE_512, PM_VARIANT_AUTO,
                   PM_VARIANT_NODE, PM_VARIANT_TILED, PM_MIXED_KEEP_DIRECTION, PM_MIXED_RESTART, PressureError,
                   load)
from .system import (PressureBatch, PressureSystem, SolveResult, default_tune_cache, footprint,  # noqa: F401
                     layout, tune_batch, tune_tile)
