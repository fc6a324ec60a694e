"""MI355X (gfx950) hot path of the modified Hermite integrators of
Dittmann (2020, arXiv:2006.02501): HIP kernels behind a C ABI
(``include/hermite.h``) and a thin ctypes binding."""
from .hermite import (  # noqa: F401
    BatchHermite, DeviceState, EnsembleHermite, Hermite, HermiteError, fma_rate, force_derivs_noalloc, load_library,
    tune_cache_clear,
    version, CORRECTORS,
    PRECISIONS,
)
