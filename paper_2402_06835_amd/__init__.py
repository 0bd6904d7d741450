"""MI355X-native transit-search hot path of nuance (arXiv:2402.06835).

Linear search (GLS box fits over epochs x durations under a fixed GP
covariance) and periodic search (common-depth fold over periods x phases),
as hand-written HIP kernels for gfx950 behind the C ABI of
include/nuance_mi355x.h. Importing this package loads nothing; the library
is loaded on first use and its absence is an error.
"""

__all__ = ["Context", "Factor", "SHO", "Nuance", "SearchResult", "gp_factor", "linear_search", "periodic_search"]


def __getattr__(name):
    if name in __all__:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
