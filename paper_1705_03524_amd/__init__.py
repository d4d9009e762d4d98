"""MI355X-native spatially weighted local histograms (SWIH) in O(1).

HIP kernels for gfx950 behind the C ABI declared in ``include/swih.h``
(libswih.so); this package is its Python binding.
"""
from ._swih import (EUCLIDEAN, EXPONENTIAL, GAUSSIAN, GAUSSIAN_SEP, KERNELS, MANHATTAN, UNIFORM, Config,
                    SwihError, argmax, argmax_decode, brute_match, build, build_phase, cake_match, cake_query, copy,
                    gauss_terms, load, match, match_noalloc, query, status_string, workspace_bytes)

__all__ = ["Config", "SwihError", "build", "build_phase", "query", "match", "match_noalloc", "workspace_bytes", "gauss_terms",
           "cake_query", "cake_match", "brute_match", "argmax", "argmax_decode", "copy",
           "load", "status_string", "UNIFORM", "MANHATTAN", "EUCLIDEAN", "GAUSSIAN", "GAUSSIAN_SEP",
           "EXPONENTIAL", "KERNELS",
           "Plan"]


def __getattr__(name):
    if name == "Plan":
        from .plan import Plan
        return Plan
    raise AttributeError(name)
