"""MI355X (gfx950) content-area estimator for endoscopic video
(Budd et al., arXiv 2210.14771, Section 2.2).

The estimator lives in libcontentarea.so (HIP kernels behind a C ABI,
``include/contentarea.h``); this package binds it to PyTorch tensors.
Importing the package does not load the library; the first estimate does,
and raises if the library has not been built.
"""
__version__ = "0.1.0"

__all__ = ["Estimator", "Result", "default_params", "estimate_area", "strip_positions",
           "score_tables"]


def __getattr__(name):
    if name in __all__:
        from . import api
        return getattr(api, name)
    raise AttributeError(name)
