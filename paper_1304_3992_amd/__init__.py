"""liblogfx: an MI355X-native (gfx950) implementation of the LoG feature
extraction pipeline of Tejaswi et al., arXiv:1304.3992.

The compute path is the C-ABI shared library ``liblogfx.so`` (hand-written HIP
kernels); :mod:`paper_1304_3992_amd.logfx` is a thin ctypes binding with the
same names.  :mod:`paper_1304_3992_amd.scenes` generates seeded synthetic
inputs.  Importing this package does not load the GPU library; the first use
of an attribute of the binding does.
"""

__all__ = ["logfx", "scenes"]


def __getattr__(name):
    if name in ("logfx", "scenes"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
