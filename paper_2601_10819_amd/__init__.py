"""MI355X-native multi-scale deformable aggregation (MSDA).

The library is libmsda.so (HIP kernels for gfx950 behind the C ABI in
include/msda.h); ``ops`` binds it to PyTorch tensors and streams and
``synth`` draws seeded synthetic inputs. Importing the package does not load
the library; the first call into ``ops`` does, and fails if it is not built.
"""
__all__ = ["ops", "synth", "build"]


def __getattr__(name):
    if name in ("ops", "synth", "build", "_lib"):
        import importlib
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
