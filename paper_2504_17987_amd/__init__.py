"""MI355X-native PIV hot path (predictor, deformation, correlation with
Gaussian sub-pixel fit, normalised-median validation, vorticity) behind the
C ABI of include/piv.h.

Submodules load lazily so that the input generator can be used without the
compiled library:
  - ``api``      Plan: torch tensors in, fields out (needs libpiv.so)
  - ``autograd`` differentiable windowed SSD and gradient refinement
  - ``serve``    continuous-batching server for streams of pairs
  - ``synth``    seeded particle-image pairs and analytic flows
"""
__all__ = ["api", "autograd", "serve", "synth", "build"]


def __getattr__(name):
    import importlib
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
