"""MI355X-native FLoD-3DGS rasterizer: multi-level Gaussian stack, selective rendering and a
differentiable tile-based splatting pipeline in hand-written HIP kernels behind a C ABI.

Submodules:
  synth     seeded synthetic scenes, cameras and request traces (no torch needed)
  render    Renderer, GaussianLevel, rasterize / FLoDRasterize (torch device memory and streams)
  serving   continuous-batching render server with HBM admission
  build     in-tree hipcc build of libflod.so
"""
import importlib

__all__ = ["synth", "render", "serving", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
