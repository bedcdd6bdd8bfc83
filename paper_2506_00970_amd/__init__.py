"""MI355X-native differentiable 2D Gaussian surfel rasterizer (gfx950 HIP kernels behind a C ABI).

``Rasterizer`` (render, backward, tracking loss, graph-captured tracking loop) and
``render`` (a ``torch.autograd.Function``) bind ``libgs2d.so``; build it with
``python -m paper_2506_00970_amd.build``.  Importing this package does not load
the library; the first ``Rasterizer`` does, and raises if it is missing.
"""

from ._lib import ERR_NONFINITE, Gs2dError  # noqa: F401


def __getattr__(name):
    if name == "Rasterizer":
        from .rasterizer import Rasterizer

        return Rasterizer
    if name in ("render", "RenderFunction"):
        from . import autograd

        return getattr(autograd, name)
    raise AttributeError(name)
