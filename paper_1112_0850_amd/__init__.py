"""MI355X (gfx950) D3Q19 BGK lattice Boltzmann hot path.

``paper_1112_0850_amd.lbm`` holds the ``LBM`` class and the differentiable
``rollout``; ``_abi`` the ctypes declarations of include/lbm.h; ``inputs``
the seeded synthetic inputs.  Attributes load lazily so that importing the
package needs neither a GPU nor the built library.
"""

__all__ = ["LBM", "rollout", "stream_copy"]


def __getattr__(name):
    if name in __all__:
        from . import lbm
        return getattr(lbm, name)
    raise AttributeError(name)
