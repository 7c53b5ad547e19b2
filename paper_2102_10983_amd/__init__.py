"""MI355X-native sub-cycled Boris particle push (arXiv:2102.10983).

The hot path lives in libpicsub.so (HIP kernels for gfx950 behind the C ABI
of include/picsub.h); ``picsub`` is its Python binding and ``workloads``
draws the seeded synthetic inputs.
"""

from . import workloads  # noqa: F401

__all__ = ["workloads", "picsub"]
