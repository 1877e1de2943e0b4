"""MI355X (gfx950) TreePM gravity: tree build, tree walk and PM long-range
force of the Arepo code behind a C ABI (``include/treepm.h``).

``binding`` wraps ``libtreepm.so``; ``workloads`` draws the seeded synthetic
inputs; ``build`` compiles the HIP sources.
"""
from . import workloads  # noqa: F401

__all__ = ["workloads", "binding", "build"]
