"""MI355X (gfx950) Barnes-Hut: octree construction and per-body tree-walk
forces (Brandt, arXiv:2203.08966, Sec. 3) as hand-written HIP kernels behind
the C ABI in include/bh.h.  ``binding`` is the ctypes layer; ``workloads``
the seeded synthetic inputs."""
from . import binding, workloads  # noqa: F401
from .binding import *  # noqa: F401,F403
