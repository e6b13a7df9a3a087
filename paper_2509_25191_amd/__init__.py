"""vggtx: MI355X-native memory-efficient dense-view aggregator (VGGT-X, arXiv 2509.25191, Sec. 3.2).

The compute path is the HIP library ``libvggtx.so`` (C-ABI in include/vggtx.h);
``paper_2509_25191_amd.vggtx`` is its thin Python binding.  There is no CPU or
PyTorch fallback: if the library is not built, importing the binding's
functions raises.
"""
from . import vggtx  # noqa: F401
from .vggtx import *  # noqa: F401,F403
