"""MI355X (gfx950) subgraph-isomorphism hot path of GSI (arXiv 1906.03420).

The library itself is libgsi.so (HIP C++, C ABI in include/gsi.h); this
package is its thin ctypes binding plus the build script.
"""
from .binding import *  # noqa: F401,F403
from .binding import Batch, Context, Graph, GsiError, Result, Server, load_library  # noqa: F401
