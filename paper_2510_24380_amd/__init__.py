"""MI355X (gfx950) engine for exhaustive constrained top-k search of
combinatorial synthesis libraries scored by a structure-factorised surrogate
(APEX, arXiv 2510.24380). The compute lives in libapex.so (include/apex.h);
this package is its Python binding."""
from .binding import (  # noqa: F401
    ApexError,
    Decoder,
    Engine,
    Library,
    ResultBuffers,
    SearchResult,
    Server,
    lib,
)
