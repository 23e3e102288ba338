"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This package draws random numbers and shapes only. It holds none of the
search method's arithmetic (no combine, no decoder, no selection), so that
the oracle and the HIP path stay independent of each other.
"""
from .gen import (  # noqa: F401
    Library,
    Decoder,
    Query,
    Constraint,
    normal_f32,
    uniform_f64,
    make_library,
    make_decoder,
    lognormal_counts,
    config_c0,
    config_c1,
    config_c3_shape,
    library_shapes_c1,
)
