"""FP64 CPU oracle for exhaustive constrained top-k over a combinatorial synthesis
library (test infrastructure: used by tests, the smoke check and the benchmark's
CPU-baseline leg only; never by the product path)."""
from .oracle import (  # noqa: F401
    build,
    max_threads,
    num_compounds,
    decode,
    heads,
    topk,
    topk_lex,
    TopK,
    assoc_embeddings,
)
