"""MI355X-native TUCKET engine: range queries of Tucker decompositions over a
stream segment tree, with the hot path (Recall, trims, Stitch, leaf
Tucker-ALS, merges) in HIP kernels for gfx950 behind the C ABI of
include/tucket.h."""

from .tucket import (  # noqa: F401
    LIB_PATH,
    PreparedBatch,
    QueryResult,
    Server,
    Tree,
    TuckerError,
    effective_ranks,
    hitset_plan,
    lib,
    make_config,
)
