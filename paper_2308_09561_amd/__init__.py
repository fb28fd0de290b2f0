"""shockleaf: ShockHash leaf seed search on MI355X (gfx950).

Thin Python binding over the C ABI of libshockleaf.so (include/shockleaf.h).
Every step of the search runs in the library's HIP kernels; this module only
marshals torch device tensors (int64 tensors carry the uint64 key bits) and
options.  Importing it without the built library raises, and so does calling
it without a GPU: there is no fallback path.
"""
from .binding import (  # noqa: F401
    SHOCK_OK, SHOCK_EINVAL, SHOCK_ENOTFOUND, SHOCK_EDUPKEY, SHOCK_ECANCELED, SHOCK_EHIP, SHOCK_ENOMEM,
    SHOCK_MODE_AUTO, SHOCK_MODE_PLAIN_PER_LEAF, SHOCK_MODE_PERSISTENT, SHOCK_DEFAULT_MAX_SEED, NOT_FOUND_SEED,
    ShockError, lib, lib_path, exported_symbols, shock_leaf_search, shock_leaf_search_ex, shock_last_stats,
    shock_strerror, shock_spec_version, shock_release_scratch, leaf_search, SearchContext, make_opts,
    shock_rf_leaf_search_ex, rf_leaf_search, leaf_query, rf_leaf_query, rice_encode, rice_decode, MPHF,
    bip_leaf_search, leaf_search_noalloc, SHOCK_NOALLOC_MAX_LEAVES, SHOCK_NOALLOC_MAX_WORKERS,
    SHOCK_NOALLOC_SCRATCH_BYTES, SHOCK_EPENDING, leaf_search_async, rf_leaf_search_async, stream_status,
    RequestQueue, queue_batch_bytes,
)
