"""ctypes binding of libshockleaf.so: argument marshalling only."""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_PKG, "libshockleaf.so")

SHOCK_OK = 0
SHOCK_EINVAL = -1
SHOCK_ENOTFOUND = -2
SHOCK_EDUPKEY = -3
SHOCK_ECANCELED = -4
SHOCK_EHIP = -5
SHOCK_ENOMEM = -6
SHOCK_EPENDING = -7

SHOCK_RETRIEVAL_RIBBON = 0
SHOCK_RETRIEVAL_XOR = 1

SHOCK_MODE_AUTO = 0
SHOCK_MODE_PLAIN_PER_LEAF = 1
SHOCK_MODE_PERSISTENT = 2

SHOCK_DEFAULT_MAX_SEED = 1 << 32
NOT_FOUND_SEED = (1 << 64) - 1

# Names declared in include/shockleaf.h (checked by the CPU test suite).
EXPORTED = [
    "shock_opts_init", "shock_leaf_search", "shock_leaf_search_ex", "shock_last_stats",
    "shock_last_error", "shock_strerror", "shock_release_scratch", "shock_spec_version",
    "shock_ctx_create", "shock_ctx_destroy", "shock_ctx_search_async", "shock_ctx_query", "shock_ctx_wait",
    "shock_ctx_graph_capture", "shock_ctx_graph_launch", "shock_rf_leaf_search_ex", "shock_ctx_rf_search_async",
    "shock_leaf_query", "shock_rf_leaf_query", "shock_rice_encode", "shock_rice_decode",
    "shock_mphf_params_init", "shock_mphf_build", "shock_mphf_query", "shock_mphf_info", "shock_mphf_export",
    "shock_mphf_export_ribbon",
    "shock_mphf_destroy", "shock_bip_leaf_search_ex", "shock_leaf_search_noalloc",
    "shock_leaf_search_async", "shock_rf_leaf_search_async", "shock_stream_status", "shock_queue_params_init",
    "shock_queue_batch_bytes", "shock_queue_create", "shock_submit", "shock_poll", "shock_cancel",
    "shock_queue_stats_get", "shock_queue_destroy",
]

# Limits of shock_leaf_search_noalloc (include/shockleaf.h).
SHOCK_NOALLOC_MAX_LEAVES = 65536
SHOCK_NOALLOC_MAX_WORKERS = 32768
SHOCK_NOALLOC_SCRATCH_BYTES = 34 << 20


class ShockOpts(ctypes.Structure):
    _fields_ = [
        ("max_seed", ctypes.c_uint64),
        ("start_seed", ctypes.c_uint64),
        ("mode", ctypes.c_int32),
        ("spl", ctypes.c_int32),
        ("block_iters", ctypes.c_int32),
        ("waves_per_wg", ctypes.c_int32),
        ("workers", ctypes.c_int32),
        ("check_dups", ctypes.c_int32),
        ("cancel", ctypes.c_void_p),
        ("leaf_size_hint", ctypes.c_int32),
        ("partial_k", ctypes.c_int32),
        ("block_iters_by_n", ctypes.c_void_p),
        ("team", ctypes.c_int32),
        ("bip_pool", ctypes.c_int32),
        ("n_keys", ctypes.c_uint64),
    ]


class ShockStats(ctypes.Structure):
    _fields_ = [
        ("seeds_tested", ctypes.c_uint64),
        ("filter_passes", ctypes.c_uint64),
        ("pf_checks", ctypes.c_uint64),
        ("blocks_claimed", ctypes.c_uint64),
        ("kernel_ms", ctypes.c_double),
        ("workers", ctypes.c_int32),
        ("spl", ctypes.c_int32),
        ("block_iters", ctypes.c_int32),
        ("waves_per_wg", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BipStats(ctypes.Structure):
    _fields_ = [("seeds_hashed", ctypes.c_uint64), ("pairs_tested", ctypes.c_uint64), ("pairs_peeled", ctypes.c_uint64),
                ("kernel_ms", ctypes.c_double),
                ("workers", ctypes.c_int32), ("second_pass_leaves", ctypes.c_int32)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class QueueParams(ctypes.Structure):
    _fields_ = [
        ("device", ctypes.c_int32),
        ("slots", ctypes.c_int32),
        ("hbm_budget_bytes", ctypes.c_uint64),
        ("max_batch_leaves", ctypes.c_uint64),
        ("max_batch_keys", ctypes.c_uint64),
        ("search", ShockOpts),
    ]


class TicketInfo(ctypes.Structure):
    _fields_ = [("submit_ns", ctypes.c_int64), ("admit_ns", ctypes.c_int64), ("done_ns", ctypes.c_int64),
                ("batch", ctypes.c_uint64), ("n_leaves", ctypes.c_uint64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class QueueStats(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64), ("cancelled", ctypes.c_uint64),
        ("batches", ctypes.c_uint64), ("queued", ctypes.c_uint64), ("running", ctypes.c_uint64),
        ("bytes_in_flight", ctypes.c_uint64), ("max_bytes_in_flight", ctypes.c_uint64),
        ("batches_in_flight", ctypes.c_int32), ("max_batches_in_flight", ctypes.c_int32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class MphfParams(ctypes.Structure):
    _fields_ = [
        ("bucket_size", ctypes.c_uint32),
        ("leaf_target", ctypes.c_uint32),
        ("leaf_max", ctypes.c_uint32),
        ("max_rho_tries", ctypes.c_uint32),
        ("rice_k_by_n", ctypes.c_void_p),
        ("rotation_fitting", ctypes.c_uint32),
        ("partial_k", ctypes.c_int32),
        ("bipartite", ctypes.c_uint32),
        ("retrieval", ctypes.c_uint32),
        ("ribbon_rows", ctypes.c_uint32),
        ("reserved0", ctypes.c_uint32),
        ("reserved1", ctypes.c_uint64),
    ]


class MphfStats(ctypes.Structure):
    _fields_ = [
        ("n_keys", ctypes.c_uint64), ("n_buckets", ctypes.c_uint64), ("n_leaves", ctypes.c_uint64),
        ("rho", ctypes.c_uint64), ("seg", ctypes.c_uint64),
        ("max_sigma", ctypes.c_uint32), ("peel_rounds", ctypes.c_uint32),
        ("seed_fixed_bits", ctypes.c_uint64), ("seed_unary_bits", ctypes.c_uint64),
        ("bits_buckets", ctypes.c_uint64), ("bits_leaf_sizes", ctypes.c_uint64), ("bits_seeds", ctypes.c_uint64),
        ("bits_retrieval", ctypes.c_uint64), ("bits_total", ctypes.c_uint64),
        ("build_ms", ctypes.c_double), ("search_ms", ctypes.c_double),
        ("layout_ms", ctypes.c_double), ("search_call_ms", ctypes.c_double), ("codes_ms", ctypes.c_double),
        ("retrieval_ms", ctypes.c_double), ("rho_tries", ctypes.c_uint32), ("retrieval", ctypes.c_uint32),
        ("max_rseed", ctypes.c_uint32), ("ribbon_walked", ctypes.c_uint32),
    ]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class ShockError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"shockleaf status {status}: {msg}")
        self.status = status


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise ImportError(f"{_LIB_PATH} is missing: build it with paper_2308_09561_amd.build.build()")
        L = ctypes.CDLL(_LIB_PATH)
        vp = ctypes.c_void_p
        L.shock_opts_init.restype = None
        L.shock_opts_init.argtypes = [ctypes.POINTER(ShockOpts)]
        L.shock_leaf_search.restype = ctypes.c_int
        L.shock_leaf_search.argtypes = [vp, vp, ctypes.c_uint64, vp, vp]
        L.shock_leaf_search_ex.restype = ctypes.c_int
        L.shock_leaf_search_ex.argtypes = [vp, vp, ctypes.c_uint64, vp, vp, ctypes.POINTER(ShockOpts), vp]
        L.shock_leaf_search_noalloc.restype = ctypes.c_int
        L.shock_leaf_search_noalloc.argtypes = [vp, vp, ctypes.c_uint64, vp, vp, ctypes.POINTER(ShockOpts), vp]
        L.shock_last_stats.restype = ctypes.c_int
        L.shock_last_stats.argtypes = [ctypes.POINTER(ShockStats)]
        L.shock_last_error.restype = ctypes.c_char_p
        L.shock_last_error.argtypes = []
        L.shock_strerror.restype = ctypes.c_char_p
        L.shock_strerror.argtypes = [ctypes.c_int]
        L.shock_release_scratch.restype = ctypes.c_int
        L.shock_release_scratch.argtypes = []
        L.shock_spec_version.restype = ctypes.c_int
        L.shock_spec_version.argtypes = []
        L.shock_ctx_create.restype = ctypes.c_int
        L.shock_ctx_create.argtypes = [ctypes.c_uint64, ctypes.POINTER(vp)]
        L.shock_ctx_destroy.restype = ctypes.c_int
        L.shock_ctx_destroy.argtypes = [vp]
        L.shock_ctx_search_async.restype = ctypes.c_int
        L.shock_ctx_search_async.argtypes = [vp, vp, vp, ctypes.c_uint64, vp, vp, ctypes.POINTER(ShockOpts), vp]
        L.shock_ctx_graph_capture.restype = ctypes.c_int
        L.shock_ctx_graph_capture.argtypes = [vp, vp, vp, ctypes.c_uint64, vp, vp, ctypes.POINTER(ShockOpts), vp]
        L.shock_ctx_graph_launch.restype = ctypes.c_int
        L.shock_ctx_graph_launch.argtypes = [vp, vp]
        L.shock_rf_leaf_search_ex.restype = ctypes.c_int
        L.shock_rf_leaf_search_ex.argtypes = [vp, vp, ctypes.c_uint64, vp, vp, vp, ctypes.POINTER(ShockOpts), vp]
        L.shock_ctx_rf_search_async.restype = ctypes.c_int
        L.shock_ctx_rf_search_async.argtypes = [vp, vp, vp, ctypes.c_uint64, vp, vp, vp, ctypes.POINTER(ShockOpts),
                                                vp]
        L.shock_leaf_query.restype = ctypes.c_int
        L.shock_leaf_query.argtypes = [vp, vp, ctypes.c_uint64, vp, vp, vp, vp]
        L.shock_rf_leaf_query.restype = ctypes.c_int
        L.shock_rf_leaf_query.argtypes = [vp, vp, ctypes.c_uint64, vp, vp, vp, ctypes.c_int32, vp, vp]
        u64p = ctypes.POINTER(ctypes.c_uint64)
        L.shock_rice_encode.restype = ctypes.c_int
        L.shock_rice_encode.argtypes = [vp, vp, ctypes.c_uint64, vp, vp, ctypes.c_uint64, vp, ctypes.c_uint64, vp,
                                        u64p, vp]
        L.shock_rice_decode.restype = ctypes.c_int
        L.shock_rice_decode.argtypes = [vp, ctypes.c_uint64, vp, ctypes.c_uint64, vp, vp, ctypes.c_uint64, vp, vp, vp]
        L.shock_mphf_params_init.restype = None
        L.shock_mphf_params_init.argtypes = [ctypes.POINTER(MphfParams)]
        L.shock_mphf_build.restype = ctypes.c_int
        L.shock_mphf_build.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(MphfParams), ctypes.POINTER(vp), vp]
        L.shock_mphf_query.restype = ctypes.c_int
        L.shock_mphf_query.argtypes = [vp, vp, ctypes.c_uint64, vp, vp]
        L.shock_mphf_info.restype = ctypes.c_int
        L.shock_mphf_info.argtypes = [vp, ctypes.POINTER(MphfStats)]
        L.shock_mphf_export.restype = ctypes.c_int
        L.shock_mphf_export.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.shock_mphf_export_ribbon.restype = ctypes.c_int
        L.shock_mphf_export_ribbon.argtypes = [vp, vp, vp, vp]
        L.shock_mphf_destroy.restype = ctypes.c_int
        L.shock_mphf_destroy.argtypes = [vp]
        L.shock_bip_leaf_search_ex.restype = ctypes.c_int
        L.shock_bip_leaf_search_ex.argtypes = [vp, vp, ctypes.c_uint64, vp, vp, vp, ctypes.POINTER(ShockOpts), vp,
                                               ctypes.POINTER(BipStats)]
        L.shock_leaf_search_async.restype = ctypes.c_int
        L.shock_leaf_search_async.argtypes = [vp, vp, ctypes.c_uint64, vp, vp, ctypes.POINTER(ShockOpts), vp]
        L.shock_rf_leaf_search_async.restype = ctypes.c_int
        L.shock_rf_leaf_search_async.argtypes = [vp, vp, ctypes.c_uint64, vp, vp, vp, ctypes.POINTER(ShockOpts), vp]
        L.shock_stream_status.restype = ctypes.c_int
        L.shock_stream_status.argtypes = [vp]
        L.shock_queue_params_init.restype = None
        L.shock_queue_params_init.argtypes = [ctypes.POINTER(QueueParams)]
        L.shock_queue_batch_bytes.restype = ctypes.c_uint64
        L.shock_queue_batch_bytes.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
        L.shock_queue_create.restype = ctypes.c_int
        L.shock_queue_create.argtypes = [ctypes.POINTER(QueueParams), ctypes.POINTER(vp)]
        L.shock_submit.restype = ctypes.c_int
        L.shock_submit.argtypes = [vp, vp, vp, ctypes.c_uint64, vp, vp, ctypes.POINTER(ctypes.c_uint64)]
        L.shock_poll.restype = ctypes.c_int
        L.shock_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(TicketInfo)]
        L.shock_cancel.restype = ctypes.c_int
        L.shock_cancel.argtypes = [vp, ctypes.c_uint64]
        L.shock_queue_stats_get.restype = ctypes.c_int
        L.shock_queue_stats_get.argtypes = [vp, ctypes.POINTER(QueueStats)]
        L.shock_queue_destroy.restype = ctypes.c_int
        L.shock_queue_destroy.argtypes = [vp]
        L.shock_ctx_query.restype = ctypes.c_int
        L.shock_ctx_query.argtypes = [vp]
        L.shock_ctx_wait.restype = ctypes.c_int
        L.shock_ctx_wait.argtypes = [vp, ctypes.POINTER(ShockStats)]
        _lib = L
    return _lib


def exported_symbols():
    L = lib()
    return {name: hasattr(L, name) for name in EXPORTED}


def shock_strerror(status: int) -> str:
    return lib().shock_strerror(status).decode()


def shock_spec_version() -> int:
    return lib().shock_spec_version()


def shock_release_scratch() -> int:
    return lib().shock_release_scratch()


def shock_last_stats() -> dict:
    st = ShockStats()
    lib().shock_last_stats(ctypes.byref(st))
    return st.as_dict()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def shock_leaf_search(keys, offsets, n_leaves, out_seeds, out_orient) -> int:
    """C call with torch device tensors (or raw integer device addresses)."""
    return lib().shock_leaf_search(*(_as_ptr(x) for x in (keys, offsets)), n_leaves,
                                   _as_ptr(out_seeds), _as_ptr(out_orient))


def _as_ptr(x):
    if x is None:
        return None
    if isinstance(x, int):
        return ctypes.c_void_p(x)
    return ctypes.c_void_p(x.data_ptr())


def make_opts(max_seed=None, start_seed=0, mode=SHOCK_MODE_AUTO, spl=0, block_iters=0, waves_per_wg=0,
              workers=0, check_dups=False, cancel_ptr=None, leaf_size_hint=0, block_iters_by_n=None,
              partial_k=0, team=0, n_keys=0, bip_pool=0) -> ShockOpts:
    """shock_opts with defaults; block_iters_by_n is a sequence of 65 ints or None."""
    o = ShockOpts()
    lib().shock_opts_init(ctypes.byref(o))
    if max_seed is not None:
        o.max_seed = max_seed
    o.start_seed = start_seed
    o.mode = mode
    o.spl = spl
    o.block_iters = block_iters
    o.waves_per_wg = waves_per_wg
    o.workers = workers
    o.check_dups = int(bool(check_dups))
    o.cancel = cancel_ptr
    o.bip_pool = bip_pool
    o.leaf_size_hint = leaf_size_hint
    o.partial_k = partial_k
    o.team = team
    o.n_keys = n_keys
    if block_iters_by_n is not None:
        if len(block_iters_by_n) != 65:
            raise ValueError("block_iters_by_n needs 65 entries (leaf sizes 0..64)")
        table = (ctypes.c_uint16 * 65)(*[int(v) for v in block_iters_by_n])
        o._table = table  # keep alive with the options
        o.block_iters_by_n = ctypes.cast(table, ctypes.c_void_p)
    return o


def shock_leaf_search_ex(keys, offsets, n_leaves, out_seeds, out_orient, opts: ShockOpts | None = None,
                         stream=None) -> int:
    s = None if stream is None else ctypes.c_void_p(stream)
    return lib().shock_leaf_search_ex(_as_ptr(keys), _as_ptr(offsets), n_leaves, _as_ptr(out_seeds),
                                      _as_ptr(out_orient), None if opts is None else ctypes.byref(opts), s)


def shock_rf_leaf_search_ex(keys, offsets, n_leaves, out_seeds, out_rot, out_orient, opts: ShockOpts | None = None,
                            stream=None) -> int:
    s = None if stream is None else ctypes.c_void_p(stream)
    return lib().shock_rf_leaf_search_ex(_as_ptr(keys), _as_ptr(offsets), n_leaves, _as_ptr(out_seeds),
                                         _as_ptr(out_rot), _as_ptr(out_orient),
                                         None if opts is None else ctypes.byref(opts), s)


def rf_leaf_search(keys, offsets, out_seeds=None, out_rot=None, out_orient=None, stream=None, **opts):
    """Rotation-fitting search of a CSR batch in torch int64 CUDA tensors.

    Returns (status, seeds, rotations, orient): seeds/orient int64 tensors
    (uint64 bit patterns), rotations an int32 tensor, all on the keys' device.
    """
    import torch

    keys, offsets, L = _batch(keys, offsets)
    dev = keys.device
    if out_seeds is None:
        out_seeds = torch.empty(max(L, 1), dtype=torch.int64, device=dev)
    if out_rot is None:
        out_rot = torch.empty(max(L, 1), dtype=torch.int32, device=dev)
    if out_orient is None:
        out_orient = torch.empty(max(L, 1), dtype=torch.int64, device=dev)
    _check_out(out_seeds, L, torch.int64, dev, "out_seeds")
    _check_out(out_rot, L, torch.int32, dev, "out_rot")
    _check_out(out_orient, L, torch.int64, dev, "out_orient")
    if stream is None:
        stream = torch.cuda.current_stream(dev).cuda_stream
    o = make_opts(n_keys=keys.numel(), **opts)
    rc = shock_rf_leaf_search_ex(keys if keys.numel() else offsets, offsets, L, out_seeds, out_rot, out_orient, o,
                                 stream)
    if rc in (SHOCK_EHIP, SHOCK_ENOMEM):
        raise ShockError(rc, lib().shock_last_error().decode())
    return rc, out_seeds[:L], out_rot[:L], out_orient[:L]


def leaf_search(keys, offsets, out_seeds=None, out_orient=None, stream=None, **opts):
    """Search a CSR batch held in torch int64 CUDA tensors.

    Returns (status, seeds, orient) with seeds/orient int64 tensors on the same
    device (uint64 bit patterns).  Raises ShockError on SHOCK_EHIP/SHOCK_ENOMEM.
    """
    import torch

    keys, offsets, L = _batch(keys, offsets)
    if out_seeds is None:
        out_seeds = torch.empty(max(L, 1), dtype=torch.int64, device=keys.device)
    if out_orient is None:
        out_orient = torch.empty(max(L, 1), dtype=torch.int64, device=keys.device)
    _check_out(out_seeds, L, torch.int64, keys.device, "out_seeds")
    _check_out(out_orient, L, torch.int64, keys.device, "out_orient")
    if stream is None:
        stream = torch.cuda.current_stream(keys.device).cuda_stream
    o = make_opts(n_keys=keys.numel(), **opts)
    rc = shock_leaf_search_ex(keys if keys.numel() else offsets, offsets, L, out_seeds, out_orient, o, stream)
    if rc in (SHOCK_EHIP, SHOCK_ENOMEM):
        raise ShockError(rc, lib().shock_last_error().decode())
    return rc, out_seeds[:L], out_orient[:L]


def leaf_search_noalloc(keys, offsets, out_seeds, out_orient, stream=None, **opts):
    """shock_leaf_search_noalloc: the persistent search with the library's
    fixed per-GPU scratch array (no device allocation in the call).  The
    caller passes the output tensors (int64, at least n_leaves entries).
    Returns the status; raises ShockError on SHOCK_EHIP."""
    import torch

    keys, offsets, L = _batch(keys, offsets)
    _check_out(out_seeds, L, torch.int64, keys.device, "out_seeds")
    _check_out(out_orient, L, torch.int64, keys.device, "out_orient")
    if stream is None:
        stream = torch.cuda.current_stream(keys.device).cuda_stream
    o = make_opts(n_keys=keys.numel(), **opts)
    rc = lib().shock_leaf_search_noalloc(_as_ptr(keys if keys.numel() else offsets), _as_ptr(offsets), L,
                                         _as_ptr(out_seeds), _as_ptr(out_orient), ctypes.byref(o),
                                         ctypes.c_void_p(stream))
    if rc == SHOCK_EHIP:
        raise ShockError(rc, lib().shock_last_error().decode())
    return rc


def leaf_search_async(keys, offsets, out_seeds, out_orient, stream=None, **opts) -> int:
    """shock_leaf_search_async: enqueue the search on `stream` (default: the
    current torch stream) and return at once; the batch's status comes from
    stream_status(stream) once the stream has passed it.  Keep every tensor
    alive until then."""
    import torch

    keys, offsets, L = _batch(keys, offsets)
    _check_out(out_seeds, L, torch.int64, keys.device, "out_seeds")
    _check_out(out_orient, L, torch.int64, keys.device, "out_orient")
    if stream is None:
        stream = torch.cuda.current_stream(keys.device).cuda_stream
    o = make_opts(n_keys=keys.numel(), **opts)
    rc = lib().shock_leaf_search_async(_as_ptr(keys if keys.numel() else offsets), _as_ptr(offsets), L,
                                       _as_ptr(out_seeds), _as_ptr(out_orient), ctypes.byref(o),
                                       ctypes.c_void_p(stream))
    if rc in (SHOCK_EHIP, SHOCK_ENOMEM):
        raise ShockError(rc, lib().shock_last_error().decode())
    return rc


def rf_leaf_search_async(keys, offsets, out_seeds, out_rot, out_orient, stream=None, **opts) -> int:
    """shock_rf_leaf_search_async (see leaf_search_async); out_rot int32."""
    import torch

    keys, offsets, L = _batch(keys, offsets)
    _check_out(out_seeds, L, torch.int64, keys.device, "out_seeds")
    _check_out(out_rot, L, torch.int32, keys.device, "out_rot")
    _check_out(out_orient, L, torch.int64, keys.device, "out_orient")
    if stream is None:
        stream = torch.cuda.current_stream(keys.device).cuda_stream
    o = make_opts(n_keys=keys.numel(), **opts)
    rc = lib().shock_rf_leaf_search_async(_as_ptr(keys if keys.numel() else offsets), _as_ptr(offsets), L,
                                          _as_ptr(out_seeds), _as_ptr(out_rot), _as_ptr(out_orient),
                                          ctypes.byref(o), ctypes.c_void_p(stream))
    if rc in (SHOCK_EHIP, SHOCK_ENOMEM):
        raise ShockError(rc, lib().shock_last_error().decode())
    return rc


def stream_status(stream) -> int:
    """shock_stream_status of a raw stream handle (e.g. torch's cuda_stream)."""
    return lib().shock_stream_status(ctypes.c_void_p(stream))


def queue_batch_bytes(n_leaves: int, n_keys: int) -> int:
    """Device bytes a batch holds in a RequestQueue's arena."""
    return int(lib().shock_queue_batch_bytes(n_leaves, n_keys))


class RequestQueue:
    """A shock_queue: host-side build requests (CSR leaves in numpy uint64
    arrays) searched on one device under an HBM budget by the library's
    dispatcher thread.  submit() returns a ticket; poll() reports completion
    and hands back the results."""

    def __init__(self, device: int = 0, hbm_budget_bytes: int = 256 << 20, slots: int = 4,
                 max_batch_leaves: int = 65536, max_batch_keys: int = 1 << 22, **search_opts):
        p = QueueParams()
        lib().shock_queue_params_init(ctypes.byref(p))
        p.device = device
        p.slots = slots
        p.hbm_budget_bytes = hbm_budget_bytes
        p.max_batch_leaves = max_batch_leaves
        p.max_batch_keys = max_batch_keys
        p.search = make_opts(**search_opts)
        self._h = ctypes.c_void_p()
        rc = lib().shock_queue_create(ctypes.byref(p), ctypes.byref(self._h))
        if rc != SHOCK_OK:
            raise ShockError(rc, lib().shock_last_error().decode())
        self._live = {}  # ticket -> (keys, offsets, seeds, orient): kept alive until polled done

    def submit(self, keys, offsets):
        """(status, ticket): keys and offsets numpy uint64 (host).  SHOCK_ENOMEM
        for a request larger than the budget or a batch's limits."""
        import numpy as np

        keys = np.ascontiguousarray(keys, dtype=np.uint64)
        offsets = np.ascontiguousarray(offsets, dtype=np.uint64)
        L = len(offsets) - 1
        if L < 0:
            raise ValueError("offsets needs n_leaves + 1 entries")
        seeds = np.empty(max(L, 1), dtype=np.uint64)
        orient = np.empty(max(L, 1), dtype=np.uint64)
        t = ctypes.c_uint64()
        rc = lib().shock_submit(self._h, keys.ctypes.data if keys.size else None, offsets.ctypes.data, L,
                                seeds.ctypes.data, orient.ctypes.data, ctypes.byref(t))
        if rc != SHOCK_OK:
            return rc, None
        self._live[t.value] = (keys, offsets, seeds[:L], orient[:L])
        return rc, t.value

    def poll(self, ticket):
        """(done, status, info dict or None, seeds, orient); results only once done."""
        done = ctypes.c_int()
        info = TicketInfo()
        rc = lib().shock_poll(self._h, ticket, ctypes.byref(done), ctypes.byref(info))
        if not done.value:
            return False, rc, None, None, None
        _, _, seeds, orient = self._live.pop(ticket)
        return True, rc, info.as_dict(), seeds, orient

    def cancel(self, ticket) -> int:
        return lib().shock_cancel(self._h, ticket)

    def stats(self) -> dict:
        st = QueueStats()
        lib().shock_queue_stats_get(self._h, ctypes.byref(st))
        return st.as_dict()

    def close(self):
        if self._h:
            lib().shock_queue_destroy(self._h)
            self._h = ctypes.c_void_p()
            self._live.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _check_tensors(keys, offsets):
    import torch

    if keys.device.type != "cuda" or offsets.device.type != "cuda":
        raise ValueError("keys and offsets must be device (cuda) tensors")
    if keys.device != offsets.device:
        raise ValueError("keys and offsets must be on the same device")
    if keys.dtype != torch.int64 or offsets.dtype != torch.int64:
        raise ValueError("keys and offsets must be int64 tensors carrying uint64 bits")


def _batch(keys, offsets):
    """Checked, contiguous (keys, offsets, n_leaves) of a CSR batch.  The
    library itself rejects leaves reaching past the keys (n_keys option)."""
    _check_tensors(keys, offsets)
    if keys.dim() != 1 or offsets.dim() != 1:
        raise ValueError("keys and offsets must be one-dimensional")
    keys = keys.contiguous()
    offsets = offsets.contiguous()
    L = offsets.numel() - 1
    if L < 0:
        raise ValueError("offsets needs n_leaves + 1 entries")
    if keys.numel() == 0 and L > 0 and bool(offsets.ne(0).any()):
        # n_keys = 0 would mean "unchecked": a batch of empty leaves only
        raise ValueError("the keys buffer is empty but the offsets give leaves keys")
    return keys, offsets, L


def _check_out(t, L, dtype, device, name):
    """An output tensor the kernels may write L entries of."""
    if t.dtype != dtype:
        raise ValueError(f"{name} must be a {dtype} tensor")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.numel() < L:
        raise ValueError(f"{name} holds {t.numel()} entries, the batch has {L} leaves")


class SearchContext:
    """A shock_ctx: asynchronous searches on a stream, and captured graphs.

    Buffers passed to search_async/capture must stay alive until wait()."""

    def __init__(self, max_leaves: int):
        self._h = ctypes.c_void_p()
        rc = lib().shock_ctx_create(max_leaves, ctypes.byref(self._h))
        if rc != SHOCK_OK:
            raise ShockError(rc, lib().shock_last_error().decode())
        self.max_leaves = max_leaves
        self._keep = None

    def close(self):
        if self._h:
            lib().shock_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _args(self, keys, offsets, out_seeds, out_orient, stream, opts):
        import torch

        keys, offsets, L = _batch(keys, offsets)
        _check_out(out_seeds, L, torch.int64, keys.device, "out_seeds")
        _check_out(out_orient, L, torch.int64, keys.device, "out_orient")
        if stream is None:
            stream = torch.cuda.current_stream(keys.device).cuda_stream
        o = make_opts(n_keys=keys.numel(), **opts)
        self._keep = (keys, offsets, out_seeds, out_orient, o)
        return (self._h, _as_ptr(keys), _as_ptr(offsets), L, _as_ptr(out_seeds), _as_ptr(out_orient),
                ctypes.byref(o), ctypes.c_void_p(stream))

    def search_async(self, keys, offsets, out_seeds, out_orient, stream=None, **opts) -> int:
        return lib().shock_ctx_search_async(*self._args(keys, offsets, out_seeds, out_orient, stream, opts))

    def capture(self, keys, offsets, out_seeds, out_orient, stream=None, **opts) -> int:
        return lib().shock_ctx_graph_capture(*self._args(keys, offsets, out_seeds, out_orient, stream, opts))

    def launch_graph(self, stream=None) -> int:
        import torch

        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        return lib().shock_ctx_graph_launch(self._h, ctypes.c_void_p(stream))

    def rf_search_async(self, keys, offsets, out_seeds, out_rot, out_orient, stream=None, **opts) -> int:
        """Rotation-fitting search; out_rot an int32 device tensor."""
        import torch

        a = self._args(keys, offsets, out_seeds, out_orient, stream, opts)
        _check_out(out_rot, a[3], torch.int32, keys.device, "out_rot")
        self._keep = self._keep + (out_rot,)
        return lib().shock_ctx_rf_search_async(*a[:5], _as_ptr(out_rot), *a[5:])

    def query(self) -> int:
        return lib().shock_ctx_query(self._h)

    def wait(self):
        """(status, stats dict) of the last search."""
        st = ShockStats()
        rc = lib().shock_ctx_wait(self._h, ctypes.byref(st))
        if rc in (SHOCK_EHIP, SHOCK_ENOMEM):
            raise ShockError(rc, lib().shock_last_error().decode())
        return rc, st.as_dict()


# ---- queries and Golomb-Rice seed codes (include/shockcode.h) ---------------

def _stream_of(t, stream):
    import torch
    return ctypes.c_void_p(stream if stream is not None else torch.cuda.current_stream(t.device).cuda_stream)


def _query_out(keys, offsets, out_pos):
    """The output tensor: the caller's (any length >= offsets[-1], returned
    as given, no host sync) or a new one sized from offsets[-1]."""
    import torch
    if out_pos is not None:
        return out_pos, out_pos
    N = int(offsets[-1].item()) if offsets.numel() else 0
    buf = torch.empty(max(N, 1), dtype=torch.int64, device=keys.device)
    return buf, buf[:N]


def leaf_query(keys, offsets, seeds, orient, out_pos=None, stream=None):
    """(status, positions) for a CSR batch: int64 device tensors in, an int64
    tensor of offsets[-1] global positions out (uint64 bit patterns)."""
    _check_tensors(keys, offsets)
    L = offsets.numel() - 1
    buf, ret = _query_out(keys, offsets, out_pos)
    rc = lib().shock_leaf_query(_as_ptr(keys if keys.numel() else offsets), _as_ptr(offsets), max(L, 0),
                                _as_ptr(seeds), _as_ptr(orient), _as_ptr(buf), _stream_of(keys, stream))
    return rc, ret


def rf_leaf_query(keys, offsets, seeds, rot, orient, partial_k=0, out_pos=None, stream=None):
    """leaf_query under rotation fitting; rot an int32 device tensor."""
    _check_tensors(keys, offsets)
    L = offsets.numel() - 1
    buf, ret = _query_out(keys, offsets, out_pos)
    rc = lib().shock_rf_leaf_query(_as_ptr(keys if keys.numel() else offsets), _as_ptr(offsets), max(L, 0),
                                   _as_ptr(seeds), _as_ptr(rot), _as_ptr(orient), partial_k, _as_ptr(buf),
                                   _stream_of(keys, stream))
    return rc, ret


def _table(k_by_n):
    if len(k_by_n) != 65:
        raise ValueError("k_by_n needs 65 entries (leaf sizes 0..64)")
    return (ctypes.c_uint8 * 65)(*[int(v) for v in k_by_n])


def rice_encode(values, offsets, k_by_n, stream=None):
    """Golomb-Rice code one value per leaf.  Returns (status, fixed, unary,
    index, (fixed_bits, unary_bits)) with int64 device tensors; a first call
    with empty streams sizes them."""
    import torch
    dev = offsets.device
    L = offsets.numel() - 1
    table = _table(k_by_n)
    bits = (ctypes.c_uint64 * 2)()
    index = torch.zeros(2 * ((L + 63) // 64 + 1), dtype=torch.int64, device=dev)
    st = _stream_of(offsets, stream)
    vals = _as_ptr(values) if L > 0 else None
    rc = lib().shock_rice_encode(vals, _as_ptr(offsets), L, table, None, 0, None, 0, _as_ptr(index), bits, st)
    if rc not in (SHOCK_OK, SHOCK_EINVAL):
        raise ShockError(rc, lib().shock_last_error().decode())
    fw, uw = (int(bits[0]) + 63) // 64, (int(bits[1]) + 63) // 64
    fixed = torch.empty(max(fw, 1), dtype=torch.int64, device=dev)
    unary = torch.empty(max(uw, 1), dtype=torch.int64, device=dev)
    rc = lib().shock_rice_encode(vals, _as_ptr(offsets), L, table, _as_ptr(fixed), fw, _as_ptr(unary), uw,
                                 _as_ptr(index), bits, st)
    if rc in (SHOCK_EHIP, SHOCK_ENOMEM):
        raise ShockError(rc, lib().shock_last_error().decode())
    return rc, fixed[:fw], unary[:uw], index, (int(bits[0]), int(bits[1]))


def rice_decode(fixed, unary, index, offsets, k_by_n, out_values=None, stream=None):
    """(status, values) decoded on the device; values an int64 tensor."""
    import torch
    L = offsets.numel() - 1
    if out_values is None:
        out_values = torch.empty(max(L, 1), dtype=torch.int64, device=offsets.device)
    rc = lib().shock_rice_decode(_as_ptr(fixed) if fixed.numel() else None, fixed.numel(),
                                 _as_ptr(unary) if unary.numel() else None, unary.numel(), _as_ptr(index),
                                 _as_ptr(offsets), max(L, 0), _table(k_by_n), _as_ptr(out_values),
                                 _stream_of(offsets, stream))
    return rc, out_values[:max(L, 0)]


# ---- flat ShockHash MPHF (include/shockmphf.h) ---------------------------------

class MPHF:
    """A minimal perfect hash function of distinct uint64 keys, built and
    queried on the GPU.  Raises ShockError if the build fails."""

    def __init__(self, keys, bucket_size=3000, leaf_target=40, leaf_max=56, rice_table=None, stream=None,
                 rotation_fitting=False, partial_k=0, bipartite=False, retrieval=SHOCK_RETRIEVAL_RIBBON,
                 ribbon_rows=0):
        import numpy as np
        if keys.device.type != "cuda" or keys.dtype.itemsize != 8:
            raise ValueError("keys must be a 64-bit device tensor")
        if rice_table is None:
            from .rice import plain_table
            rice_table = plain_table()
        keys = keys.contiguous()
        p = MphfParams()
        lib().shock_mphf_params_init(ctypes.byref(p))
        p.bucket_size, p.leaf_target, p.leaf_max = bucket_size, leaf_target, leaf_max
        p.rotation_fitting, p.partial_k = int(bool(rotation_fitting)), partial_k
        p.bipartite = int(bool(bipartite))
        p.retrieval = retrieval
        p.ribbon_rows = ribbon_rows
        table = _table(rice_table)
        p.rice_k_by_n = ctypes.cast(table, ctypes.c_void_p)
        self._h = ctypes.c_void_p()
        self.rice_table = [int(v) for v in rice_table]
        rc = lib().shock_mphf_build(_as_ptr(keys) if keys.numel() else None, keys.numel(), ctypes.byref(p),
                                    ctypes.byref(self._h), _stream_of(keys, stream))
        self.status = rc
        if rc != SHOCK_OK:
            raise ShockError(rc, shock_strerror(rc) + " / " + lib().shock_last_error().decode())
        self.n_keys = keys.numel()
        self._np = np

    def query(self, queries, out=None, stream=None):
        """Positions (an int64 device tensor) of the query keys."""
        import torch
        if out is None:
            out = torch.empty(max(queries.numel(), 1), dtype=torch.int64, device=queries.device)
        rc = lib().shock_mphf_query(self._h, _as_ptr(queries) if queries.numel() else None, queries.numel(),
                                    _as_ptr(out), _stream_of(queries, stream))
        if rc != SHOCK_OK:
            raise ShockError(rc, shock_strerror(rc))
        return out[:queries.numel()]

    def info(self) -> dict:
        st = MphfStats()
        lib().shock_mphf_info(self._h, ctypes.byref(st))
        d = st.as_dict()
        d["bits_per_key"] = d["bits_total"] / max(d["n_keys"], 1)
        return d

    def export(self) -> dict:
        """The stored parts as numpy arrays (leaf seeds decoded)."""
        np = self._np
        st = self.info()
        B, L = st["n_buckets"], st["n_leaves"]
        bo = np.zeros(B + 1, np.uint64)
        lb = np.zeros(B + 1, np.uint64)
        sg = np.zeros(max(B, 1), np.uint32)
        sz = np.zeros(max(L, 1), np.uint8)
        sd = np.zeros(max(L, 1), np.uint64)
        xor = st["retrieval"] == SHOCK_RETRIEVAL_XOR
        z = np.zeros(max(3 * st["seg"], 1), np.uint8)
        rc = lib().shock_mphf_export(self._h, bo.ctypes.data, lb.ctypes.data, sg.ctypes.data, sz.ctypes.data,
                                     sd.ctypes.data, z.ctypes.data if xor else None)
        if rc != SHOCK_OK:
            raise ShockError(rc, shock_strerror(rc))
        out = {"bucket_offset": bo, "leaf_base": lb, "sigma": sg[:B], "leaf_sizes": sz[:L], "seeds": sd[:L],
               "rho": st["rho"], "seg": st["seg"], "retrieval": st["retrieval"]}
        if xor:
            out["z"] = z[:3 * st["seg"]]
        else:
            rs = np.zeros(max(B, 1), np.uint8)
            rb = np.zeros(B + 1, np.uint64)
            lib().shock_mphf_export_ribbon(self._h, rs.ctypes.data, rb.ctypes.data, None)
            bits = np.zeros(max(int(rb[-1]), 1), np.uint8)
            rc = lib().shock_mphf_export_ribbon(self._h, None, None, bits.ctypes.data)
            if rc != SHOCK_OK:
                raise ShockError(rc, shock_strerror(rc))
            out.update({"rseed": rs[:B], "rbit_offset": rb, "z": bits[:int(rb[-1])]})
        return out

    def close(self):
        if getattr(self, "_h", None):
            lib().shock_mphf_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bip_leaf_search(keys, offsets, out_a=None, out_b=None, out_orient=None, stream=None, **opts):
    """Bipartite ShockHash over a CSR batch in int64 CUDA tensors.  Returns
    (status, a, b, orient, stats): seed pairs and orientations as int64
    tensors (uint64 bit patterns) and a dict of device counters."""
    import torch
    keys, offsets, L = _batch(keys, offsets)
    dev = keys.device
    out_a = torch.empty(max(L, 1), dtype=torch.int64, device=dev) if out_a is None else out_a
    out_b = torch.empty(max(L, 1), dtype=torch.int64, device=dev) if out_b is None else out_b
    out_orient = torch.empty(max(L, 1), dtype=torch.int64, device=dev) if out_orient is None else out_orient
    for t, name in ((out_a, "out_a"), (out_b, "out_b"), (out_orient, "out_orient")):
        _check_out(t, L, torch.int64, dev, name)
    o = make_opts(n_keys=keys.numel(), **opts)
    st = BipStats()
    rc = lib().shock_bip_leaf_search_ex(_as_ptr(keys if keys.numel() else offsets), _as_ptr(offsets), max(L, 0),
                                        _as_ptr(out_a), _as_ptr(out_b), _as_ptr(out_orient), ctypes.byref(o),
                                        _stream_of(keys, stream), ctypes.byref(st))
    if rc in (SHOCK_EHIP, SHOCK_ENOMEM):
        raise ShockError(rc, lib().shock_last_error().decode())
    return rc, out_a[:L], out_b[:L], out_orient[:L], st.as_dict()

