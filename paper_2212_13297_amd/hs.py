"""Python binding of the C ABI in ``include/hs.h`` (ctypes; argument marshalling only).

The functions ``hs_*`` below carry the C names and signatures; ``Index`` wraps
them for callers that hold data in torch tensors.  torch supplies device
memory and the stream; every step of the search runs in the HIP library.
Nothing here falls back to a CPU path: if the library is not built, loading
raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhercules_hip.so")

HS_OK = 0
HS_EINVAL = -1
HS_ENOMEM = -2
HS_EHIP = -3
HS_EBUSY = -4
HS_ECANCEL = -5
HS_KMAX = 128
HS_SHADOW_BF16 = 1
HS_SHADOW_FP16 = 2


HS_BUILD_HOST_PARTITION = 1


class hs_params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("w", ctypes.c_int32), ("card_bits", ctypes.c_int32),
                ("leaf_size", ctypes.c_int32), ("l_max", ctypes.c_int32), ("seed_rows", ctypes.c_int32),
                ("eapca_th", ctypes.c_float), ("cand_per_query", ctypes.c_int32), ("build_flags", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class hs_index_info(ctypes.Structure):
    _fields_ = [("n_series", ctypes.c_int64), ("n", ctypes.c_int32), ("w", ctypes.c_int32),
                ("row_stride", ctypes.c_int32), ("word_stride", ctypes.c_int32), ("n_leaves", ctypes.c_int64),
                ("max_leaf", ctypes.c_int64), ("index_bytes", ctypes.c_int64), ("n_chunks", ctypes.c_int64),
                ("sigma_step", ctypes.c_double)]


class hs_query_stats(ctypes.Structure):
    _fields_ = [("leaves_kept", ctypes.c_uint64), ("rows_filtered", ctypes.c_uint64),
                ("rows_refined", ctypes.c_uint64), ("chunks_read", ctypes.c_uint64), ("path", ctypes.c_uint64),
                ("rounds", ctypes.c_uint64), ("candidates", ctypes.c_uint64), ("chunks_tested", ctypes.c_uint64),
                ("rows_bounded", ctypes.c_uint64), ("bound_pairs", ctypes.c_uint64),
                ("rows_sigma", ctypes.c_uint64)]


class hs_server_config(ctypes.Structure):
    _fields_ = [("streams_per_coll", ctypes.c_int32), ("max_slots", ctypes.c_int32), ("max_batch", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class hs_completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("coll", ctypes.c_int32), ("k", ctypes.c_int32),
                ("status", ctypes.c_int32), ("batch", ctypes.c_int32), ("t_submit", ctypes.c_double),
                ("t_launch", ctypes.c_double), ("t_done", ctypes.c_double), ("ids", ctypes.c_int64 * HS_KMAX),
                ("d2", ctypes.c_float * HS_KMAX), ("err", ctypes.c_double * HS_KMAX)]


class hs_server_stats(ctypes.Structure):
    _fields_ = [("in_system", ctypes.c_int64), ("batches", ctypes.c_int64), ("queries", ctypes.c_int64),
                ("padded_queries", ctypes.c_int64), ("graphs", ctypes.c_int64), ("failed", ctypes.c_int64)]


STATS_FIELDS = [f for f, _ in hs_query_stats._fields_]

_P = ctypes.c_void_p
_SIGS = {
    "hs_index_bytes": (ctypes.c_int32, [ctypes.c_int64, ctypes.POINTER(hs_params), ctypes.POINTER(ctypes.c_int64)]),
    "hs_build_summaries": (ctypes.c_int32, [_P, ctypes.c_int64, ctypes.POINTER(hs_params), _P, ctypes.c_int64, _P,
                                            ctypes.POINTER(_P)]),
    "hs_get_info": (ctypes.c_int32, [_P, ctypes.POINTER(hs_index_info)]),
    "hs_build_begin": (ctypes.c_int32, [ctypes.c_int64, ctypes.POINTER(hs_params), _P, ctypes.c_int64, _P,
                                        ctypes.POINTER(_P)]),
    "hs_build_add_stats": (ctypes.c_int32, [_P, _P, ctypes.c_int64, ctypes.c_int64]),
    "hs_build_partition": (ctypes.c_int32, [_P]),
    "hs_build_add_rows": (ctypes.c_int32, [_P, _P, ctypes.c_int64, ctypes.c_int64]),
    "hs_build_finish": (ctypes.c_int32, [_P, ctypes.POINTER(_P)]),
    "hs_build_abort": (ctypes.c_int32, [_P]),
    "hs_get_leaves": (ctypes.c_int32, [_P, _P, _P]),
    "hs_get_chunks": (ctypes.c_int32, [_P, _P, _P]),
    "hs_query_workspace_bytes": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int64)]),
    "hs_knn_exact": (ctypes.c_int32, [_P, _P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int64, _P, _P, _P, _P,
                                      _P]),
    "hs_knn_exact_noalloc": (ctypes.c_int32, [_P, _P, ctypes.c_int32, ctypes.c_int32, _P, _P, _P, _P, _P]),
    "hs_shadow_bytes": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64)]),
    "hs_build_shadow": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int64, _P, ctypes.c_int64, _P]),
    "hs_knn_mixed": (ctypes.c_int32, [_P, _P, ctypes.c_int32, ctypes.c_int32, _P, ctypes.c_int64, _P, _P, _P, _P,
                                      _P]),
    "hs_server_create": (ctypes.c_int32, [_P, _P, ctypes.c_int32, _P, ctypes.c_int64,
                                          ctypes.POINTER(hs_server_config), ctypes.POINTER(_P)]),
    "hs_submit": (ctypes.c_int32, [_P, ctypes.c_int32, _P, ctypes.c_int32, ctypes.c_uint64]),
    "hs_poll": (ctypes.c_int32, [_P, _P, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "hs_cancel": (ctypes.c_int32, [_P, ctypes.c_uint64]),
    "hs_sched_cancel": (ctypes.c_int32, [_P, ctypes.c_uint64]),
    "hs_server_info": (ctypes.c_int32, [_P, ctypes.POINTER(hs_server_stats)]),
    "hs_server_destroy": (ctypes.c_int32, [_P]),
    "hs_server_now": (ctypes.c_double, []),
    "hs_sched_create": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, ctypes.POINTER(_P)]),
    "hs_sched_submit": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64]),
    "hs_sched_next": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                       ctypes.POINTER(ctypes.c_int32), _P, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_int32)]),
    "hs_sched_complete": (ctypes.c_int32, [_P, ctypes.c_int32, ctypes.c_int32]),
    "hs_sched_in_system": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int32)]),
    "hs_sched_destroy": (ctypes.c_int32, [_P]),
    "hs_index_free": (ctypes.c_int32, [_P]),
    "hs_last_error": (ctypes.c_char_p, []),
    "hs_breakpoints": (ctypes.c_int32, [ctypes.c_int32, _P]),
    "hs_profile_enable": (ctypes.c_int32, [ctypes.c_int32]),
    "hs_profile_read": (ctypes.c_int32, [ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]),
    "hs_read_probe": (ctypes.c_int32, [_P, ctypes.c_int64, ctypes.c_int32, _P, _P, ctypes.POINTER(ctypes.c_double)]),
    "hs_lds_probe": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, _P, _P,
                                      ctypes.POINTER(ctypes.c_double)]),
    "hs_union_bytes": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int64)]),
    "hs_union_enable": (ctypes.c_int32, [_P, ctypes.c_int64]),
    "hs_union_count": (ctypes.c_int32, [_P, _P, _P, _P]),
}

_LIB = None


def load():
    """Load the built HIP library (raises if it has not been built)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} (run __graft_entry__.build())")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib
    return _LIB


class HSError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"hs error {code}: {msg}")
        self.code = code


def _check(code):
    if code != HS_OK:
        raise HSError(code, load().hs_last_error().decode())


# ---------------------------------------------------------------- C names

def hs_index_bytes(N: int, params: hs_params) -> int:
    out = ctypes.c_int64()
    _check(load().hs_index_bytes(N, ctypes.byref(params), ctypes.byref(out)))
    return out.value


def hs_build_summaries(x_ptr: int, N: int, params: hs_params, mem_ptr: int, mem_bytes: int, stream: int):
    h = _P()
    _check(load().hs_build_summaries(x_ptr, N, ctypes.byref(params), mem_ptr, mem_bytes, stream, ctypes.byref(h)))
    return h


def hs_build_begin(N: int, params: hs_params, mem_ptr: int, mem_bytes: int, stream: int):
    b = _P()
    _check(load().hs_build_begin(N, ctypes.byref(params), mem_ptr, mem_bytes, stream, ctypes.byref(b)))
    return b


def hs_build_add_stats(b, x_ptr: int, row0: int, rows: int) -> None:
    _check(load().hs_build_add_stats(b, x_ptr, row0, rows))


def hs_build_partition(b) -> None:
    _check(load().hs_build_partition(b))


def hs_build_add_rows(b, x_ptr: int, row0: int, rows: int) -> None:
    _check(load().hs_build_add_rows(b, x_ptr, row0, rows))


def hs_build_finish(b):
    h = _P()
    _check(load().hs_build_finish(b, ctypes.byref(h)))
    return h


def hs_build_abort(b) -> None:
    _check(load().hs_build_abort(b))


def hs_get_info(h) -> hs_index_info:
    info = hs_index_info()
    _check(load().hs_get_info(h, ctypes.byref(info)))
    return info


def hs_get_leaves(h, info: hs_index_info):
    import numpy as np
    ls = np.empty(info.n_leaves + 1, dtype=np.int64)
    env = np.empty((info.n_leaves, info.w, 4), dtype=np.float32)
    _check(load().hs_get_leaves(h, ls.ctypes.data, env.ctypes.data))
    return ls, env


def hs_get_chunks(h, info: hs_index_info):
    import numpy as np
    cs = np.empty(info.n_chunks + 1, dtype=np.int64)
    cenv = np.empty((info.n_chunks, info.w, 4), dtype=np.float32)
    _check(load().hs_get_chunks(h, cs.ctypes.data, cenv.ctypes.data))
    return cs, cenv


def hs_query_workspace_bytes(h, Q: int, k: int) -> int:
    out = ctypes.c_int64()
    _check(load().hs_query_workspace_bytes(h, Q, k, ctypes.byref(out)))
    return out.value


def hs_knn_exact(h, q_ptr: int, Q: int, k: int, ws_ptr: int, ws_bytes: int, ids_ptr: int, d2_ptr: int,
                 err_ptr: int, stats_ptr: int, stream: int) -> None:
    _check(load().hs_knn_exact(h, q_ptr, Q, k, ws_ptr, ws_bytes, ids_ptr, d2_ptr, err_ptr, stats_ptr, stream))


def hs_knn_exact_noalloc(h, q_ptr: int, Q: int, k: int, ids_ptr: int, d2_ptr: int, err_ptr: int, stats_ptr: int,
                         stream: int) -> None:
    _check(load().hs_knn_exact_noalloc(h, q_ptr, Q, k, ids_ptr, d2_ptr, err_ptr, stats_ptr, stream))


def hs_shadow_bytes(h, kind: int, shadow_rows: int = -1) -> int:
    out = ctypes.c_int64()
    _check(load().hs_shadow_bytes(h, kind, shadow_rows, ctypes.byref(out)))
    return out.value


def hs_build_shadow(h, kind: int, shadow_rows: int, mem_ptr: int, mem_bytes: int, stream: int) -> None:
    _check(load().hs_build_shadow(h, kind, shadow_rows, mem_ptr, mem_bytes, stream))


def hs_knn_mixed(h, q_ptr: int, Q: int, k: int, ws_ptr: int, ws_bytes: int, ids_ptr: int, d2_ptr: int,
                 err_ptr: int, stats_ptr: int, stream: int) -> None:
    _check(load().hs_knn_mixed(h, q_ptr, Q, k, ws_ptr, ws_bytes, ids_ptr, d2_ptr, err_ptr, stats_ptr, stream))


def hs_server_create(handles, forms, budget_ptr: int, budget_bytes: int, cfg: hs_server_config):
    C = len(handles)
    arr = (_P * C)(*[h.value if isinstance(h, _P) else h for h in handles])
    fa = (ctypes.c_int32 * C)(*forms)
    out = _P()
    _check(load().hs_server_create(ctypes.cast(arr, _P), ctypes.cast(fa, _P), C, budget_ptr, budget_bytes,
                                   ctypes.byref(cfg), ctypes.byref(out)))
    return out


def hs_submit(srv, coll: int, q_ptr: int, k: int, tag: int) -> int:
    """Returns HS_OK or HS_EBUSY; raises on other errors."""
    code = load().hs_submit(srv, coll, q_ptr, k, tag)
    if code not in (HS_OK, HS_EBUSY):
        _check(code)
    return code


def hs_cancel(srv, tag: int) -> int:
    """Returns HS_OK (withdrawn) or HS_EBUSY (already running); raises on other errors."""
    code = load().hs_cancel(srv, tag)
    if code not in (HS_OK, HS_EBUSY):
        _check(code)
    return code


def hs_sched_cancel(h, tag: int) -> None:
    _check(load().hs_sched_cancel(h, tag))


def hs_poll(srv, buf, max_n: int) -> int:
    got = ctypes.c_int32()
    _check(load().hs_poll(srv, ctypes.cast(buf, _P), max_n, ctypes.byref(got)))
    return got.value


def hs_server_info(srv) -> hs_server_stats:
    st = hs_server_stats()
    _check(load().hs_server_info(srv, ctypes.byref(st)))
    return st


def hs_server_destroy(srv) -> None:
    _check(load().hs_server_destroy(srv))


def hs_server_now() -> float:
    return load().hs_server_now()


def hs_sched_create(C: int, streams: int, max_slots: int, max_q):
    import numpy as np
    mq = np.ascontiguousarray(np.asarray(max_q, dtype=np.int32).reshape(C, 8))
    out = _P()
    _check(load().hs_sched_create(C, streams, max_slots, mq.ctypes.data, ctypes.byref(out)))
    return out


def hs_sched_submit(h, coll: int, k: int, tag: int) -> int:
    code = load().hs_sched_submit(h, coll, k, tag)
    if code not in (HS_OK, HS_EBUSY):
        _check(code)
    return code


def hs_sched_next(h, coll: int, stream: int, max_tags: int = 1024):
    """(q_pad, k_batch, [tags]) or None when no batch forms."""
    import numpy as np
    qp = ctypes.c_int32()
    kb = ctypes.c_int32()
    cnt = ctypes.c_int32()
    tags = np.zeros(max_tags, dtype=np.uint64)
    _check(load().hs_sched_next(h, coll, stream, ctypes.byref(qp), ctypes.byref(kb), tags.ctypes.data, max_tags,
                                ctypes.byref(cnt)))
    if cnt.value == 0:
        return None
    return qp.value, kb.value, tags[:cnt.value].tolist()


def hs_sched_complete(h, coll: int, stream: int) -> None:
    _check(load().hs_sched_complete(h, coll, stream))


def hs_sched_in_system(h) -> int:
    n = ctypes.c_int32()
    _check(load().hs_sched_in_system(h, ctypes.byref(n)))
    return n.value


def hs_sched_destroy(h) -> None:
    _check(load().hs_sched_destroy(h))


def hs_index_free(h) -> None:
    _check(load().hs_index_free(h))


def hs_last_error() -> str:
    return load().hs_last_error().decode()


def hs_breakpoints(card_bits: int = 8):
    import numpy as np
    out = np.empty(255, dtype=np.float32)
    _check(load().hs_breakpoints(card_bits, out.ctypes.data))
    return out


def hs_profile_enable(on: bool) -> None:
    _check(load().hs_profile_enable(1 if on else 0))


HS_PROF_FILTER, HS_PROF_REFINE, HS_PROF_FUSED, HS_PROF_BOUND = 0, 1, 2, 3
PROF_KINDS = {"filter": HS_PROF_FILTER, "refine": HS_PROF_REFINE, "fused": HS_PROF_FUSED, "bound": HS_PROF_BOUND}


def hs_profile_read(kind: int, reset: bool = False):
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    _check(load().hs_profile_read(kind, ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0))
    return ms.value, n.value


def hs_read_probe(buf_dev: int, nbytes: int, passes: int, sink_dev: int, stream: int) -> float:
    ms = ctypes.c_double()
    _check(load().hs_read_probe(buf_dev, nbytes, passes, sink_dev, stream, ctypes.byref(ms)))
    return ms.value


def read_probe_gbs(buf, passes: int = 5, stream=None) -> float:
    """Achievable read-stream rate (GB/s) over the device tensor buf."""
    import torch
    nbytes = (buf.numel() * buf.element_size()) // 16 * 16
    sink = torch.zeros(1, dtype=torch.int32, device=buf.device)
    ms = hs_read_probe(buf.data_ptr(), nbytes, passes, sink.data_ptr(), _stream_ptr(stream))
    return nbytes * passes / (ms / 1e3) / 1e9


def hs_lds_probe(pattern: int, rounds: int, passes: int, sink_dev: int, stream: int) -> float:
    out = ctypes.c_double()
    _check(load().hs_lds_probe(pattern, rounds, passes, sink_dev, stream, ctypes.byref(out)))
    return out.value


def lds_probe_tps(pattern: int, rounds: int = 4096, passes: int = 3, device="cuda", stream=None) -> float:
    """Achievable LDS table lookups per second (pattern 0: conflict-free, 1: random symbols)."""
    import torch
    sink = torch.zeros(1, dtype=torch.int32, device=device)
    return hs_lds_probe(pattern, rounds, passes, sink.data_ptr(), _stream_ptr(stream))


def hs_union_bytes(h) -> int:
    out = ctypes.c_int64()
    _check(load().hs_union_bytes(h, ctypes.byref(out)))
    return out.value


def hs_union_enable(bits_ptr, nbytes: int) -> None:
    _check(load().hs_union_enable(bits_ptr, nbytes))


def hs_union_count(h, bits_ptr: int, counts_ptr: int, stream: int) -> None:
    _check(load().hs_union_count(h, bits_ptr, counts_ptr, stream))


def union_counts(index, fn):
    """Run fn() with batch-union marking on for `index`; returns the distinct
    (raw chunk pairs, words, envelopes) its calls read."""
    import torch
    nbytes = hs_union_bytes(index.h)
    bits = torch.zeros(nbytes // 4, dtype=torch.int32, device=index.device)
    counts = torch.zeros(3, dtype=torch.int64, device=index.device)
    torch.cuda.synchronize()
    hs_union_enable(bits.data_ptr(), nbytes)
    try:
        fn()
    finally:
        hs_union_enable(None, 0)
    hs_union_count(index.h, bits.data_ptr(), counts.data_ptr(), _stream_ptr(None))
    torch.cuda.synchronize()
    return tuple(int(v) for v in counts.cpu().tolist())


def profile_read_all(reset: bool = False):
    """{kind name: (milliseconds, launches)} for every scan-kernel kind."""
    return {name: hs_profile_read(k, reset) for name, k in PROF_KINDS.items()}


# ---------------------------------------------------------------- torch glue

@dataclass
class Params:
    w: int = 16
    leaf_size: int = 10_000
    l_max: int = 1
    seed_rows: int = 256
    eapca_th: float = 0.0
    card_bits: int = 8
    cand_per_query: int = 0
    build_flags: int = 0

    def c(self, n: int) -> hs_params:
        return hs_params(n, self.w, self.card_bits, self.leaf_size, self.l_max, self.seed_rows,
                         float(self.eapca_th), self.cand_per_query, self.build_flags, 0)


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


class Index:
    """An index over float32 series held in a CUDA (HIP) torch tensor."""

    def __init__(self, x, params: Params | None = None, stream=None):
        import torch
        if not (x.is_cuda and x.dtype == torch.float32 and x.dim() == 2 and x.is_contiguous()):
            raise ValueError("x must be a contiguous float32 [N, n] GPU tensor")
        self.params = params or Params()
        N, n = x.shape
        self.n = n
        cp = self.params.c(n)
        nbytes = hs_index_bytes(N, cp)
        self.device = x.device
        self.mem = torch.empty(nbytes, dtype=torch.uint8, device=x.device)
        self.h = hs_build_summaries(x.data_ptr(), N, cp, self.mem.data_ptr(), nbytes, _stream_ptr(stream))
        self.info = hs_get_info(self.h)
        self._ws = None
        self.shadow = None
        self.shadow_kind = 0

    @classmethod
    def from_chunks(cls, chunk, N: int, n: int, params: Params | None = None, device="cuda:0", stream=None):
        """Streaming build: chunk(row0) returns a contiguous float32 [rows, n]
        GPU tensor of series row0 .. row0 + rows - 1 (rows >= 1); it is called
        twice per chunk, in order, and must return the same values both times."""
        import torch
        self = cls.__new__(cls)
        self.params = params or Params()
        self.n = n
        self.device = torch.device(device)
        cp = self.params.c(n)
        nbytes = hs_index_bytes(N, cp)
        self.mem = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        sp = _stream_ptr(stream)
        b = hs_build_begin(N, cp, self.mem.data_ptr(), nbytes, sp)
        try:
            for add in (hs_build_add_stats, hs_build_add_rows):
                r0 = 0
                while r0 < N:
                    x = chunk(r0)
                    if not (x.is_cuda and x.dtype == torch.float32 and x.dim() == 2 and x.shape[1] == n
                            and x.is_contiguous() and 1 <= x.shape[0] <= N - r0):
                        raise ValueError("chunk must be a contiguous float32 [rows, n] GPU tensor within [0, N)")
                    add(b, x.data_ptr(), r0, x.shape[0])
                    torch.cuda.current_stream().synchronize()  # the chunk may be freed once the build has read it
                    r0 += x.shape[0]
                if add is hs_build_add_stats:
                    hs_build_partition(b)
            self.h = hs_build_finish(b)
            b = None
        finally:
            if b is not None:
                hs_build_abort(b)
        self.info = hs_get_info(self.h)
        self._ws = None
        self.shadow = None
        self.shadow_kind = 0
        return self

    def build_shadow(self, kind: int = HS_SHADOW_BF16, stream=None, shadow_rows: int = -1):
        """Build the low-precision copy that the precision form (knn_mixed) reads:
        of every stored series, or (shadow_rows >= 0) of the whole parts that fit
        in the first shadow_rows stored series."""
        import torch
        nbytes = hs_shadow_bytes(self.h, kind, shadow_rows)
        self.shadow = None
        mem = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        hs_build_shadow(self.h, kind, shadow_rows, mem.data_ptr(), nbytes, _stream_ptr(stream))
        self.shadow, self.shadow_kind = mem, kind
        self._ws = None  # a partial copy changes the workspace layout

    def layout(self):
        """Views of the stored arrays inside the index memory (rows, ids, words)
        plus the host copies of the leaf table and envelopes."""
        import torch
        N, info = self.info.n_series, self.info

        def up(v):
            return (v + 255) // 256 * 256

        rb = N * info.row_stride * 4
        ib = N * 4
        rows = self.mem[:rb].view(torch.float32).view(N, info.row_stride)
        ids = self.mem[up(rb):up(rb) + ib].view(torch.int32)
        words = self.mem[up(rb) + up(ib):up(rb) + up(ib) + N * info.word_stride].view(N, info.word_stride)
        ls, env = hs_get_leaves(self.h, info)
        return rows, ids, words, ls, env

    def sigma_codes(self):
        """The deviation codes ([N, word_stride] uint8 view, stored after the
        words) and their width h."""
        N, info = self.info.n_series, self.info

        def up(v):
            return (v + 255) // 256 * 256

        at = up(N * info.row_stride * 4) + up(N * 4) + up(N * info.word_stride)
        return self.mem[at:at + N * info.word_stride].view(N, info.word_stride), info.sigma_step

    def workspace(self, Q: int, k: int):
        import torch
        need = hs_query_workspace_bytes(self.h, Q, k)
        if self._ws is None or self._ws.numel() < need:
            self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._ws, need

    def _check_q(self, q):
        import torch
        if not (q.is_cuda and q.dtype == torch.float32 and q.dim() == 2 and q.shape[1] == self.n
                and q.is_contiguous()):
            raise ValueError("q must be a contiguous float32 [Q, n] GPU tensor")
        return q.shape[0]

    def knn_mixed(self, q, k: int, stats: bool = False, stream=None):
        """Exact k-NN through the precision form: (ids, d2, err float64 [Q, k]) [, stats]."""
        import torch
        Q = self._check_q(q)
        ws, nbytes = self.workspace(Q, k)
        ids = torch.empty((Q, k), dtype=torch.int64, device=self.device)
        d2 = torch.empty((Q, k), dtype=torch.float32, device=self.device)
        err = torch.empty((Q, k), dtype=torch.float64, device=self.device)
        st = torch.zeros((Q, len(STATS_FIELDS)), dtype=torch.int64, device=self.device) if stats else None
        hs_knn_mixed(self.h, q.data_ptr(), Q, k, ws.data_ptr(), nbytes, ids.data_ptr(), d2.data_ptr(),
                     err.data_ptr(), st.data_ptr() if st is not None else None, _stream_ptr(stream))
        if stats:
            return ids, d2, err, {f: st[:, i] for i, f in enumerate(STATS_FIELDS)}
        return ids, d2, err

    def knn(self, q, k: int, stats: bool = False, stream=None, out=None, err: bool = False):
        """Exact k-NN: returns (ids int64 [Q, k], d2 float32 [Q, k]) [, err float64 [Q, k] if err]
        [, stats dict of tensors]."""
        import torch
        Q = self._check_q(q)
        ws, nbytes = self.workspace(Q, k)
        if out is None:
            ids = torch.empty((Q, k), dtype=torch.int64, device=self.device)
            d2 = torch.empty((Q, k), dtype=torch.float32, device=self.device)
        else:
            ids, d2 = out
        eb = torch.empty((Q, k), dtype=torch.float64, device=self.device) if err else None
        st = torch.zeros((Q, len(STATS_FIELDS)), dtype=torch.int64, device=self.device) if stats else None
        hs_knn_exact(self.h, q.data_ptr(), Q, k, ws.data_ptr(), nbytes, ids.data_ptr(), d2.data_ptr(),
                     eb.data_ptr() if eb is not None else None, st.data_ptr() if st is not None else None,
                     _stream_ptr(stream))
        res = (ids, d2) + ((eb,) if err else ())
        if stats:
            return res + ({f: st[:, i] for i, f in enumerate(STATS_FIELDS)},)
        return res

    def close(self):
        if getattr(self, "h", None):
            hs_index_free(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Server:
    """Continuous-batching server over several Index objects (serving form)."""

    def __init__(self, indexes, forms=None, budget_bytes: int = 4 << 30, streams_per_coll: int = 2,
                 max_slots: int = 4096, max_batch: int = 256):
        import torch
        self.indexes = list(indexes)
        self.forms = list(forms) if forms is not None else [0] * len(self.indexes)
        dev = self.indexes[0].device
        self.budget = torch.empty(budget_bytes, dtype=torch.uint8, device=dev)
        torch.cuda.synchronize()
        cfg = hs_server_config(streams_per_coll, max_slots, max_batch, 0)
        self.h = hs_server_create([ix.h for ix in self.indexes], self.forms, self.budget.data_ptr(),
                                  budget_bytes, cfg)
        self._buf = (hs_completion * 1024)()

    def submit(self, coll: int, q, k: int, tag: int) -> bool:
        """Queue one request (q: float32 numpy [n]); False if every slot is busy."""
        import numpy as np
        q = np.ascontiguousarray(q, dtype=np.float32)
        if 0 <= coll < len(self.indexes) and (q.ndim != 1 or q.shape[0] != self.indexes[coll].n):
            raise ValueError("q must be float32 [n] of the collection")
        return hs_submit(self.h, coll, q.ctypes.data, k, tag) == HS_OK

    def cancel(self, tag: int) -> bool:
        """Withdraw a queued request (its completion comes with status HS_ECANCEL);
        False if it is already running."""
        return hs_cancel(self.h, tag) == HS_OK

    def poll(self):
        """List of completions (dicts with tag, coll, k, status, batch, times, ids, d2, err)."""
        out = []
        while True:
            got = hs_poll(self.h, self._buf, len(self._buf))
            for i in range(got):
                c = self._buf[i]
                k = c.k
                out.append({"tag": c.tag, "coll": c.coll, "k": k, "status": c.status, "batch": c.batch,
                            "t_submit": c.t_submit, "t_launch": c.t_launch, "t_done": c.t_done,
                            "ids": list(c.ids[:k]), "d2": list(c.d2[:k]), "err": list(c.err[:k])})
            if got < len(self._buf):
                return out

    def info(self) -> dict:
        st = hs_server_info(self.h)
        return {f: getattr(st, f) for f, _ in hs_server_stats._fields_}

    def close(self):
        if getattr(self, "h", None):
            hs_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
