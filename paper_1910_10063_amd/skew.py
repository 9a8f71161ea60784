"""Python binding of libskew.so (include/skew.h): argument marshalling only.

Every step runs in the HIP kernels behind the C ABI; this module only checks
tensor dtypes/devices, allocates outputs and workspace with torch, and passes
raw device pointers and the current torch stream.  There is no fallback: if
the library is not built or no gfx950 device is present the calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "lib", "libskew.so")

SKEW_OK = 0
SKEW_EINVAL = -1
SKEW_ERANGE = -2
SKEW_ENOSPACE = -3
SKEW_EHIP = -4
SKEW_EDEVICE = -5

SKEW_OP_BUILD = 1
SKEW_OP_JOIN = 2
SKEW_OP_GROUP = 3
SKEW_OP_JOIN_SINGLE_PASS = 4
SKEW_OP_GROUP_SINGLE_PASS = 5
SKEW_OP_MATERIALIZE = 6
SKEW_OP_SELECT = 7
SKEW_OP_HEAVY = 8
SKEW_OP_CACHE_MODEL = 9
SKEW_OP_STAR = 10

SKEW_HOT_AUTO = -1
SKEW_HOT_NONE = -2

EXPORTED = ("skew_last_error", "skew_workspace_bytes", "build_skew_layout", "fk_join_aggregate", "group_aggregate",
            "skew_query_status", "skew_profile_enable", "skew_profile_report", "skew_max_hot_rows",
            "skew_max_hot_groups", "materialize_column", "select_fact_rows", "heavy_hitter_counts", "skew_max_hot",
            "cache_model_hit_rate", "star_join_batch", "star_join_autotune", "stream_probe",
            "fk_join_aggregate_noalloc", "skew_join_hot_rows", "skew_join_choose", "skew_group_choose",
            "append_skew_layout")


class StarTuning(ctypes.Structure):
    """skew_star_tuning of include/skew.h."""
    _fields_ = [("prod_hot_rows", ctypes.c_int32), ("cust_hot_rows", ctypes.c_int32),
                ("tile_rows", ctypes.c_int32), ("blocks", ctypes.c_int32)]


class Choice(ctypes.Structure):
    _fields_ = [("hot_rows", ctypes.c_int32), ("partitioned", ctypes.c_int32), ("cold_share", ctypes.c_double),
                ("l2_hit", ctypes.c_double), ("bytes_single", ctypes.c_double),
                ("bytes_partitioned", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


class SkewError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"skew error {code}: {msg}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libskew.so (after torch, so both use torch's HIP runtime) and declare signatures."""
    global _lib
    if _lib is not None and path == LIB_PATH:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built: run `python -m paper_1910_10063_amd.build_ext`")
    lib = ctypes.CDLL(path)
    P, I64, I32, SZ = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_size_t
    lib.skew_last_error.argtypes = []
    lib.skew_last_error.restype = ctypes.c_char_p
    lib.skew_workspace_bytes.argtypes = [ctypes.c_int, I64, I32]
    lib.skew_workspace_bytes.restype = SZ
    lib.build_skew_layout.argtypes = [P, I64, I32, P, P, P, P, P, P, P, P, P, SZ, P]
    lib.build_skew_layout.restype = ctypes.c_int
    lib.fk_join_aggregate.argtypes = [P, I64, P, P, I32, I32, I32, I32, P, P, P, SZ, P]
    lib.fk_join_aggregate.restype = ctypes.c_int
    lib.fk_join_aggregate_noalloc.argtypes = [P, I64, P, P, I32, I32, I32, I32, P, P, P]
    lib.fk_join_aggregate_noalloc.restype = ctypes.c_int
    lib.group_aggregate.argtypes = [P, P, I64, I32, I32, P, P, P, P, SZ, P]
    lib.group_aggregate.restype = ctypes.c_int
    lib.skew_query_status.argtypes = [P, SZ, P]
    lib.skew_query_status.restype = ctypes.c_int
    lib.skew_max_hot_rows.argtypes = [I32]
    lib.skew_max_hot_rows.restype = I32
    lib.append_skew_layout.argtypes = [I32, I32, P, P, P, P, P, P, P, P, I64, P, P]
    lib.append_skew_layout.restype = ctypes.c_int
    lib.skew_join_choose.argtypes = [P, I32, I64, I32, P, P, SZ, P]
    lib.skew_join_choose.restype = ctypes.c_int
    lib.skew_group_choose.argtypes = [P, I32, I64, P, P, SZ, P]
    lib.skew_group_choose.restype = ctypes.c_int
    lib.skew_join_hot_rows.argtypes = [I64, I32, I32, I32, SZ]
    lib.skew_join_hot_rows.restype = I32
    lib.skew_max_hot_groups.argtypes = []
    lib.skew_max_hot_groups.restype = I32
    lib.skew_profile_enable.argtypes = [ctypes.c_int]
    lib.skew_profile_enable.restype = None
    lib.skew_profile_report.argtypes = [ctypes.c_char_p, ctypes.c_int, P, P, ctypes.c_int]
    lib.skew_profile_report.restype = ctypes.c_int
    lib.materialize_column.argtypes = [P, I64, P, I32, I32, P, P, SZ, P]
    lib.materialize_column.restype = ctypes.c_int
    lib.select_fact_rows.argtypes = [P, I64, P, I32, I32, I32, P, P, P, SZ, P]
    lib.select_fact_rows.restype = ctypes.c_int
    lib.heavy_hitter_counts.argtypes = [P, I64, I32, I32, P, P, P, P, SZ, P]
    lib.heavy_hitter_counts.restype = ctypes.c_int
    lib.cache_model_hit_rate.argtypes = [P, I32, P, I32, I64, P, P, SZ, P]
    lib.cache_model_hit_rate.restype = ctypes.c_int
    lib.star_join_batch.argtypes = [P, P, P, P, I32, P, P, I32, P, I32, P, P, P, P, SZ, P]
    lib.star_join_batch.restype = ctypes.c_int
    lib.star_join_autotune.argtypes = [P, P, P, P, I32, P, P, I32, P, I32, P, P, P, P, P, SZ, P]
    lib.star_join_autotune.restype = ctypes.c_int
    lib.stream_probe.argtypes = [P, SZ, P, P]
    lib.stream_probe.restype = ctypes.c_int
    lib.skew_max_hot.argtypes = [ctypes.c_int]
    lib.skew_max_hot.restype = I64
    if path == LIB_PATH:
        _lib = lib
    return lib


def hip_runtimes_loaded() -> list[str]:
    """Paths of the HIP runtime libraries mapped into this process."""
    maps = open("/proc/self/maps").read().splitlines()
    return sorted({m.split()[-1] for m in maps if "libamdhip64" in m})


def _check(rc: int):
    if rc != SKEW_OK:
        raise SkewError(rc, _lib.skew_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _need(t, dtype, name):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be on the GPU")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def workspace_bytes(op: int, n_fact: int, n_keys: int) -> int:
    return int(load_library().skew_workspace_bytes(op, n_fact, n_keys))


def workspace(op: int, n_fact: int, n_keys: int, device) -> torch.Tensor:
    """A workspace tensor for `op` (uint8, 256-byte aligned by torch's allocator)."""
    nb = workspace_bytes(op, n_fact, n_keys)
    ws = torch.empty(max(nb, 256), dtype=torch.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


@dataclass
class Layout:
    """Device tensors of one permutation index and the data it rewrote."""

    perm: torch.Tensor  # int32[n_keys]: key of rank r
    rank: torch.Tensor  # int32[n_keys]: rank of key k
    counts_by_rank: torch.Tensor  # uint32 values in an int32 tensor (frequencies < 2^31 here) [n_keys]
    fact_recoded: torch.Tensor | None
    price: torch.Tensor | None
    category: torch.Tensor | None


def build_skew_layout(fact_keys: torch.Tensor, n_keys: int, price: torch.Tensor | None = None,
                      category: torch.Tensor | None = None, in_place: bool = False, recode: bool = True,
                      ws: torch.Tensor | None = None) -> Layout:
    lib = load_library()
    _need(fact_keys, torch.int32, "fact_keys")
    dev = fact_keys.device
    if price is not None:
        _need(price, torch.int32, "price")
    if category is not None:
        _need(category, torch.int8, "category")
    perm = torch.empty(n_keys, dtype=torch.int32, device=dev)
    rank = torch.empty(n_keys, dtype=torch.int32, device=dev)
    cbr = torch.empty(n_keys, dtype=torch.int32, device=dev)
    fr = (fact_keys if in_place else torch.empty_like(fact_keys)) if recode else None
    po = torch.empty(n_keys, dtype=torch.int32, device=dev) if price is not None else None
    co = torch.empty(n_keys, dtype=torch.int8, device=dev) if category is not None else None
    if ws is None:
        ws = workspace(SKEW_OP_BUILD, fact_keys.numel(), n_keys, dev)
    _check(lib.build_skew_layout(_ptr(fact_keys), fact_keys.numel(), n_keys, _ptr(price), _ptr(category),
                                 _ptr(perm), _ptr(rank), _ptr(cbr), _ptr(fr), _ptr(po), _ptr(co), _ptr(ws),
                                 ws.numel(), _stream(dev)))
    return Layout(perm, rank, cbr, fr, po, co)


def append_skew_layout(L: "Layout", n_new: int, price: torch.Tensor | None = None, category: torch.Tensor | None = None,
                       fact_keys_new: torch.Tensor | None = None, in_place: bool = False) -> tuple["Layout", torch.Tensor | None]:
    """Index maintenance without a rebuild (Section 3.1): L (a layout of n_old dimension rows) extended to n_new rows
    (the new ids become its least frequent items; price/category are the whole dimension, new rows at the end) and
    the new fact keys recoded through it.  Returns the extended layout (new tensors; its fact_recoded is L's) and
    the recoded new keys."""
    lib = load_library()
    n_old = L.perm.numel()
    dev = L.perm.device
    perm = torch.empty(n_new, dtype=torch.int32, device=dev)
    rank = torch.empty(n_new, dtype=torch.int32, device=dev)
    cbr = torch.empty(n_new, dtype=torch.int32, device=dev)
    perm[:n_old].copy_(L.perm)
    rank[:n_old].copy_(L.rank)
    cbr[:n_old].copy_(L.counts_by_rank)
    po = co = None
    if price is not None:
        _need(price, torch.int32, "price")
        po = torch.empty(n_new, dtype=torch.int32, device=dev)
        po[:n_old].copy_(L.price)
    if category is not None:
        _need(category, torch.int8, "category")
        co = torch.empty(n_new, dtype=torch.int8, device=dev)
        co[:n_old].copy_(L.category)
    fr = None
    nf = 0
    if fact_keys_new is not None:
        _need(fact_keys_new, torch.int32, "fact_keys_new")
        nf = fact_keys_new.numel()
        fr = fact_keys_new if in_place else torch.empty_like(fact_keys_new)
    _check(lib.append_skew_layout(n_old, n_new, _ptr(perm), _ptr(rank), _ptr(cbr), _ptr(price), _ptr(category),
                                  _ptr(po), _ptr(co), _ptr(fact_keys_new), nf, _ptr(fr), _stream(dev)))
    return Layout(perm, rank, cbr, L.fact_recoded, po, co), fr


def fk_join_aggregate(fact_keys: torch.Tensor, price: torch.Tensor, category: torch.Tensor, cat_lt: int,
                      group_by_category: bool, hot_rows: int = SKEW_HOT_AUTO, ws: torch.Tensor | None = None,
                      out: tuple[torch.Tensor, torch.Tensor] | None = None):
    """Returns (sum, count): int64 tensors of 1 or 16 groups."""
    lib = load_library()
    _need(fact_keys, torch.int32, "fact_keys")
    _need(price, torch.int32, "price")
    _need(category, torch.int8, "category")
    if price.numel() != category.numel():
        raise ValueError("price and category must have the same length")
    dev = fact_keys.device
    g = 16 if group_by_category else 1
    if out is None:
        out = (torch.empty(g, dtype=torch.int64, device=dev), torch.empty(g, dtype=torch.int64, device=dev))
    if ws is None:
        ws = workspace(SKEW_OP_JOIN, fact_keys.numel(), price.numel(), dev)
    _check(lib.fk_join_aggregate(_ptr(fact_keys), fact_keys.numel(), _ptr(price), _ptr(category), price.numel(),
                                 int(cat_lt), 1 if group_by_category else 0, int(hot_rows), _ptr(out[0]),
                                 _ptr(out[1]), _ptr(ws), ws.numel(), _stream(dev)))
    return out


SKEW_NOALLOC_MAX_ROWS = 1 << 24


def fk_join_aggregate_noalloc(fact_keys: torch.Tensor, price: torch.Tensor, category: torch.Tensor, cat_lt: int,
                              group_by_category: bool, out: tuple[torch.Tensor, torch.Tensor],
                              hot_rows: int = SKEW_HOT_AUTO):
    """fk_join_aggregate without a workspace: the library's fixed per-device scratch (single pass, at most
    SKEW_NOALLOC_MAX_ROWS dimension rows).  The caller passes the int64 outputs [1] or [16]."""
    lib = load_library()
    _need(fact_keys, torch.int32, "fact_keys")
    _need(price, torch.int32, "price")
    _need(category, torch.int8, "category")
    if price.numel() != category.numel():
        raise ValueError("price and category must have the same length")
    _check(lib.fk_join_aggregate_noalloc(_ptr(fact_keys), fact_keys.numel(), _ptr(price), _ptr(category),
                                         price.numel(), int(cat_lt), 1 if group_by_category else 0, int(hot_rows),
                                         _ptr(out[0]), _ptr(out[1]), _stream(fact_keys.device)))
    return out


def group_aggregate(group_keys: torch.Tensor, values: torch.Tensor, n_groups: int,
                    hot_groups: int = SKEW_HOT_AUTO, perm: torch.Tensor | None = None,
                    ws: torch.Tensor | None = None, out: tuple[torch.Tensor, torch.Tensor] | None = None):
    """Returns (sum, count): int64 tensors of n_groups entries, in original key order."""
    lib = load_library()
    _need(group_keys, torch.int32, "group_keys")
    _need(values, torch.int32, "values")
    if group_keys.numel() != values.numel():
        raise ValueError("group_keys and values must have the same length")
    if perm is not None:
        _need(perm, torch.int32, "perm")
    dev = group_keys.device
    if out is None:
        out = (torch.empty(n_groups, dtype=torch.int64, device=dev),
               torch.empty(n_groups, dtype=torch.int64, device=dev))
    if ws is None:
        ws = workspace(SKEW_OP_GROUP, group_keys.numel(), n_groups, dev)
    _check(lib.group_aggregate(_ptr(group_keys), _ptr(values), group_keys.numel(), n_groups, int(hot_groups),
                               _ptr(perm), _ptr(out[0]), _ptr(out[1]), _ptr(ws), ws.numel(), _stream(dev)))
    return out


def materialize_column(fact_keys: torch.Tensor, col: torch.Tensor, hot_rows: int = SKEW_HOT_AUTO,
                       ws: torch.Tensor | None = None, out: torch.Tensor | None = None) -> torch.Tensor:
    """out[j] = col[fact_keys[j]] (0 for out-of-range keys), int32."""
    lib = load_library()
    _need(fact_keys, torch.int32, "fact_keys")
    _need(col, torch.int32, "col")
    dev = fact_keys.device
    if out is None:
        out = torch.empty_like(fact_keys)
    _need(out, torch.int32, "out")
    if out.numel() != fact_keys.numel():
        raise ValueError("out must have one entry per fact key")
    if ws is None:
        ws = workspace(SKEW_OP_MATERIALIZE, fact_keys.numel(), col.numel(), dev)
    _check(lib.materialize_column(_ptr(fact_keys), fact_keys.numel(), _ptr(col), col.numel(), int(hot_rows),
                                  _ptr(out), _ptr(ws), ws.numel(), _stream(dev)))
    return out


def select_fact_rows(fact_keys: torch.Tensor, col: torch.Tensor, lt: int, hot_rows: int = SKEW_HOT_AUTO,
                     ws: torch.Tensor | None = None,
                     out: tuple[torch.Tensor, torch.Tensor] | None = None) -> tuple[torch.Tensor, torch.Tensor]:
    """(offsets int32[n_fact] of which the first count are valid, count int64[1]) for col[key] < lt."""
    lib = load_library()
    _need(fact_keys, torch.int32, "fact_keys")
    _need(col, torch.int32, "col")
    dev = fact_keys.device
    if out is None:
        out = (torch.empty(max(fact_keys.numel(), 1), dtype=torch.int32, device=dev),
               torch.empty(1, dtype=torch.int64, device=dev))
    if ws is None:
        ws = workspace(SKEW_OP_SELECT, fact_keys.numel(), col.numel(), dev)
    _check(lib.select_fact_rows(_ptr(fact_keys), fact_keys.numel(), _ptr(col), col.numel(), int(lt), int(hot_rows),
                                _ptr(out[0]), _ptr(out[1]), _ptr(ws), ws.numel(), _stream(dev)))
    return out


def heavy_hitter_counts(ranked_keys: torch.Tensor, n_keys: int, k: int, perm: torch.Tensor | None = None,
                        ws: torch.Tensor | None = None) -> tuple[torch.Tensor, torch.Tensor]:
    """(keys int32[k], counts int64[k]) of ranks [0, k) on the frequency-ordered layout."""
    lib = load_library()
    _need(ranked_keys, torch.int32, "ranked_keys")
    if perm is not None:
        _need(perm, torch.int32, "perm")
    dev = ranked_keys.device
    keys = torch.empty(max(k, 1), dtype=torch.int32, device=dev)
    counts = torch.empty(max(k, 1), dtype=torch.int64, device=dev)
    if ws is None:
        ws = workspace(SKEW_OP_HEAVY, ranked_keys.numel(), n_keys, dev)
    _check(lib.heavy_hitter_counts(_ptr(ranked_keys), ranked_keys.numel(), n_keys, int(k), _ptr(perm), _ptr(keys),
                                   _ptr(counts), _ptr(ws), ws.numel(), _stream(dev)))
    return keys[:k], counts[:k]


def cache_model_hit_rate(counts_by_rank: torch.Tensor, cache_lines: int, values_per_line: int = 32,
                         rank: torch.Tensor | None = None, ws: torch.Tensor | None = None) -> float:
    """Hit rate of the stack-distance model (Section 3.3); rank=None: frequency-ordered layout."""
    lib = load_library()
    _need(counts_by_rank, torch.int32, "counts_by_rank")
    if rank is not None:
        _need(rank, torch.int32, "rank")
    dev = counts_by_rank.device
    if ws is None:
        ws = workspace(SKEW_OP_CACHE_MODEL, 0, counts_by_rank.numel(), dev)
    out = ctypes.c_double(0.0)
    _check(lib.cache_model_hit_rate(_ptr(counts_by_rank), counts_by_rank.numel(), _ptr(rank), int(values_per_line),
                                    int(cache_lines), ctypes.byref(out), _ptr(ws), ws.numel(), _stream(dev)))
    return out.value


def stream_probe(buf: torch.Tensor) -> torch.Tensor:
    """One read pass over a contiguous device tensor (16-byte multiple); returns the 64-bit wrapping sum of its
    32-bit words as a device int64[1] (measurement of the achievable read rate)."""
    lib = load_library()
    if not buf.is_contiguous():
        raise SkewError(SKEW_EINVAL, "buf must be contiguous")
    out = torch.empty(1, dtype=torch.int64, device=buf.device)
    nbytes = buf.numel() * buf.element_size()
    _check(lib.stream_probe(ctypes.c_void_p(buf.data_ptr() if nbytes else 0), nbytes, _ptr(out), _stream(buf.device)))
    return out


@dataclass
class StarBatch:
    """Device tensors of one batch: keys of all queries one after the other, the query table, dimensions."""

    prod_keys: torch.Tensor      # int32[N], 16-byte aligned
    cust_keys: torch.Tensor      # int32[N], 16-byte aligned
    query_start: torch.Tensor    # int64[n_queries + 1]
    query_cust_lt: torch.Tensor  # int32[n_queries]
    price: torch.Tensor          # int32[n_prod]
    category: torch.Tensor       # int8[n_prod]
    segment: torch.Tensor        # int8[n_cust]


def _star_args(b: StarBatch):
    for name, t, dt in (("prod_keys", b.prod_keys, torch.int32), ("cust_keys", b.cust_keys, torch.int32),
                        ("query_start", b.query_start, torch.int64), ("query_cust_lt", b.query_cust_lt, torch.int32),
                        ("price", b.price, torch.int32), ("category", b.category, torch.int8),
                        ("segment", b.segment, torch.int8)):
        _need(t, dt, name)
    nq = b.query_cust_lt.numel()
    if b.query_start.numel() != nq + 1:
        raise ValueError("query_start must have n_queries + 1 entries")
    return nq, (_ptr(b.prod_keys), _ptr(b.cust_keys), _ptr(b.query_start), _ptr(b.query_cust_lt), nq, _ptr(b.price),
                _ptr(b.category), b.price.numel(), _ptr(b.segment), b.segment.numel())


def star_workspace(b: StarBatch) -> torch.Tensor:
    return workspace(SKEW_OP_STAR, b.query_cust_lt.numel(), max(b.price.numel(), b.segment.numel()),
                     b.prod_keys.device)


def star_join_batch(b: StarBatch, tuning: StarTuning | None = None, ws: torch.Tensor | None = None,
                    out: tuple[torch.Tensor, torch.Tensor] | None = None):
    """(sum, count): int64[n_queries, 16]."""
    lib = load_library()
    nq, args = _star_args(b)
    dev = b.prod_keys.device
    if out is None:
        out = (torch.empty(nq, 16, dtype=torch.int64, device=dev), torch.empty(nq, 16, dtype=torch.int64, device=dev))
    if ws is None:
        ws = star_workspace(b)
    _check(lib.star_join_batch(*args, ctypes.byref(tuning) if tuning is not None else None, _ptr(out[0]),
                               _ptr(out[1]), _ptr(ws), ws.numel(), _stream(dev)))
    return out


def star_join_autotune(b: StarBatch, ws: torch.Tensor | None = None) -> tuple[StarTuning, float]:
    lib = load_library()
    nq, args = _star_args(b)
    dev = b.prod_keys.device
    out = (torch.empty(nq, 16, dtype=torch.int64, device=dev), torch.empty(nq, 16, dtype=torch.int64, device=dev))
    if ws is None:
        ws = star_workspace(b)
    best = StarTuning()
    ms = ctypes.c_float(0.0)
    _check(lib.star_join_autotune(*args, _ptr(out[0]), _ptr(out[1]), ctypes.byref(best), ctypes.byref(ms), _ptr(ws),
                                  ws.numel(), _stream(dev)))
    return best, ms.value


def max_hot(op: int) -> int:
    v = load_library().skew_max_hot(op)
    if v < 0:
        _check(int(v))
    return int(v)


def query_status(ws: torch.Tensor) -> int:
    """SKEW_OK, or raises SkewError(SKEW_ERANGE) if the last query on ws saw an out-of-range key."""
    lib = load_library()
    rc = lib.skew_query_status(_ptr(ws), ws.numel(), _stream(ws.device))
    _check(rc)
    return rc


def max_hot_rows(group_by_category: bool) -> int:
    v = load_library().skew_max_hot_rows(1 if group_by_category else 0)
    if v < 0:
        _check(v)
    return int(v)


def join_hot_rows(n_fact: int, n_rows: int, group_by_category: bool, hot_rows: int = SKEW_HOT_AUTO,
                  ws: torch.Tensor | None = None) -> int:
    """The hot prefix fk_join_aggregate uses with these arguments (ws: the workspace it is given; None: one of
    SKEW_OP_JOIN size)."""
    lib = load_library()
    nb = ws.numel() if ws is not None else workspace_bytes(SKEW_OP_JOIN, n_fact, n_rows)
    v = lib.skew_join_hot_rows(n_fact, n_rows, 1 if group_by_category else 0, int(hot_rows), nb)
    if v < 0:
        _check(v)
    return int(v)


def join_choose(counts_by_rank: torch.Tensor, n_fact: int, group_by_category: bool,
                ws: torch.Tensor | None = None) -> dict:
    """The library's threshold prior for fk_join_aggregate on a layout (its counts_by_rank): hot_rows, form and the
    modelled quantities."""
    lib = load_library()
    _need(counts_by_rank, torch.int32, "counts_by_rank")
    n = counts_by_rank.numel()
    if ws is None:
        ws = workspace(SKEW_OP_CACHE_MODEL, 0, n, counts_by_rank.device)
    c = Choice()
    _check(lib.skew_join_choose(_ptr(counts_by_rank), n, n_fact, 1 if group_by_category else 0, ctypes.byref(c),
                                _ptr(ws), ws.numel(), _stream(counts_by_rank.device)))
    return c.as_dict()


def group_choose(counts_by_rank: torch.Tensor, n_fact: int, ws: torch.Tensor | None = None) -> dict:
    """The library's threshold prior for group_aggregate on a layout of its group keys."""
    lib = load_library()
    _need(counts_by_rank, torch.int32, "counts_by_rank")
    n = counts_by_rank.numel()
    if ws is None:
        ws = workspace(SKEW_OP_CACHE_MODEL, 0, n, counts_by_rank.device)
    c = Choice()
    _check(lib.skew_group_choose(_ptr(counts_by_rank), n, n_fact, ctypes.byref(c), _ptr(ws), ws.numel(),
                                 _stream(counts_by_rank.device)))
    return c.as_dict()


def max_hot_groups() -> int:
    v = load_library().skew_max_hot_groups()
    if v < 0:
        _check(v)
    return int(v)


def profile_enable(on: bool = True) -> None:
    """Record HIP events around every launch stage from now on (see skew_profile_report)."""
    load_library().skew_profile_enable(1 if on else 0)


def profile_report(max_stages: int = 64) -> dict:
    """{stage: (total_ms, launches)} of the stages recorded since the last report."""
    lib = load_library()
    names = ctypes.create_string_buffer(64 * max_stages)
    ms = (ctypes.c_float * max_stages)()
    calls = (ctypes.c_int * max_stages)()
    n = lib.skew_profile_report(names, len(names), ctypes.cast(ms, ctypes.c_void_p),
                                ctypes.cast(calls, ctypes.c_void_p), max_stages)
    keys = names.raw.split(b"\0")[:n]
    return {k.decode(): (float(ms[i]), int(calls[i])) for i, k in enumerate(keys)}
