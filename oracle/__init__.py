"""ctypes wrapper of the plain C oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only callers.  The product path never imports this
package.  All functions take and return numpy arrays and compute on the host.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")

_lib = None


def compile_source(src: str, out: str) -> str:
    """Compile an oracle source file with gcc into a shared library (plain -O2)."""
    tmp = out + f".tmp{os.getpid()}"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, src, "-lm"])
    os.replace(tmp, out)
    return out


def build(force: bool = False) -> str:
    """Compile oracle.c into liboracle.so."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        compile_source(SRC, LIB)
    return LIB


def bind(path: str):
    """Load an oracle shared library and declare its signatures."""
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    I64, I32 = ctypes.c_int64, ctypes.c_int32
    lib.oracle_key_counts.argtypes = [P, I64, I32, P]
    lib.oracle_key_counts.restype = I64
    lib.oracle_permutation_index.argtypes = [P, I32, P, P]
    lib.oracle_permutation_index.restype = None
    lib.oracle_recode.argtypes = [P, I64, P, I32, P]
    lib.oracle_recode.restype = None
    lib.oracle_permute_i32.argtypes = [P, P, I32, P]
    lib.oracle_permute_i32.restype = None
    lib.oracle_permute_i8.argtypes = [P, P, I32, P]
    lib.oracle_permute_i8.restype = None
    lib.oracle_fk_join_aggregate.argtypes = [P, I64, P, P, I32, I32, I32, P, P]
    lib.oracle_fk_join_aggregate.restype = None
    lib.oracle_group_aggregate.argtypes = [P, P, I64, I32, P, P]
    lib.oracle_group_aggregate.restype = I64
    lib.oracle_build_layout.argtypes = [P, I64, I32, P, P, P, P, P, P, P, P]
    lib.oracle_build_layout.restype = I64
    lib.oracle_append_layout.argtypes = [I32, I32, P, P, P, P, P, P, P, I64, P]
    lib.oracle_append_layout.restype = I64
    lib.oracle_materialize.argtypes = [P, I64, P, I32, P]
    lib.oracle_materialize.restype = I64
    lib.oracle_select.argtypes = [P, I64, P, I32, I32, P]
    lib.oracle_select.restype = I64
    lib.oracle_heavy_hitters.argtypes = [P, I64, I32, I32, P, P]
    lib.oracle_heavy_hitters.restype = I32
    lib.oracle_cache_model.argtypes = [P, I64, I64]
    lib.oracle_cache_model.restype = ctypes.c_double
    lib.oracle_star_join.argtypes = [P, P, I64, P, P, I32, P, I32, I32, P, P]
    lib.oracle_star_join.restype = None
    return lib


def use_library(path: str | None):
    """Point this module at another oracle build (None = the default liboracle.so)."""
    global _lib
    _lib = None if path is None else bind(path)


def _load():
    global _lib
    if _lib is None:
        _lib = bind(build())  # rebuilt when oracle.c is newer than the library
    return _lib


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def key_counts(C, n_keys: int):
    C = _c(C, np.int32)
    cnt = np.zeros(max(n_keys, 1), dtype=np.int64)[:n_keys]
    invalid = _load().oracle_key_counts(_p(C), C.size, n_keys, _p(cnt))
    return cnt, int(invalid)


def permutation_index(cnt):
    cnt = _c(cnt, np.int64)
    n = cnt.size
    perm = np.empty(n, dtype=np.int32)
    rank = np.empty(n, dtype=np.int32)
    _load().oracle_permutation_index(_p(cnt), n, _p(perm), _p(rank))
    return perm, rank


def recode(C, rank):
    C = _c(C, np.int32)
    rank = _c(rank, np.int32)
    out = np.empty_like(C)
    _load().oracle_recode(_p(C), C.size, _p(rank), rank.size, _p(out))
    return out


def permute_dim(col, perm):
    perm = _c(perm, np.int32)
    if np.asarray(col).dtype == np.int8:
        col = _c(col, np.int8)
        out = np.empty(perm.size, dtype=np.int8)
        _load().oracle_permute_i8(_p(col), _p(perm), perm.size, _p(out))
    else:
        col = _c(col, np.int32)
        out = np.empty(perm.size, dtype=np.int32)
        _load().oracle_permute_i32(_p(col), _p(perm), perm.size, _p(out))
    return out


def fk_join_aggregate(C, price, category, cat_lt: int, by_category: bool):
    """Returns (sum, count) int64 arrays of length 1, or 16 when by_category."""
    C = _c(C, np.int32)
    price = _c(price, np.int32)
    category = _c(category, np.int8)
    assert price.size == category.size
    g = 16 if by_category else 1
    s = np.zeros(g, dtype=np.int64)
    c = np.zeros(g, dtype=np.int64)
    _load().oracle_fk_join_aggregate(_p(C), C.size, _p(price), _p(category), price.size, int(cat_lt),
                                     1 if by_category else 0, _p(s), _p(c))
    return s, c


def group_aggregate(G, V, n_groups: int):
    G = _c(G, np.int32)
    V = _c(V, np.int32)
    assert G.size == V.size
    s = np.zeros(max(n_groups, 1), dtype=np.int64)[:n_groups]
    c = np.zeros(max(n_groups, 1), dtype=np.int64)[:n_groups]
    invalid = _load().oracle_group_aggregate(_p(G), _p(V), G.size, n_groups, _p(s), _p(c))
    return s, c, int(invalid)


def materialize(C, col):
    """out[j] = col[C[j]] (0 for out-of-range keys); returns (out, invalid)."""
    C = _c(C, np.int32)
    col = _c(col, np.int32)
    out = np.empty(C.size, dtype=np.int32)
    inv = _load().oracle_materialize(_p(C), C.size, _p(col), col.size, _p(out))
    return out, int(inv)


def select(C, col, lt: int):
    """Increasing int64 offsets j with col[C[j]] < lt."""
    C = _c(C, np.int32)
    col = _c(col, np.int32)
    out = np.empty(max(C.size, 1), dtype=np.int64)
    n = _load().oracle_select(_p(C), C.size, _p(col), col.size, int(lt), _p(out))
    return out[:n].copy()


def heavy_hitters(G, n_keys: int, k: int):
    """(keys, counts) of the k most frequent keys, most frequent first, ties by ascending key."""
    G = _c(G, np.int32)
    keys = np.empty(max(min(k, n_keys), 1), dtype=np.int32)
    counts = np.empty(max(min(k, n_keys), 1), dtype=np.int64)
    kk = _load().oracle_heavy_hitters(_p(G), G.size, n_keys, int(k), _p(keys), _p(counts))
    return keys[:kk].copy(), counts[:kk].copy()


def star_join(P, U, price, category, cust_attr, cust_lt: int):
    """(sum, count) int64[16]: SUM(price), COUNT(*) by product category over rows whose customer passes."""
    P = _c(P, np.int32)
    U = _c(U, np.int32)
    price = _c(price, np.int32)
    category = _c(category, np.int8)
    cust_attr = _c(cust_attr, np.int8)
    assert P.size == U.size and price.size == category.size
    s = np.zeros(16, dtype=np.int64)
    c = np.zeros(16, dtype=np.int64)
    _load().oracle_star_join(_p(P), _p(U), P.size, _p(price), _p(category), price.size, _p(cust_attr), cust_attr.size,
                             int(cust_lt), _p(s), _p(c))
    return s, c


def cache_model(f, cache_lines: int) -> float:
    """Hit rate of the stack-distance model of Section 3.3 for line frequencies f (summing to 1)."""
    f = _c(f, np.float64)
    return float(_load().oracle_cache_model(_p(f), f.size, int(cache_lines)))


def line_frequencies(counts_by_key, values_per_line: int):
    """Access frequency of every cache line of `values_per_line` consecutive keys (Section 3.3)."""
    c = np.asarray(counts_by_key, dtype=np.float64)
    n_lines = (c.size + values_per_line - 1) // values_per_line
    pad = np.zeros(n_lines * values_per_line)
    pad[:c.size] = c
    lines = pad.reshape(n_lines, values_per_line).sum(axis=1)
    tot = lines.sum()
    return lines / tot if tot > 0 else lines


class Layout:
    """Result of the oracle's index build (Section 3.1/3.2)."""

    def __init__(self, perm, rank, counts_by_rank, fact_recoded, price=None, category=None, invalid=0):
        self.perm = perm
        self.rank = rank
        self.counts_by_rank = counts_by_rank
        self.fact_recoded = fact_recoded
        self.price = price
        self.category = category
        self.invalid = invalid


def build_layout(C, n_keys: int, price=None, category=None) -> Layout:
    C = _c(C, np.int32)
    perm = np.empty(n_keys, dtype=np.int32)
    rank = np.empty(n_keys, dtype=np.int32)
    cbr = np.empty(n_keys, dtype=np.int64)
    Cn = np.empty_like(C)
    pn = cn = None
    if price is not None:
        price = _c(price, np.int32)
        pn = np.empty(n_keys, dtype=np.int32)
    if category is not None:
        category = _c(category, np.int8)
        cn = np.empty(n_keys, dtype=np.int8)
    inv = _load().oracle_build_layout(_p(C), C.size, n_keys, _p(price), _p(category), _p(perm), _p(rank),
                                      _p(cbr), _p(Cn), _p(pn), _p(cn))
    return Layout(perm, rank, cbr, Cn, pn, cn, int(inv))


def append_layout(layout: Layout, n_new: int, price=None, category=None, C_add=None):
    """Index maintenance without a rebuild (Section 3.1): the layout of n_old = layout.perm.size dimension rows
    extended to n_new rows (new ids become the least frequent items) and the fact rows C_add recoded through it.
    price/category are the whole new dimension columns (n_new rows).  Returns (perm, rank, price', category',
    C_add', invalid)."""
    n_old = layout.perm.size
    perm = np.empty(n_new, dtype=np.int32)
    rank = np.empty(n_new, dtype=np.int32)
    perm[:n_old] = layout.perm
    rank[:n_old] = layout.rank
    pn = cn = None
    if price is not None:
        price = _c(price, np.int32)
        pn = np.empty(n_new, dtype=np.int32)
        pn[:n_old] = layout.price
    if category is not None:
        category = _c(category, np.int8)
        cn = np.empty(n_new, dtype=np.int8)
        cn[:n_old] = layout.category
    C_add = _c(C_add if C_add is not None else np.zeros(0, np.int32), np.int32)
    out = np.empty_like(C_add)
    inv = _load().oracle_append_layout(n_old, n_new, _p(perm), _p(rank), _p(price), _p(category), _p(pn), _p(cn),
                                       _p(C_add), C_add.size, _p(out))
    return perm, rank, pn, cn, out, int(inv)
