"""The C ABI of libskew.so on the host: symbols and argument checks (no GPU needed).

Fake device addresses are passed where the call must fail before touching
the device; every case here returns before the first HIP call.
"""
import ctypes
import os
import re

import pytest

from paper_1910_10063_amd import skew

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "skew.h")

A = ctypes.c_void_p(0x10000)  # aligned fake device address
A2 = ctypes.c_void_p(0x20000)
MIS = ctypes.c_void_p(0x10002)  # not 4-byte aligned
WS = ctypes.c_void_p(0x40000)  # 256-byte aligned
WS_MIS = ctypes.c_void_p(0x40010)
NULL = None
S = ctypes.c_void_p(0)


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    return skew.load_library()


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert set(names) == set(skew.EXPORTED), names
    for n in names:
        assert hasattr(lib, n), n


def test_workspace_sizes(lib):
    assert lib.skew_workspace_bytes(skew.SKEW_OP_JOIN, 10, 1000) >= 256 + 4000
    assert lib.skew_workspace_bytes(skew.SKEW_OP_GROUP, 10, 1000) >= 256 + 16000
    b = lib.skew_workspace_bytes(skew.SKEW_OP_BUILD, 10, 100_000)
    assert b >= 256 + 4 * 5 * 100_000
    assert lib.skew_workspace_bytes(99, 10, 10) == 0
    assert lib.skew_workspace_bytes(skew.SKEW_OP_JOIN, -1, 10) == 0
    assert all(lib.skew_workspace_bytes(op, 0, 7) % 256 == 0 for op in (1, 2, 3))


def _build(lib, **kw):
    a = dict(fact=A, n_fact=10, n_keys=5, price=NULL, cat=NULL, perm=A, rank=A2, cbr=NULL, fr=NULL, po=NULL,
             co=NULL, ws=WS, wsb=1 << 20, stream=S)
    a.update(kw)
    return lib.build_skew_layout(a["fact"], a["n_fact"], a["n_keys"], a["price"], a["cat"], a["perm"], a["rank"],
                                 a["cbr"], a["fr"], a["po"], a["co"], a["ws"], a["wsb"], a["stream"])


@pytest.mark.parametrize("kw,code", [
    (dict(n_fact=-1), skew.SKEW_EINVAL),
    (dict(n_fact=1 << 32), skew.SKEW_EINVAL),
    (dict(n_keys=0), skew.SKEW_EINVAL),
    (dict(fact=NULL), skew.SKEW_EINVAL),
    (dict(perm=NULL), skew.SKEW_EINVAL),
    (dict(rank=NULL), skew.SKEW_EINVAL),
    (dict(ws=NULL), skew.SKEW_EINVAL),
    (dict(price=A), skew.SKEW_EINVAL),            # price without price_out
    (dict(co=A), skew.SKEW_EINVAL),               # category_out without category
    (dict(fact=MIS), skew.SKEW_EINVAL),
    (dict(ws=WS_MIS), skew.SKEW_EINVAL),
    (dict(wsb=100), skew.SKEW_ENOSPACE),
])
def test_build_rejects(lib, kw, code):
    assert _build(lib, **kw) == code
    assert lib.skew_last_error().decode()


def _join(lib, **kw):
    a = dict(fact=A, n_fact=10, price=A, cat=A2, n_rows=5, cat_lt=4, by=0, hot=0, s=A, c=A2, ws=WS, wsb=1 << 20)
    a.update(kw)
    return lib.fk_join_aggregate(a["fact"], a["n_fact"], a["price"], a["cat"], a["n_rows"], a["cat_lt"], a["by"],
                                 a["hot"], a["s"], a["c"], a["ws"], a["wsb"], S)


@pytest.mark.parametrize("kw,code", [
    (dict(n_fact=-5), skew.SKEW_EINVAL),
    (dict(n_rows=0), skew.SKEW_EINVAL),
    (dict(fact=NULL), skew.SKEW_EINVAL),
    (dict(price=NULL), skew.SKEW_EINVAL),
    (dict(cat=NULL), skew.SKEW_EINVAL),
    (dict(s=NULL), skew.SKEW_EINVAL),
    (dict(by=2), skew.SKEW_EINVAL),
    (dict(hot=-3), skew.SKEW_EINVAL),
    (dict(s=ctypes.c_void_p(0x10004)), skew.SKEW_EINVAL),  # int64 output not 8-byte aligned
    (dict(ws=NULL), skew.SKEW_EINVAL),
    (dict(wsb=255), skew.SKEW_ENOSPACE),
])
def test_join_rejects(lib, kw, code):
    assert _join(lib, **kw) == code


def _group(lib, **kw):
    a = dict(keys=A, vals=A2, n=10, m=5, hot=0, perm=NULL, s=A, c=A2, ws=WS, wsb=1 << 20)
    a.update(kw)
    return lib.group_aggregate(a["keys"], a["vals"], a["n"], a["m"], a["hot"], a["perm"], a["s"], a["c"], a["ws"],
                               a["wsb"], S)


@pytest.mark.parametrize("kw,code", [
    (dict(n=-1), skew.SKEW_EINVAL),
    (dict(m=0), skew.SKEW_EINVAL),
    (dict(keys=NULL), skew.SKEW_EINVAL),
    (dict(vals=NULL), skew.SKEW_EINVAL),
    (dict(hot=-3), skew.SKEW_EINVAL),
    (dict(perm=MIS), skew.SKEW_EINVAL),
    (dict(c=NULL), skew.SKEW_EINVAL),
    (dict(wsb=300), skew.SKEW_ENOSPACE),
])
def test_group_rejects(lib, kw, code):
    assert _group(lib, **kw) == code


def test_status_rejects_null(lib):
    assert lib.skew_query_status(NULL, 0, S) == skew.SKEW_EINVAL


def test_valid_call_without_gpu_reports_edevice(lib):
    import torch

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    assert _join(lib) == skew.SKEW_EDEVICE
    assert "device" in lib.skew_last_error().decode()


def _mat(lib, **kw):
    a = dict(keys=A, n=10, col=A2, n_rows=5, hot=0, out=ctypes.c_void_p(0x80000), ws=WS, wsb=1 << 20)
    a.update(kw)
    return lib.materialize_column(a["keys"], a["n"], a["col"], a["n_rows"], a["hot"], a["out"], a["ws"], a["wsb"], S)


@pytest.mark.parametrize("kw,code", [
    (dict(n=-1), skew.SKEW_EINVAL),
    (dict(n_rows=0), skew.SKEW_EINVAL),
    (dict(keys=NULL), skew.SKEW_EINVAL),
    (dict(col=NULL), skew.SKEW_EINVAL),
    (dict(out=NULL), skew.SKEW_EINVAL),
    (dict(out=ctypes.c_void_p(0x10008)), skew.SKEW_EINVAL),  # overlaps the keys
    (dict(hot=-3), skew.SKEW_EINVAL),
    (dict(col=MIS), skew.SKEW_EINVAL),
    (dict(wsb=100), skew.SKEW_ENOSPACE),
])
def test_materialize_rejects(lib, kw, code):
    assert _mat(lib, **kw) == code


def _sel(lib, **kw):
    a = dict(keys=A, n=10, col=A2, n_rows=5, lt=7, hot=0, out=ctypes.c_void_p(0x80000), cnt=ctypes.c_void_p(0x90000),
             ws=WS, wsb=1 << 26)
    a.update(kw)
    return lib.select_fact_rows(a["keys"], a["n"], a["col"], a["n_rows"], a["lt"], a["hot"], a["out"], a["cnt"],
                                a["ws"], a["wsb"], S)


@pytest.mark.parametrize("kw,code", [
    (dict(n=-1), skew.SKEW_EINVAL),
    (dict(n=1 << 31), skew.SKEW_EINVAL),
    (dict(n_rows=0), skew.SKEW_EINVAL),
    (dict(keys=NULL), skew.SKEW_EINVAL),
    (dict(cnt=NULL), skew.SKEW_EINVAL),
    (dict(cnt=ctypes.c_void_p(0x90004)), skew.SKEW_EINVAL),
    (dict(hot=-5), skew.SKEW_EINVAL),
    (dict(wsb=1000), skew.SKEW_ENOSPACE),
])
def test_select_rejects(lib, kw, code):
    assert _sel(lib, **kw) == code


def _heavy(lib, **kw):
    a = dict(keys=A, n=10, n_keys=5, k=3, perm=NULL, ok=A2, oc=ctypes.c_void_p(0x80000), ws=WS, wsb=1 << 20)
    a.update(kw)
    return lib.heavy_hitter_counts(a["keys"], a["n"], a["n_keys"], a["k"], a["perm"], a["ok"], a["oc"], a["ws"],
                                   a["wsb"], S)


@pytest.mark.parametrize("kw,code", [
    (dict(n=-1), skew.SKEW_EINVAL),
    (dict(n_keys=0), skew.SKEW_EINVAL),
    (dict(k=-1), skew.SKEW_EINVAL),
    (dict(k=6), skew.SKEW_EINVAL),
    (dict(keys=NULL), skew.SKEW_EINVAL),
    (dict(ok=NULL), skew.SKEW_EINVAL),
    (dict(oc=ctypes.c_void_p(0x80004)), skew.SKEW_EINVAL),
    (dict(wsb=10), skew.SKEW_ENOSPACE),
])
def test_heavy_rejects(lib, kw, code):
    assert _heavy(lib, **kw) == code


def test_operator_workspace_sizes(lib):
    assert lib.skew_workspace_bytes(skew.SKEW_OP_MATERIALIZE, 10, 10) == 256
    assert lib.skew_workspace_bytes(skew.SKEW_OP_HEAVY, 10, 10) == 256
    # bitmap + one round of segments (with the chunk slack) + tables
    assert lib.skew_workspace_bytes(skew.SKEW_OP_SELECT, 1 << 20, 1000) >= 256 + 4 * (1 << 20)
    assert lib.skew_workspace_bytes(skew.SKEW_OP_SELECT, 3_000_000_000, 10) < 4 * 3_000_000_000


def test_stream_probe_rejects(lib):
    ok = ctypes.c_void_p(0x10000)
    assert lib.stream_probe(ok, 16, NULL, S) == skew.SKEW_EINVAL          # no output
    assert lib.stream_probe(NULL, 16, A2, S) == skew.SKEW_EINVAL          # no buffer
    assert lib.stream_probe(ctypes.c_void_p(0x10004), 16, A2, S) == skew.SKEW_EINVAL  # not 16-byte aligned
    assert lib.stream_probe(ok, 20, A2, S) == skew.SKEW_EINVAL            # not a 16-byte multiple
    assert lib.stream_probe(ok, 16, ctypes.c_void_p(0x20004), S) == skew.SKEW_EINVAL  # output not 8-byte aligned


def _star(lib, fn="star_join_batch", **kw):
    a = dict(pk=A, uk=A2, qs=A, lt=A2, nq=4, price=A, cat=A2, n_prod=100, seg=A, n_cust=50, s=A, c=A2, ws=WS,
             wsb=1 << 30)
    a.update(kw)
    head = (a["pk"], a["uk"], a["qs"], a["lt"], a["nq"], a["price"], a["cat"], a["n_prod"], a["seg"], a["n_cust"])
    if fn == "star_join_batch":
        return lib.star_join_batch(*head, None, a["s"], a["c"], a["ws"], a["wsb"], S)
    best, ms = skew.StarTuning(), ctypes.c_float(0)
    return lib.star_join_autotune(*head, a["s"], a["c"], ctypes.byref(best), ctypes.byref(ms), a["ws"], a["wsb"], S)


@pytest.mark.parametrize("fn", ["star_join_batch", "star_join_autotune"])
@pytest.mark.parametrize("kw,code", [
    (dict(nq=0), skew.SKEW_EINVAL),
    (dict(nq=4097), skew.SKEW_EINVAL),  # more queries than the tile table holds
    (dict(n_prod=0), skew.SKEW_EINVAL),
    (dict(n_cust=0), skew.SKEW_EINVAL),
    (dict(pk=NULL), skew.SKEW_EINVAL),
    (dict(lt=NULL), skew.SKEW_EINVAL),
    (dict(seg=NULL), skew.SKEW_EINVAL),
    (dict(c=NULL), skew.SKEW_EINVAL),
    (dict(pk=ctypes.c_void_p(0x10004)), skew.SKEW_EINVAL),  # keys not 16-byte aligned
    (dict(qs=ctypes.c_void_p(0x10004)), skew.SKEW_EINVAL),  # int64 table not 8-byte aligned
    (dict(ws=WS_MIS), skew.SKEW_EINVAL),
    (dict(wsb=1024), skew.SKEW_ENOSPACE),
])
def test_star_rejects(lib, fn, kw, code):
    assert _star(lib, fn, **kw) == code


def test_star_workspace_holds_the_customer_bitmaps(lib):
    # one bitmap per query over every customer row while all of them fit 1 GiB, on top of the product words and
    # the segment copy
    small = lib.skew_workspace_bytes(skew.SKEW_OP_STAR, 1, 2_000_000)
    big = lib.skew_workspace_bytes(skew.SKEW_OP_STAR, 65, 2_000_000)
    assert 64 * 2_000_000 // 8 <= big - small < 64 * 2_000_000 // 8 + 4096
    d = lib.skew_workspace_bytes(skew.SKEW_OP_STAR, 9, 100_000) - lib.skew_workspace_bytes(skew.SKEW_OP_STAR, 1, 100_000)
    assert 8 * 100_000 // 8 <= d < 8 * 100_000 // 8 + 2048
    # beyond the budget the sizing bound is the budget itself: every call with at most this many rows in either
    # dimension fits, whichever bitmaps it builds
    base = lib.skew_workspace_bytes(skew.SKEW_OP_STAR, 0, 2_500_000)
    over = lib.skew_workspace_bytes(skew.SKEW_OP_STAR, 4096, 2_500_000) - base
    assert (1 << 30) <= over < (1 << 30) + 4096 * 4 + 4096


def _join_noalloc(lib, **kw):
    a = dict(keys=A, n=10, price=A2, cat=A, rows=100, lt=4, by=1, hot=0, s=A, c=A2)
    a.update(kw)
    return lib.fk_join_aggregate_noalloc(a["keys"], a["n"], a["price"], a["cat"], a["rows"], a["lt"], a["by"],
                                         a["hot"], a["s"], a["c"], S)


@pytest.mark.parametrize("kw,code", [
    (dict(n=-1), skew.SKEW_EINVAL),
    (dict(rows=0), skew.SKEW_EINVAL),
    (dict(rows=skew.SKEW_NOALLOC_MAX_ROWS + 1), skew.SKEW_EINVAL),  # larger than the library's scratch
    (dict(keys=NULL), skew.SKEW_EINVAL),
    (dict(keys=MIS), skew.SKEW_EINVAL),
    (dict(by=2), skew.SKEW_EINVAL),
    (dict(hot=-3), skew.SKEW_EINVAL),
    (dict(s=ctypes.c_void_p(0x10004)), skew.SKEW_EINVAL),
])
def test_join_noalloc_rejects(lib, kw, code):
    assert _join_noalloc(lib, **kw) == code


def test_choose_rejects(lib):
    c = skew.Choice()
    assert lib.skew_join_choose(NULL, 10, 100, 1, ctypes.byref(c), WS, 1 << 20, S) == skew.SKEW_EINVAL
    assert lib.skew_join_choose(A, 0, 100, 1, ctypes.byref(c), WS, 1 << 20, S) == skew.SKEW_EINVAL
    assert lib.skew_join_choose(A, 10, 100, 2, ctypes.byref(c), WS, 1 << 20, S) == skew.SKEW_EINVAL
    assert lib.skew_join_choose(A, 10, 100, 1, ctypes.byref(c), WS_MIS, 1 << 20, S) == skew.SKEW_EINVAL
    assert lib.skew_group_choose(A, 10, -1, ctypes.byref(c), WS, 1 << 20, S) == skew.SKEW_EINVAL
    assert lib.skew_group_choose(MIS, 10, 100, ctypes.byref(c), WS, 1 << 20, S) == skew.SKEW_EINVAL
    assert lib.skew_join_hot_rows(10, 0, 1, -1, 0) == skew.SKEW_EINVAL


def test_append_rejects(lib):
    def app(**kw):
        a = dict(n_old=10, n_new=12, perm=A, rank=A2, cbr=NULL, price=NULL, cat=NULL, po=NULL, co=NULL, keys=A,
                 nf=5, out=A2)
        a.update(kw)
        return lib.append_skew_layout(a["n_old"], a["n_new"], a["perm"], a["rank"], a["cbr"], a["price"], a["cat"],
                                      a["po"], a["co"], a["keys"], a["nf"], a["out"], S)
    assert app(n_old=0) == skew.SKEW_EINVAL
    assert app(n_new=9) == skew.SKEW_EINVAL
    assert app(nf=-1) == skew.SKEW_EINVAL
    assert app(perm=NULL) == skew.SKEW_EINVAL
    assert app(price=A) == skew.SKEW_EINVAL  # price without its output
    assert app(keys=NULL) == skew.SKEW_EINVAL
    assert app(out=MIS) == skew.SKEW_EINVAL
