#!/usr/bin/env python3
"""Benchmark of the skew-layout FK join-aggregate on one MI355X.

Workload (defaults): a 1e7-row dimension table (price U[1,10000] int32,
category U[0,15] int8) and 1e9 int32 fact keys drawn Zipf s=1.0 over ranks and
mapped to keys by a seeded permutation; query SUM(price), COUNT(*) grouped by
category (16 groups), int64 results.  All inputs are synthetic and generated
on the device from fixed seeds.

One timed step is one query over the whole fact column on the skew layout
(recoded keys + permuted dimension): the per-query dimension pack and the
join-aggregate kernel, inputs already resident in HBM.  The layout build is
timed on its own, as the paper reports index-build cost apart from queries
(Section 5.1).  Beside the headline number the JSON line carries the
identity-layout baseline, the build time, the Zipf and hot-prefix sweeps, the
grouped aggregation on a 1e6-group / 5e8-row workload, the roofline of the
dominant kernel and the CPU oracle timed on the host.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
METRIC = "fact tuples/s and % of HBM roofline, skew layout vs identity layout (bit-exact)"

# The paper's own results for this path, reported beside ours as context only: they were measured on CPUs
# (Section 5, hardware table: Skylake Xeon 8175M, 24 cores x 2 SMT, 2.5 GHz, 60 GB/s; Xeon Phi 7210, 64 cores
# x 4 SMT, 1.3 GHz, 55 GB/s), with 4-byte keys, on Zipf columns of 1e9 facts and 128M keys unless noted.
PAPER_CONTEXT = {
    "hardware": {"skylake": "Xeon 8175M, 24 cores x 2 SMT, 2.5 GHz, 33 MB L3, 60 GB/s",
                 "phi": "Xeon Phi 7210, 64 cores x 4 SMT, 1.3 GHz, no L3, 55 GB/s"},
    "speedups_freq_vs_rand": [
        {"query": "Q1 materialize, SIMD, z=1", "speedup": ">1.2x on both", "where": "Section 5.1"},
        {"query": "Q1 materialize with software prefetch, z=1", "speedup": "3x", "hardware": "phi",
         "where": "Section 5.1"},
        {"query": "Q1 materialize, multithreaded", "speedup": ">1.3x", "hardware": "both, up to 48/256 threads",
         "where": "Section 5.1"},
        {"query": "Q2 select, multithreaded", "speedup": "1.4-2.2x (phi), 1.3-1.8x (skylake)", "where": "Section 5.1"},
        {"query": "top-4k heavy hitters vs the full aggregate, z=0.5", "speedup": "8.6x (phi), 6.6x (skylake)",
         "where": "Section 5.1"},
        {"query": "hybrid aggregation vs independent per-thread buffers", "speedup": "4.7x (skylake, 48 threads), "
         "10.4x (phi, 256 threads)", "where": "Section 5.1"},
        {"query": "Pageview Q1 / Q2 / Q3 / top-4k, one thread", "speedup": "1.5x / 2.2x / 1.3x / 4.0x",
         "hardware": "skylake", "where": "Section 5.2"},
    ],
    "index_build": "a Q3 plus a Q1 on the rand layout: a few seconds with all threads (Section 5.1)",
    "gpu_numbers": None,
}
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "join_query_traffic.json")
# sources of the query's kernels: the HBM byte counters stay valid while these are unchanged
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1910_10063_amd", "csrc", f)
                  for f in ("join_kernels.hip", "partition_kernels.hip", "query_common.h", "device_common.h")]


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def timed_runs(fn, steps, warmup, stream):
    """Run fn warmup times, then `steps` times back to back, each run between its own pair of HIP events
    on `stream` (run i spans events i and i + 1, so no synchronisation separates the runs).  Returns the
    per-run times in ms."""
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record(stream)
    for i in range(steps):
        fn()
        ev[i + 1].record(stream)
    torch.cuda.synchronize()
    return [ev[i].elapsed_time(ev[i + 1]) for i in range(steps)]


def timed(fn, steps, warmup, stream):
    """Median ms per run of `steps` individually event-timed runs after `warmup` untimed ones."""
    import numpy as np

    return float(np.median(timed_runs(fn, steps, warmup, stream)))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n-rows", type=int, default=10_000_000)
    ap.add_argument("--n-fact", type=int, default=1_000_000_000)
    ap.add_argument("--zipf", type=float, default=1.0)
    ap.add_argument("--hot-rows", type=int, default=-1, help="hot prefix in LDS (-1: library default)")
    ap.add_argument("--cpu-rows", type=int, default=1_000_000_000, help="fact rows the CPU oracle is timed on")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-extras", action="store_true", help="headline query only (for profiler runs)")
    ap.add_argument("--with-group", action="store_true", help="run the group-by workload even with --no-extras")
    ap.add_argument("--with-ops", action="store_true", help="run the operator variants even with --no-extras")
    ap.add_argument("--with-star", action="store_true", help="run the batched star join even with --no-extras")
    ap.add_argument("--with-serve", action="store_true", help="run the serving loop even with --no-extras")
    ap.add_argument("--serve-seconds", type=float, default=40.0, help="length of the serving run (0: skip)")
    ap.add_argument("--model-validation", action="store_true",
                    help="only the cache-model check: single-pass queries without LDS prefix on both layouts "
                         "(3 skew, then 3 identity) for an L2 hit-rate profile, and the model's predictions")
    ap.add_argument("--skew-only", action="store_true",
                    help="skip the identity-layout query (profiler runs: one kernel name per stage)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one device copy of 1 GiB (reference for profiler byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the skew-layout path runs on a single MI355X; "
              "a multi-GPU run would shard the fact column and is not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1910_10063_amd import skew
    from paper_1910_10063_amd import workload as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)
    N, F, S = args.n_rows, args.n_fact, args.zipf
    K, WU = args.steps, args.warmup
    k = 2  # seeds of the 16-group join workload

    if args.copy_calibration:
        a = torch.ones(1 << 28, dtype=torch.int32, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    log(f"generating N={N} F={F} s={S}")
    inp = W.device_join_inputs(k, N, F, S, dev)
    C, price, cat = inp["fact"], inp["price"], inp["category"]

    # ---- layout build (Section 3.1): histogram, rank sort, inverse, dimension copy, recode
    bws = skew.workspace(skew.SKEW_OP_BUILD, F, N, dev)
    Cp = torch.empty_like(C)
    perm = torch.empty(N, dtype=torch.int32, device=dev)
    rank = torch.empty(N, dtype=torch.int32, device=dev)
    cbr = torch.empty(N, dtype=torch.int32, device=dev)
    pp = torch.empty(N, dtype=torch.int32, device=dev)
    cp = torch.empty(N, dtype=torch.int8, device=dev)
    lib = skew.load_library()

    def build():
        rc = lib.build_skew_layout(C.data_ptr(), F, N, price.data_ptr(), cat.data_ptr(), perm.data_ptr(),
                                   rank.data_ptr(), cbr.data_ptr(), Cp.data_ptr(), pp.data_ptr(), cp.data_ptr(),
                                   bws.data_ptr(), bws.numel(), stream.cuda_stream)
        if rc:
            raise skew.SkewError(rc, lib.skew_last_error().decode())

    log("layout build")
    build_ms = timed(build, 3, 1, stream)

    cache_model = bench_cache_model(cbr, rank, N, F, dev)
    if args.model_validation:
        sws = skew.workspace(skew.SKEW_OP_JOIN_SINGLE_PASS, F, N, dev)
        o = (torch.empty(16, dtype=torch.int64, device=dev), torch.empty(16, dtype=torch.int64, device=dev))
        for keys, pr, ca in ((Cp, pp, cp), (C, price, cat)):
            for _ in range(3):
                skew.fk_join_aggregate(keys, pr, ca, 16, True, hot_rows=0, ws=sws, out=o)
        torch.cuda.synchronize()
        print(json.dumps({"cache_model": cache_model, "n_fact": F, "n_rows": N, "zipf_s": S,
                          "dispatches": "join_kernel<16>: 3 skew layout, then 3 identity layout, hot_rows=0"}))
        return

    # ---- queries
    jws = skew.workspace(skew.SKEW_OP_JOIN, F, N, dev)
    out_s = torch.empty(16, dtype=torch.int64, device=dev)
    out_c = torch.empty(16, dtype=torch.int64, device=dev)
    t_hot = args.hot_rows

    def query(keys, pr, ca, t, ws=jws):
        return lambda: skew.fk_join_aggregate(keys, pr, ca, 16, True, hot_rows=t, ws=ws, out=(out_s, out_c))

    log("skew-layout query (timed steps)")
    ms_skew = timed(query(Cp, pp, cp, t_hot), K, WU, stream)
    skew_res = (out_s.cpu().numpy().copy(), out_c.cpu().numpy().copy())
    # achievable read rate of this device: one read pass over the 4 GB column with 16-byte loads
    log("stream probe (read bandwidth)")
    ms_probe = timed(lambda: skew.stream_probe(Cp), K, 1, stream)
    probe_gbs = 4.0 * F / (ms_probe * 1e-3) / 1e9
    ms_ident, agree = None, None
    if not args.skew_only:
        log("identity-layout query")
        ms_ident = timed(query(C, price, cat, 0), K, WU, stream)
        ident_res = (out_s.cpu().numpy().copy(), out_c.cpu().numpy().copy())
        agree = bool((skew_res[0] == ident_res[0]).all() and (skew_res[1] == ident_res[1]).all())

    # ---- per-stage times from HIP events recorded by the library on this stream
    KP = max(K // 2, 3)
    skew.profile_report()
    skew.profile_enable(True)
    for _ in range(KP):
        query(Cp, pp, cp, t_hot)()
    st_skew = skew.profile_report()
    st_ident = {}
    if not args.skew_only:
        for _ in range(KP):
            query(C, price, cat, 0)()
        st_ident = skew.profile_report()
    build()
    st_build = skew.profile_report()
    skew.profile_enable(False)

    def per_query(st, n):
        return {k: {"ms": round(v[0] / n, 4), "launches": round(v[1] / n, 3)} for k, v in st.items()}

    stages_skew = per_query(st_skew, KP)
    stages_ident = per_query(st_ident, KP)
    # Roofline of the whole query (its algorithmic bytes: every fact key once, 4 B, and both dimension
    # columns once, 5 B per row, plus the 16 x 2 int64 outputs) over the median query time, and,
    # beside it, the dominant kernel on its own share: the keys one launch streams, 4 B each.
    dom = max(stages_skew, key=lambda k: stages_skew[k]["ms"])
    launches = stages_skew[dom]["launches"]
    hot_used = skew.join_hot_rows(F, N, True, t_hot, ws=jws)
    cold = int(cbr[hot_used:].to(torch.int64).sum().item())  # fact keys at or above the threshold
    keys_per_launch = F / launches
    dom_bytes = {"join_split": 4.0 * keys_per_launch, "join_single_pass": 4.0 * keys_per_launch,
                 "join_pack": 5.0 * N}.get(dom, 4.0 * keys_per_launch)
    dom_ms = stages_skew[dom]["ms"] / launches
    dom_gbs = dom_bytes / (dom_ms * 1e-3) / 1e9
    q_bytes = 4.0 * F + 5.0 * N + 256.0
    q_gbs = q_bytes / (ms_skew * 1e-3) / 1e9
    traffic, kernel_traffic = None, None
    if os.path.exists(TRAFFIC_FILE):
        tr = json.load(open(TRAFFIC_FILE))
        if tr.get("source_sha") == kernel_source_sha() and tr.get("n_fact") == F and tr.get("n_rows") == N \
                and tr.get("zipf_s") == S:
            traffic = tr.get("hbm_bytes_per_query")
            kernel_traffic = tr.get("kernels", {}).get(dom, {}).get("hbm_bytes_per_launch")
    roofline = {"bound": "hbm", "scope": "whole query", "achieved": round(q_gbs, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(q_gbs / HBM_PEAK_GBS, 4), "traffic": traffic,
                "algorithmic_bytes": q_bytes, "query_ms": round(ms_skew, 4),
                "frac_of_read_probe": round(q_gbs / probe_gbs, 4),
                "kernel": dom, "kernel_achieved": round(dom_gbs, 1), "kernel_frac": round(dom_gbs / HBM_PEAK_GBS, 4),
                "kernel_algorithmic_bytes_per_launch": dom_bytes, "kernel_ms": round(dom_ms, 4),
                "kernel_traffic": kernel_traffic, "launches_per_query": launches, "cold_fact_keys": cold,
                "kernel_frac_of_read_probe": round(dom_gbs / probe_gbs, 4)}

    result = {
        "metric": METRIC,
        "value": F / (ms_skew * 1e-3),
        "unit": "fact tuples/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": WU,
        "ms_per_step": ms_skew,
        "timing": "median of the individually event-timed steps",
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic (seeded Zipf fact keys and uniform dimension columns, generated on the device)",
        "config": {"workload": f"fk-join-aggregate: {N:.0e}-row dimension, {F:.0e} Zipf(s={S}) int32 fact keys, "
                               "SUM(price), COUNT(*) GROUP BY category (16 groups), skew layout",
                   "n_rows": N, "n_fact": F, "zipf_s": S, "groups": 16, "hot_rows": t_hot,
                   "hot_rows_used": hot_used,
                   "seeds": {"fact": W.fact_seed(k), "perm": W.perm_seed(k), "price": W.price_seed(k),
                             "category": W.category_seed(k)}},
        "roofline": roofline,
        "paper_context": PAPER_CONTEXT,
        "read_probe": {"kernel": "stream_probe", "bytes": 4.0 * F, "ms": round(ms_probe, 4),
                       "GB_per_s": round(probe_gbs, 1), "frac_of_peak": round(probe_gbs / HBM_PEAK_GBS, 4)},
        "identity": {"value": F / (ms_ident * 1e-3), "ms_per_step": ms_ident} if ms_ident else None,
        "speedup_vs_identity": ms_ident / ms_skew if ms_ident else None,
        "stages_ms": {"skew": stages_skew, "identity": stages_ident, "build": per_query(st_build, 1)},
        "build": {"ms": build_ms, "fact_tuples_per_s": F / (build_ms * 1e-3)},
        "layouts_agree": agree,
        "cache_model": cache_model,
    }

    if not args.no_extras:
        single_ws = skew.workspace(skew.SKEW_OP_JOIN_SINGLE_PASS, F, N, dev)
        ms_sp = timed(query(Cp, pp, cp, t_hot, single_ws), max(K // 2, 10), 1, stream)
        ms_sp_i = timed(query(C, price, cat, 0, single_ws), max(K // 2, 10), 1, stream)
        result["single_pass"] = {"skew_tuples_per_s": F / (ms_sp * 1e-3), "identity_tuples_per_s": F / (ms_sp_i * 1e-3)}
        del single_ws
    if not args.no_extras:
        # hot-threshold sweep: up to the LDS capacity every hot row is read from LDS; past it (64K, 128K, 256K)
        # the rows between the capacity and t are warm, gathered in pass 1 through the caches
        sweep_t = []
        for t in (0, 4096, 8192, 16384, 32768, skew.SKEW_HOT_AUTO, 65536, 131072, 262144):
            ms = timed(query(Cp, pp, cp, t), max(K // 2, 10), 1, stream)
            used = skew.join_hot_rows(F, N, True, t, ws=jws)
            sweep_t.append({"hot_rows": t, "hot_rows_used": used, "ms": round(ms, 4), "tuples_per_s": F / (ms * 1e-3),
                            "cold_share": float(cbr[used:].to(torch.int64).sum().item()) / F})
        result["hot_prefix_sweep"] = sweep_t
        # the library's threshold prior (frequencies of the layout, the stack-distance model of the cold lookups)
        # beside the measured best of the sweep
        ch = skew.join_choose(cbr, F, True)
        ws_ch = jws if ch["partitioned"] else skew.workspace(skew.SKEW_OP_JOIN_SINGLE_PASS, F, N, dev)
        ms_ch = timed(query(Cp, pp, cp, ch["hot_rows"], ws_ch), max(K // 2, 10), 1, stream)
        best = min(sweep_t, key=lambda r: r["ms"])
        result["model_choice"] = dict(ch, ms=round(ms_ch, 4), tuples_per_s=F / (ms_ch * 1e-3),
                                      sweep_best={"hot_rows": best["hot_rows"], "ms": best["ms"]},
                                      ms_over_sweep_best=round(ms_ch / best["ms"], 4))
        del ws_ch
        # cold caches: a 512 MB write (twice the memory-side cache) before each query, outside the timed region
        flush = torch.empty(1 << 27, dtype=torch.int32, device=dev)
        cold_ms = []
        for _ in range(max(K // 2, 10)):
            flush.fill_(1)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            query(Cp, pp, cp, t_hot)()
            b.record(stream)
            torch.cuda.synchronize()
            cold_ms.append(a.elapsed_time(b))
        del flush
        cold = float(np.median(cold_ms))
        result["cold_cache"] = {"ms": round(cold, 4), "tuples_per_s": F / (cold * 1e-3), "runs": len(cold_ms),
                                "flush": "512 MB device write before each query"}
        # Zipf sweep: each exponent gets its own fact column and layout
        sweep_s = []
        for s in (0.0, 0.5, 1.0, 1.5):
            log(f"zipf sweep s={s}")
            d = W.device_join_inputs(k, N, F, s, dev)
            L = skew.build_skew_layout(d["fact"], N, d["price"], d["category"], in_place=False, ws=bws)
            ms_i = timed(lambda: skew.fk_join_aggregate(d["fact"], d["price"], d["category"], 16, True, hot_rows=0,
                                                        ws=jws, out=(out_s, out_c)), max(K // 2, 10), 1, stream)
            ri = out_s.cpu().numpy().copy()
            ms_s = timed(lambda: skew.fk_join_aggregate(L.fact_recoded, L.price, L.category, 16, True,
                                                        hot_rows=t_hot, ws=jws, out=(out_s, out_c)),
                         max(K // 2, 10), 1, stream)
            rs = out_s.cpu().numpy().copy()
            ch = skew.join_choose(L.counts_by_rank, F, True)
            ws_ch = jws if ch["partitioned"] else skew.workspace(skew.SKEW_OP_JOIN_SINGLE_PASS, F, N, dev)
            ms_c = timed(lambda: skew.fk_join_aggregate(L.fact_recoded, L.price, L.category, 16, True,
                                                        hot_rows=ch["hot_rows"], ws=ws_ch, out=(out_s, out_c)),
                         max(K // 2, 10), 1, stream)
            rc = out_s.cpu().numpy().copy()
            del ws_ch
            sweep_s.append({"zipf_s": s, "identity_tuples_per_s": F / (ms_i * 1e-3),
                            "skew_tuples_per_s": F / (ms_s * 1e-3), "speedup": ms_i / ms_s,
                            "model_choice": {"hot_rows": ch["hot_rows"], "partitioned": ch["partitioned"],
                                             "l2_hit": round(ch["l2_hit"], 4), "cold_share": round(ch["cold_share"], 4),
                                             "tuples_per_s": F / (ms_c * 1e-3)},
                            "layouts_agree": bool((ri == rs).all() and (ri == rc).all())})
            del d, L
            torch.cuda.empty_cache()
        result["zipf_sweep"] = sweep_s
    if not args.no_extras:
        result["small_config"] = bench_small(dev, stream)
    if not args.no_extras or args.with_ops:
        result["operators"] = bench_operators(K, C, price, Cp, pp, perm, N, F, dev, stream)
    if not args.no_extras or args.with_star:
        result["star_batch"] = bench_star(K, dev, stream)
    if (not args.no_extras or args.with_serve) and args.serve_seconds > 0:
        result["serving"] = bench_serve(args.serve_seconds, dev)
    if not args.no_extras or args.with_group:
        result["group_by"] = bench_group_by(K, WU, dev, stream)

    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(C, price, cat, args.cpu_rows, skew_res if args.cpu_rows >= F else None,
                                              layout=(Cp, pp, cp))
        if not args.no_extras:
            result["cpu_baseline"]["other_rows"] = cpu_baseline_rows()
        if "bit_exact_vs_oracle" in result["cpu_baseline"]:
            result["bit_exact_vs_oracle"] = result["cpu_baseline"].pop("bit_exact_vs_oracle")
    print(json.dumps(result), flush=True)


def bench_small(dev, stream, launches=100, replays=10):
    """The plain method at small size: a 1e5-row dimension, 1e6 Zipf(1.0) fact keys, SUM(price) and COUNT(*)
    WHERE category < 4, on both layouts.  Launch-bound, so the query is captured 100 times in one HIP graph and
    the graph replayed; the per-query time is reported, and the two layouts' answers are compared (the GPU tests
    check this workload against the oracle)."""
    import torch

    from paper_1910_10063_amd import skew
    from paper_1910_10063_amd import workload as W

    k, N, F = 1, 100_000, 1_000_000
    h = W.host_join_inputs(k, N, F, 1.0)
    C = torch.from_numpy(h["fact"]).to(dev)
    price = torch.from_numpy(h["price"]).to(dev)
    cat = torch.from_numpy(h["category"]).to(dev)
    L = skew.build_skew_layout(C, N, price, cat)
    res = {"workload": f"plain method: {N:.0e}-row dimension, {F:.0e} Zipf(1.0) keys, SUM(price), COUNT(*) "
                       "WHERE category < 4", "queries_per_graph": launches, "graph_replays": replays}
    for name, keys, pr, ca, t in (("skew", L.fact_recoded, L.price, L.category, skew.SKEW_HOT_AUTO),
                                  ("identity", C, price, cat, 0)):
        ws = skew.workspace(skew.SKEW_OP_JOIN, F, N, dev)
        out = (torch.empty(1, dtype=torch.int64, device=dev), torch.empty(1, dtype=torch.int64, device=dev))
        skew.fk_join_aggregate(keys, pr, ca, 4, False, hot_rows=t, ws=ws, out=out)  # eager: sets LDS limits
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):
            for _ in range(launches):
                skew.fk_join_aggregate(keys, pr, ca, 4, False, hot_rows=t, ws=ws, out=out)
        ms = timed(g.replay, replays, 1, stream) / launches
        res[name] = {"us_per_query": round(ms * 1e3, 2), "tuples_per_s": F / (ms * 1e-3),
                     "sum": int(out[0].cpu()[0]), "count": int(out[1].cpu()[0])}
        del g, ws
    res["speedup_vs_identity"] = res["identity"]["us_per_query"] / res["skew"]["us_per_query"]
    res["layouts_agree"] = (res["skew"]["sum"], res["skew"]["count"]) == (res["identity"]["sum"],
                                                                         res["identity"]["count"])
    return res


def bench_group_by(K, WU, dev, stream):
    """Grouped SUM/COUNT over 5e8 rows of Zipf(1.1) keys in 1e6 groups, values U[0,1000]."""
    import torch

    from paper_1910_10063_amd import skew
    from paper_1910_10063_amd import workload as W

    M, F, s = 1_000_000, 500_000_000, 1.1
    log(f"group-by M={M} F={F} s={s}")
    g = W.device_group_inputs(3, M, F, s, device=dev)
    G, V = g["keys"], g["vals"]
    bws = skew.workspace(skew.SKEW_OP_BUILD, F, M, dev)
    t0 = time.time()
    L = skew.build_skew_layout(G, M, ws=bws)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    gws = skew.workspace(skew.SKEW_OP_GROUP, F, M, dev)
    gws1 = skew.workspace(skew.SKEW_OP_GROUP_SINGLE_PASS, F, M, dev)
    out = (torch.empty(M, dtype=torch.int64, device=dev), torch.empty(M, dtype=torch.int64, device=dev))
    res = {}
    runs = (("skew", L.fact_recoded, skew.SKEW_HOT_AUTO, L.perm, gws),
            ("identity", G, 0, None, gws),                       # partitioned, no id-based privatisation
            ("skew_single_pass", L.fact_recoded, skew.SKEW_HOT_AUTO, L.perm, gws1),
            ("identity_hash_single_pass", G, 0, None, gws1),
            ("identity_atomic", G, skew.SKEW_HOT_NONE, None, gws1))
    for name, keys, t, perm, ws in runs:
        steps = K if name != "identity_atomic" else max(K // 4, 2)
        ms = timed(lambda: skew.group_aggregate(keys, V, M, hot_groups=t, perm=perm, ws=ws, out=out), steps,
                   1, stream)
        res[name] = {"ms": ms, "tuples_per_s": F / (ms * 1e-3),
                     "sum_digest": hashlib.sha256(out[0].cpu().numpy().tobytes() +
                                                  out[1].cpu().numpy().tobytes()).hexdigest()[:16]}
    # hot-group threshold sweep (Section 4.3's hybrid private/shared aggregation; Section 5.1 sweeps its
    # threshold): t_g groups privatised in LDS, the rest partitioned (large workspace) or sent to global
    # atomics (single pass); t_g = 0 is the layout-oblivious method of each form
    sweep = []
    for form, ws in (("partitioned", gws), ("single_pass", gws1)):
        cap = skew.max_hot_groups() if form == "partitioned" else skew.max_hot(skew.SKEW_OP_GROUP_SINGLE_PASS)
        for t in (0, 1024, 4096, 8192, cap):
            ms = timed(lambda: skew.group_aggregate(L.fact_recoded, V, M, hot_groups=t, perm=L.perm, ws=ws,
                                                    out=out), max(K // 2, 10), 1, stream)
            dg = hashlib.sha256(out[0].cpu().numpy().tobytes() + out[1].cpu().numpy().tobytes()).hexdigest()[:16]
            sweep.append({"form": form, "hot_groups": t, "ms": round(ms, 4), "tuples_per_s": F / (ms * 1e-3),
                          "same_result": dg == res["skew"]["sum_digest"]})
    # the library's threshold prior for the group-by
    ch = skew.group_choose(L.counts_by_rank, F)
    ws_ch = gws if ch["partitioned"] else gws1
    t_ch = ch["hot_rows"] if ch["hot_rows"] > 0 else (0 if ch["partitioned"] else skew.SKEW_HOT_NONE)
    ms_ch = timed(lambda: skew.group_aggregate(L.fact_recoded, V, M, hot_groups=t_ch, perm=L.perm, ws=ws_ch, out=out),
                  max(K // 2, 10), 1, stream)
    dg = hashlib.sha256(out[0].cpu().numpy().tobytes() + out[1].cpu().numpy().tobytes()).hexdigest()[:16]
    best = min(sweep, key=lambda r: r["ms"])
    model_choice = dict(ch, ms=round(ms_ch, 4), same_result=dg == res["skew"]["sum_digest"],
                        sweep_best={"form": best["form"], "hot_groups": best["hot_groups"], "ms": best["ms"]})
    skew.profile_report()
    skew.profile_enable(True)
    for _ in range(3):
        skew.group_aggregate(L.fact_recoded, V, M, hot_groups=skew.SKEW_HOT_AUTO, perm=L.perm, ws=gws, out=out)
    st = skew.profile_report()
    skew.profile_enable(False)
    stages = {k: {"ms": round(v[0] / 3, 4), "launches": round(v[1] / 3, 3)} for k, v in st.items()}
    alg = 8.0 * F + 16.0 * M
    ms = res["skew"]["ms"]
    return {"workload": f"group-aggregate: {M:.0e} groups, {F:.0e} rows, Zipf(s={s}) keys, values U[0,1000]",
            "runs": res, "speedup_vs_identity": res["identity"]["ms"] / ms,
            "speedup_vs_best_identity": min(r["ms"] for n, r in res.items() if n.startswith("identity")) / ms,
            "roofline_frac": alg / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "stages_ms": stages,
            "hot_group_sweep": sweep, "model_choice": model_choice,
            "build_s_incl_sync": build_s,
            "layouts_agree": len({r["sum_digest"] for r in res.values()}) == 1}


def bench_star(K, dev, stream):
    """64 star-join queries, fact sizes log-uniform in [1e5, 1e8], product dimension 1e7 rows (Zipf 1.0), customer
    dimension 2e6 rows (Zipf 0.8), 1-50 % customer filters, SUM(price) by 16 categories; one persistent kernel
    replayed from a HIP graph, tuning from the autotuner."""
    import numpy as np
    import torch

    from paper_1910_10063_amd import skew
    from paper_1910_10063_amd import workload as W

    k, n_prod, n_cust, nq = 4, 10_000_000, 2_000_000, 64
    sizes, lt, start = W.star_batch_spec(k, nq, 1e5, 1e8)
    total = int(start[-1])
    log(f"star batch: {nq} queries, {total} rows")
    d = W.device_star_inputs(k, n_prod, n_cust, sizes, device=dev)
    qs = torch.from_numpy(start).to(dev)
    ql = torch.from_numpy(lt).to(dev)
    ident = skew.StarBatch(d["prod"], d["cust"], qs, ql, d["price"], d["category"], d["cust_attr"])
    bws = skew.workspace(skew.SKEW_OP_BUILD, total, n_prod, dev)
    t0 = time.time()
    Lp = skew.build_skew_layout(d["prod"], n_prod, d["price"], d["category"], ws=bws)
    Lc = skew.build_skew_layout(d["cust"], n_cust, None, d["cust_attr"], ws=bws)
    torch.cuda.synchronize()
    build_s = time.time() - t0
    del bws
    sk = skew.StarBatch(Lp.fact_recoded, Lc.fact_recoded, qs, ql, Lp.price, Lp.category, Lc.category)
    ws = skew.star_workspace(sk)
    out = (torch.empty(nq, 16, dtype=torch.int64, device=dev), torch.empty(nq, 16, dtype=torch.int64, device=dev))
    t0 = time.time()
    best, best_ms = skew.star_join_autotune(sk, ws=ws)
    tune_s = time.time() - t0
    skew.star_join_batch(sk, best, ws=ws, out=out)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        skew.star_join_batch(sk, best, ws=ws, out=out)
    torch.cuda.synchronize()
    ms_graph = timed(g.replay, K, 1, stream)
    res_s = (out[0].cpu().numpy().copy(), out[1].cpu().numpy().copy())
    ms_eager = timed(lambda: skew.star_join_batch(sk, best, ws=ws, out=out), K, 1, stream)
    zero = skew.StarTuning(0, 0, best.tile_rows, 0)
    ms_ident = timed(lambda: skew.star_join_batch(ident, zero, ws=ws, out=out), K, 1, stream)
    res_i = (out[0].cpu().numpy().copy(), out[1].cpu().numpy().copy())
    ibest, ibest_ms = skew.star_join_autotune(ident, ws=ws)
    ms_ident_tuned = timed(lambda: skew.star_join_batch(ident, ibest, ws=ws, out=out), K, 1, stream)
    skew.profile_report()
    skew.profile_enable(True)
    for _ in range(3):
        skew.star_join_batch(sk, best, ws=ws, out=out)
    st = skew.profile_report()
    skew.profile_enable(False)
    kern_ms = st["star_batch"][0] / st["star_batch"][1]
    # two keys per row, the product prefix, and the customer segments the bitmaps are built from plus the bitmaps
    alg = 8.0 * total + 4.0 * best.prod_hot_rows + best.cust_hot_rows * (1.0 + nq / 8.0)
    res = {"workload": f"batched star join: {nq} queries, {total} fact rows (log-uniform 1e5..1e8), product "
                       f"{n_prod} rows Zipf(1.0), customer {n_cust} rows Zipf(0.8), 1-50 % customer filters, "
                       "SUM(price) by 16 categories",
           "total_rows": total, "graph_ms": ms_graph, "tuples_per_s": total / (ms_graph * 1e-3),
           "eager_ms": ms_eager, "identity_ms": ms_ident, "identity_autotuned_ms": ms_ident_tuned,
           "speedup_vs_identity": min(ms_ident, ms_ident_tuned) / ms_graph,
           "tuning": {"prod_hot_rows": best.prod_hot_rows, "cust_hot_rows": best.cust_hot_rows,
                      "tile_rows": best.tile_rows, "blocks": best.blocks, "autotune_best_ms": best_ms,
                      "autotune_s": tune_s},
           "identity_tuning": {"prod_hot_rows": ibest.prod_hot_rows, "cust_hot_rows": ibest.cust_hot_rows,
                               "tile_rows": ibest.tile_rows},
           "kernel_ms": kern_ms, "roofline": {"bound": "hbm", "algorithmic_bytes": alg,
                                              "achieved_GBps": alg / (kern_ms * 1e-3) / 1e9,
                                              "frac": alg / (kern_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
           "layout_build_s": build_s,
           "layouts_agree": bool((res_s[0] == res_i[0]).all() and (res_s[1] == res_i[1]).all())}
    del d, Lp, Lc, sk, ident, ws, g
    torch.cuda.empty_cache()
    return res


def bench_serve(seconds, dev):
    """Serving loop: Poisson arrivals at 200 requests/s of grouped aggregations over row ranges (log-uniform
    1e5..5e8 rows) of the resident group-by table (5e8 rows, 1e6 groups, Zipf 1.1); slots from a 64 GB memory
    budget (9 GB per slot: the partitioned group-by's workspace for 5e8 rows); at 15 s 1e7 rows are inserted (recoded through the current layout, no rebuild); at 30 s a new table
    version with re-permuted popularity arrives (drift, rebuild)."""
    import torch

    from paper_1910_10063_amd import serving
    from paper_1910_10063_amd import workload as W

    M, F = 1_000_000, 500_000_000
    log(f"serving: {seconds} s at 200 requests/s")
    tabs = []
    for v, k in ((1, 3), (2, 13)):
        g = W.device_group_inputs(k, M, F, 1.1, device=dev)
        tabs.append(serving.TableVersion(v, g["keys"], g["vals"], M))
    budget = 64 << 30
    max_rows = F
    slots = serving.plan_slots(budget, max_rows, M)
    srv = serving.Server(tabs[0], slots, max_rows)
    t0 = time.time()
    serving.start_layout(srv, tabs[0])
    first_build_s = time.time() - t0
    # at 15 s, 1e7 rows (keys resampled from the table) are inserted and served on the current layout without a
    # rebuild (Section 3.1's maintenance); at 30 s a version with re-permuted popularity arrives (drift, rebuild)
    n_ins = 10_000_000
    g = torch.Generator(device=dev).manual_seed(19)
    pick = torch.randint(0, F, (n_ins,), device=dev, generator=g)
    ins = serving.InsertBatch(tabs[0].keys[pick].contiguous(), tabs[0].vals[pick].contiguous())
    arr = serving.poisson_arrivals(200.0, float(seconds), 17)
    reqs = serving.make_requests(arr, F + n_ins, 100_000, F, 17)
    versions = [(15.0, ins)] if seconds > 15 else []
    versions += [(30.0, tabs[1])] if seconds > 30 else []
    done = srv.run(reqs, versions)
    rep = serving.latency_report(done)
    rep.update({"workload": f"grouped aggregation requests over row ranges of a {F:.0e}-row, {M:.0e}-group "
                            "Zipf(1.1) table, Poisson 200/s, ranges log-uniform 1e5..5e8 rows",
                "seconds": seconds, "slots": slots, "memory_budget_bytes": budget,
                "slot_bytes": serving.slot_bytes(max_rows, M), "first_layout_build_s": first_build_s,
                "events": srv.events})
    del srv, tabs
    torch.cuda.empty_cache()
    return rep


def bench_cache_model(cbr, rank, N, F, dev):
    """Section 3.3's model for the dimension lookups: 128-byte lines of 32 values, one XCD's 4 MB L2
    (32768 lines; each XCD sees the whole access distribution) and the 256 MB memory-side cache."""
    import torch

    from paper_1910_10063_amd import skew

    ws = skew.workspace(skew.SKEW_OP_CACHE_MODEL, 0, N, dev)
    t0 = time.time()
    out = {"values_per_line": 32}
    for name, S in (("l2", 32768), ("mall", 2_097_152)):
        out[f"{name}_lines"] = S
        out[f"{name}_hit_skew"] = skew.cache_model_hit_rate(cbr, S, 32, ws=ws)
        out[f"{name}_hit_identity"] = skew.cache_model_hit_rate(cbr, S, 32, rank=rank, ws=ws)
    out["seconds_for_4_evaluations"] = round(time.time() - t0, 3)
    t = skew.join_hot_rows(F, N, True)
    out["lds_prefix_rows"] = t
    out["lds_prefix_share"] = float(cbr[:t].to(torch.int64).sum().item()) / F
    return out


def bench_operators(K, C, price, Cp, pp, perm, N, F, dev, stream):
    """Q1 materialization, Q2 selection and Q3a heavy hitters (Section 4.1) on the join workload, both layouts."""
    import torch

    from paper_1910_10063_amd import skew

    steps = max(K // 2, 3)
    res = {}
    # Q1: out[j] = price[key[j]]: 4 B key read + 4 B written per row, plus the dimension column once
    log("operators: materialize")
    mws = skew.workspace(skew.SKEW_OP_MATERIALIZE, F, N, dev)
    out = torch.empty_like(C)
    ms_s = timed(lambda: skew.materialize_column(Cp, pp, ws=mws, out=out), steps, 1, stream)
    d_s = hashlib.sha256(out[:: 997].cpu().numpy().tobytes()).hexdigest()[:16]
    ms_i = timed(lambda: skew.materialize_column(C, price, hot_rows=0, ws=mws, out=out), steps, 1, stream)
    d_i = hashlib.sha256(out[:: 997].cpu().numpy().tobytes()).hexdigest()[:16]
    alg = 8.0 * F + 4.0 * N
    res["materialize"] = {"skew_ms": ms_s, "identity_ms": ms_i, "skew_tuples_per_s": F / (ms_s * 1e-3),
                          "identity_tuples_per_s": F / (ms_i * 1e-3), "speedup": ms_i / ms_s,
                          "roofline_frac": alg / (ms_s * 1e-3) / 1e9 / HBM_PEAK_GBS, "layouts_agree": d_s == d_i}
    # Q2: offsets of the rows with price < 100 (about 1 % of U[1, 10000])
    log("operators: select")
    sws = skew.workspace(skew.SKEW_OP_SELECT, F, N, dev)
    cnt = torch.empty(1, dtype=torch.int64, device=dev)
    ms_s = timed(lambda: skew.select_fact_rows(Cp, pp, 100, ws=sws, out=(out, cnt)), steps, 1, stream)
    n_s = int(cnt.item())
    d_s = hashlib.sha256(out[:n_s].cpu().numpy().tobytes()).hexdigest()[:16]
    ms_i = timed(lambda: skew.select_fact_rows(C, price, 100, hot_rows=0, ws=sws, out=(out, cnt)), steps, 1, stream)
    n_i = int(cnt.item())
    d_i = hashlib.sha256(out[:n_i].cpu().numpy().tobytes()).hexdigest()[:16]
    res["select"] = {"predicate": "price < 100", "selected": n_s, "skew_ms": ms_s, "identity_ms": ms_i,
                     "skew_tuples_per_s": F / (ms_s * 1e-3), "identity_tuples_per_s": F / (ms_i * 1e-3),
                     "speedup": ms_i / ms_s, "layouts_agree": (n_s, d_s) == (n_i, d_i)}
    del sws
    # Q3a: counts of the 4000 most frequent keys on the skew layout, against the full grouped
    # aggregate (SUM(price), COUNT(*) per key) on the identity layout, the conventional method
    log("operators: heavy hitters")
    hws = skew.workspace(skew.SKEW_OP_HEAVY, F, N, dev)
    ms_h = timed(lambda: skew.heavy_hitter_counts(Cp, N, 4000, perm=perm, ws=hws), steps, 1, stream)
    hk, hc = skew.heavy_hitter_counts(Cp, N, 4000, perm=perm, ws=hws)
    skew.materialize_column(C, price, ws=mws, out=out)  # the value column of the full aggregate
    gws = skew.workspace(skew.SKEW_OP_GROUP, F, N, dev)
    gout = (torch.empty(N, dtype=torch.int64, device=dev), torch.empty(N, dtype=torch.int64, device=dev))
    ms_f = timed(lambda: skew.group_aggregate(C, out, N, hot_groups=0, ws=gws, out=gout), max(K // 4, 2), 1, stream)
    agree = bool((gout[1][hk.long()] == hc).all().item())
    res["heavy_hitters"] = {"k": 4000, "skew_ms": ms_h, "skew_tuples_per_s": F / (ms_h * 1e-3),
                            "identity_full_aggregate_ms": ms_f, "speedup_vs_full_aggregate": ms_f / ms_h,
                            "roofline_frac": 4.0 * F / (ms_h * 1e-3) / 1e9 / HBM_PEAK_GBS,
                            "counts_agree_with_full_aggregate": agree}
    del gws, gout, out, hws, mws
    torch.cuda.empty_cache()
    return res


def cpu_baseline(C, price, cat, rows, gpu_res, repeats=3, layout=None):
    """The CPU oracle, as it stands, on the first `rows` fact rows of the identity layout: median of `repeats`
    runs on one thread, then median of `repeats` runs on every host core this process may use, up to the 16
    cores that one GPU's share of the host grants (contiguous chunks of the column, one per thread; the
    foreign call releases the interpreter lock; partial sums added in chunk order).  With `layout` (recoded
    keys, permuted price and category), the same one-thread loop also runs over the frequency-ordered layout:
    the paper's CPU effect of the layout, on this host."""
    import concurrent.futures as cf

    import numpy as np

    import oracle

    n = min(rows, C.numel())
    log(f"cpu oracle on {n} rows, {repeats} runs on one thread")
    Ch = C[:n].cpu().numpy()
    ph = price.cpu().numpy()
    ch = cat.cpu().numpy()
    times = []
    for _ in range(repeats):
        t = time.perf_counter()
        s, c = oracle.fk_join_aggregate(Ch, ph, ch, 16, True)
        times.append(time.perf_counter() - t)
    dt = dt_one = float(np.median(times))
    out = {"value": n / dt, "unit": "fact tuples/s", "cores": 1, "kind": "oracle",
           "sample": f"first {n} of {C.numel()} fact rows, identity layout, same query; median of {repeats} runs "
                     f"on 1 thread: {dt:.2f} s", "runs_s": [round(x, 3) for x in times], "cpu_model": _cpu_model()}
    if gpu_res is not None:
        out["bit_exact_vs_oracle"] = bool((s == gpu_res[0]).all() and (c == gpu_res[1]).all())
    affinity = len(os.sched_getaffinity(0))
    cores = min(16, affinity)
    log(f"cpu oracle on {cores} threads ({affinity} cores in the affinity mask)")
    bounds = np.linspace(0, n, cores + 1).astype(np.int64)
    times = []
    with cf.ThreadPoolExecutor(cores) as ex:
        for _ in range(repeats):
            t = time.perf_counter()
            parts = list(ex.map(lambda i: oracle.fk_join_aggregate(Ch[bounds[i]:bounds[i + 1]], ph, ch, 16, True),
                                range(cores)))
            times.append(time.perf_counter() - t)
    dt = float(np.median(times))
    sp = np.sum([p[0] for p in parts], axis=0)
    cp = np.sum([p[1] for p in parts], axis=0)
    out["all_cores"] = {"value": n / dt, "unit": "fact tuples/s", "cores": cores, "affinity_cores": affinity,
                        "kind": "oracle",
                        "sample": f"the same {n} rows in {cores} contiguous chunks, one thread each; median of "
                                  f"{repeats} runs: {dt:.2f} s", "runs_s": [round(x, 3) for x in times],
                        "equals_one_thread": bool((sp == s).all() and (cp == c).all())}
    if layout is not None:
        log(f"cpu oracle on the frequency-ordered layout, {repeats} runs on one thread")
        Lk, Lp, Lc = layout[0][:n].cpu().numpy(), layout[1].cpu().numpy(), layout[2].cpu().numpy()
        times = []
        for _ in range(repeats):
            t = time.perf_counter()
            s2, c2 = oracle.fk_join_aggregate(Lk, Lp, Lc, 16, True)
            times.append(time.perf_counter() - t)
        dt2 = float(np.median(times))
        out["skew_layout"] = {"value": n / dt2, "unit": "fact tuples/s", "cores": 1, "kind": "oracle",
                              "sample": f"the same {n} rows recoded, with the permuted dimension; median of "
                                        f"{repeats} runs on 1 thread: {dt2:.2f} s",
                              "runs_s": [round(x, 3) for x in times], "speedup_vs_identity": dt_one / dt2,
                              "equals_identity": bool((s2 == s).all() and (c2 == c).all())}
    return out


def cpu_baseline_rows(n=20_000_000):
    """The oracle timed on bounded samples of every other row's workload (one thread each): the first n
    rows of the same seeded columns the device sections use (the generators are counter-based)."""
    import numpy as np

    import oracle
    from paper_1910_10063_amd import workload as W

    out = {}

    def timed_cpu(name, fn, rows, sample):
        t = time.perf_counter()
        fn()
        dt = time.perf_counter() - t
        out[name] = {"value": rows / dt, "unit": "tuples/s", "cores": 1, "kind": "oracle",
                     "sample": f"{sample}; {dt:.2f} s on 1 thread"}

    log(f"cpu oracle samples of {n} rows")
    h = W.host_join_inputs(2, 10_000_000, n, 1.0)
    timed_cpu("build_layout", lambda: oracle.build_layout(h["fact"], 10_000_000, h["price"], h["category"]), n,
              f"first {n} keys of the 1e9-key join column, N = 1e7")
    timed_cpu("materialize", lambda: oracle.materialize(h["fact"], h["price"]), n, f"first {n} keys of the join column")
    timed_cpu("select", lambda: oracle.select(h["fact"], h["price"], 100), n, f"first {n} keys, price < 100")
    timed_cpu("heavy_hitters", lambda: oracle.heavy_hitters(h["fact"], 10_000_000, 4000), n,
              f"first {n} keys, k = 4000 (count every key, then sort)")
    del h
    g = W.host_group_inputs(3, 1_000_000, n, 1.1)
    timed_cpu("group_by", lambda: oracle.group_aggregate(g["keys"], g["vals"], 1_000_000), n,
              f"first {n} rows of the 5e8-row group-by table")
    del g
    sizes, lt, start = W.star_batch_spec(4, 64, 1e5, 1e8)
    m = min(n, int(start[-1]))
    st = W.host_star_inputs(4, 10_000_000, 2_000_000, np.array([m]))  # rows [0, m) of the batch columns
    cuts = [int(x) for x in start if x < m] + [m]

    def star():
        for i in range(len(cuts) - 1):  # each piece of [0, m) with the threshold of its query
            a, b = cuts[i], cuts[i + 1]
            if b > a:
                oracle.star_join(st["prod"][a:b], st["cust"][a:b], st["price"], st["category"], st["cust_attr"],
                                 int(lt[i]))

    timed_cpu("star_batch", star, m, f"the first {m} rows of the batch, each with its query's threshold")
    return out


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
