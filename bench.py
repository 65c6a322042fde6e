#!/usr/bin/env python3
"""Benchmark of the triangular-domain hot path on one MI355X.

Default workload (one "step"): the global-memory triangular elementwise
kernel C[i][j] = a X[i][j] + Y[j][i] over the lower triangle (diagonal
included) of n = 32768 FP32 matrices in full n x n storage, lambda(omega)
map, one launch per step, inputs resident in HBM.  Prints ONE JSON line.

The same line carries, under "extra", the other workloads measured on the
same run: lambda vs bounding box at n = 2048 (int32), the triangular Game of
Life (n = 16384, 100 steps), and the distance map (n = 65536, d = 128).

    python bench.py [--steps K] [--warmup W] [--tile 0=autotuned] [--map lambda]
                    [--no-extra] [--no-cpu] [--gpus 1]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


class Timer:
    """HIP events on the stream the kernels are launched on."""

    def __init__(self, torch):
        self.torch = torch

    def run(self, fn, steps, warmup):
        torch = self.torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(steps):
            fn()
        e1.record(s)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps  # ms per call

    def interleaved(self, fns, reps, warmup, reset=None):
        """Medians of several functions timed in turn (one call of each per
        round, each between its own pair of events), so that none of them
        is favoured by its place in the run; reset() runs before every call,
        outside the timed region."""
        torch = self.torch
        for _ in range(warmup):
            for f in fns:
                if reset:
                    reset()
                f()
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        times = [[] for _ in fns]
        for _ in range(reps):
            for k, f in enumerate(fns):
                if reset:
                    reset()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record(s)
                f()
                e1.record(s)
                torch.cuda.synchronize()
                times[k].append(e0.elapsed_time(e1))
        return [float(np.median(t)) for t in times]

    def median(self, fn, reps, warmup):
        """Median over `reps` calls, each between its own pair of events."""
        torch = self.torch
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        s = torch.cuda.current_stream()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(reps + 1)]
        ev[0].record(s)
        for r in range(reps):
            fn()
            ev[r + 1].record(s)
        torch.cuda.synchronize()
        return float(np.median([ev[r].elapsed_time(ev[r + 1]) for r in range(reps)]))


def src_digest(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1609_01490_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profile_value(kernel_tag: str, field: str, digest: str):
    """A figure measured with rocprofv3 counters (e.g. hbm_bytes_per_launch:
    FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known size;
    mfma_busy: the matrix cores' busy fraction), recorded under profiles/
    with the digest of the kernel sources it was taken on.  None when no
    record matches the current sources."""
    pdir = os.path.join(ROOT, "profiles")
    if not os.path.isdir(pdir):
        return None
    for fn in sorted(os.listdir(pdir)):
        if not fn.endswith(".md"):
            continue
        txt = open(os.path.join(pdir, fn)).read()
        if f"traffic_kernel: {kernel_tag}" not in txt:
            continue
        m_d = re.search(r"src_digest: (\w+)", txt)
        m_b = re.search(field + r": ([0-9.eE+]+)", txt)
        if m_d and m_b and m_d.group(1) == digest:
            return float(m_b.group(1))
    return None


def traffic_from_profiles(kernel_tag: str, digest: str):
    return profile_value(kernel_tag, "hbm_bytes_per_launch", digest)


def host_threads():
    """Worker threads for the oracle on this host: the CPUs this process may
    run on, at most 16 (one GPU's share of a shared host)."""
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count() or 1
    return max(1, min(16, avail))


def host_cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline_elementwise(a, X, Y, passes=3):
    """The oracle (plain C, no GIL while it runs) on the whole workload: the
    triangle split into bands of 64 rows handed to a pool of host threads,
    each band written to the thread's own buffer; `passes` passes, the
    median reported."""
    import concurrent.futures as cf
    import threading
    import oracle
    n = X.shape[0]
    threads = host_threads()
    local = threading.local()

    def band(r0):
        out = getattr(local, "out", None)
        if out is None:
            out = local.out = np.empty((64, n), dtype=np.float32)
        oracle.c1(a, X, Y, out, r0=r0, r1=min(n, r0 + 64))

    # heaviest bands first, so the last ones to finish are short
    starts = list(range(0, n, 64))[::-1]
    times = []
    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(band, starts[:threads]))  # first touch of the thread buffers
        for _ in range(passes):
            t0 = time.perf_counter()
            list(ex.map(band, starts))
            times.append(time.perf_counter() - t0)
    dt = float(np.median(times))
    E = n * (n + 1) // 2
    return {"value": E / dt, "unit": "elements/s", "cores": threads, "kind": "oracle",
            "host_cpus": os.cpu_count(), "cpu_model": host_cpu_model(),
            "sample": f"the whole n={n} fp32 elementwise triangle ({E} cells) in "
                      f"{len(starts)} bands of 64 rows on {threads} threads, median of "
                      f"{passes} passes ({dt:.2f} s each)"}


def tune_table(tm, workload, n, d=0, reps=3):
    """Every tile x map candidate timed by the library's autotuner."""
    tm.tune_cache_clear()
    best, allc = tm.autotune(workload, n, d, reps=reps, use_cache=False)
    return best, allc


def best_of(table, map_name):
    c = [x for x in table if x["map"] == map_name]
    return min(c, key=lambda x: x["ms"]) if c else None


def bench_elementwise(tm, torch, args, timer):
    from paper_1609_01490_amd import inputs
    n = 32768
    log("generating fp32 inputs", n)
    a, X, Y, _ = inputs.f32_elementwise(n, with_fill=False)
    xd = torch.from_numpy(X).cuda()
    yd = torch.from_numpy(Y).cuda()
    c = torch.empty((n, n), dtype=torch.float32, device="cuda")
    E = n * (n + 1) // 2
    # tile and swizzle of each map from the autotuner (all maps x tiles timed)
    _, table = tune_table(tm, tm.TUNE_ELEMENTWISE_F32, n)
    lam = best_of(table, args.map)
    bb = best_of(table, "bb")
    tile = args.tile or lam["tile"]
    flags = args.flags if args.tile else lam["flags"]
    res = {}
    for map_name, t_, f_ in ((args.map, tile, flags), ("bb", args.tile or bb["tile"], 0)):
        p = tm.Plan(n, t_, map_name, flags=f_)
        ms = timer.run(lambda: p.elementwise(tm.OP_AXPYT_F32, xd, yd, c, ld=n, a=float(a)),
                       args.steps, args.warmup)
        res[map_name] = (ms, t_, f_)
        log(f"elementwise {map_name} tile {t_} flags {f_}: {ms:.4f} ms")
    # streaming ceiling: c = x + y over the same 3 x 4 GiB buffers
    flat = [t.view(-1) for t in (c, xd, yd)]
    ms_add = timer.run(lambda: tm.stream_add(*flat), args.steps, args.warmup)
    res["stream_add_GBps"] = 12 * n * n / (ms_add * 1e-3) / 1e9
    log(f"stream add (12 B per element over {n}x{n}): {ms_add:.4f} ms, "
        f"{res['stream_add_GBps']:.0f} GB/s")
    if not args.no_extra:
        res["probes"] = bench_probes(tm, torch, timer, c, xd, yd)
    cpu = None if args.no_cpu else cpu_baseline_elementwise(a, X, Y)
    del xd, yd, c
    torch.cuda.empty_cache()
    return n, E, res, cpu, table


def named_tiles(table, E, headline_GBps):
    """Tiles 16 and 32 (the tiles the elementwise workload names), from the
    autotuner's table: for each map its fastest candidate with one tile per
    workgroup (flags without strip bits) and with strips (TRI_FLAG_STRIP),
    HBM GB/s (12 B per cell), I = t_BB / t_map within each form, and
    lambda's bandwidth over the headline launch's."""
    out = {}
    for t in (16, 32):
        row = {}
        for form, want_strip in (("per_tile", False), ("strips", True)):
            best = {}
            for c in table:
                if c["tile"] != t or bool(c["flags"] & 0xF00) != want_strip:
                    continue
                if c["map"] not in best or c["ms"] < best[c["map"]]["ms"]:
                    best[c["map"]] = c
            if not best:
                continue
            ent = {mp: {"ms": round(c["ms"], 4), "flags": c["flags"],
                        "GBps": round(12 * E / (c["ms"] * 1e-3) / 1e9, 1)} for mp, c in best.items()}
            if "bb" in best:
                for mp, c in best.items():
                    ent[mp]["I_vs_bb"] = round(best["bb"]["ms"] / c["ms"], 4)
            if "lambda" in best:
                ent["lambda_vs_headline_bw"] = round(ent["lambda"]["GBps"] / headline_GBps, 4)
            row[form] = ent
        out[f"t{t}"] = row
    return out


def bench_probes(tm, torch, timer, c, x, y):
    """The bandwidth a plain streaming kernel reaches for each access mix
    (read, two reads and one write, write, copy) over the same 4 GiB
    buffers as the elementwise workload: a sweep of vectors in flight per
    thread, workgroup size, cache policy and grid (one chunk per workgroup,
    or 8 persistent workgroups per CU), each timed as the median of 5
    launches.  Bytes counted: 4 GiB per read or written buffer."""
    flat = [t.view(-1) for t in (c, x, y)]
    nbytes = flat[0].numel() * 4
    streams = {tm.PROBE_READ: 1, tm.PROBE_ADD: 3, tm.PROBE_FILL: 1, tm.PROBE_COPY: 2}
    names = {tm.PROBE_READ: "read", tm.PROBE_ADD: "add_2r1w", tm.PROBE_FILL: "fill",
             tm.PROBE_COPY: "copy_1r1w"}
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    out = {}
    for kind in (tm.PROBE_READ, tm.PROBE_ADD, tm.PROBE_FILL, tm.PROBE_COPY):
        table = {}
        for unroll in (1, 2, 4, 8):
            for threads in (256, 512, 1024):
                for nt in (False, True):
                    for wg in (0, 8 * cus):
                        fn = lambda: tm.stream_probe(kind, flat[0], flat[1], flat[2],
                                                     unroll=unroll, threads=threads,
                                                     nontemporal=nt, workgroups=wg)
                        ms = timer.median(fn, 5, 1)
                        key = f"u{unroll}/t{threads}/{'nt' if nt else 'c'}/" + \
                              ("persistent" if wg else "chunked")
                        table[key] = round(streams[kind] * nbytes / (ms * 1e-3) / 1e9, 1)
        best = max(table, key=table.get)
        out[names[kind]] = {"best": best, "best_GBps": table[best],
                            "best_frac_of_hbm": round(table[best] / HBM_PEAK_GBS, 4),
                            "GBps": table}
        log(f"probe {names[kind]}: best {best} {table[best]:.0f} GB/s")
    return out


def graph_time(torch, timer, fn, launches):
    """GPU time per call of fn (ms) from a captured graph of `launches`
    back-to-back calls, so that short launches are not host-bound."""
    fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            for _ in range(launches):
                fn()
    torch.cuda.synchronize()
    ms = timer.run(lambda: g.replay(), 5, 1) / launches
    del g
    return ms


def bench_int_elementwise(tm, torch, timer, tile=16, launches=200):
    """n = 2048 int32, lambda vs BB (and the other maps): GPU time per launch
    from a captured graph of `launches` back-to-back launches (a single
    launch is a few microseconds, below the host's launch rate)."""
    from paper_1609_01490_amd import inputs
    n = 2048
    A, B, C0 = inputs.int_elementwise(n)
    ad, bd, cd = (torch.from_numpy(v).cuda() for v in (A, B, C0))
    out = {}
    for t_ in (8, 16, 32):
        for map_name in ("lambda", "bb", "rb", "rec", "utm"):
            if map_name == "utm" and t_ != tile:
                continue
            p = tm.Plan(n, t_, map_name)
            fn = lambda: p.elementwise(tm.OP_XORMUL_I32, ad, bd, cd, ld=n)
            fn()
            torch.cuda.synchronize()
            g = torch.cuda.CUDAGraph()
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                with torch.cuda.graph(g, stream=s):
                    for _ in range(launches):
                        fn()
            torch.cuda.synchronize()
            ms = timer.run(lambda: g.replay(), 5, 1) / launches
            out[f"{map_name}/t{t_}"] = round(ms * 1e3, 3)
            del g
    return {"n": n, "tile": tile, "us_per_launch_graph": out,
            "I_lambda_vs_bb": round(out[f"bb/t{tile}"] / out[f"lambda/t{tile}"], 4)}


def bench_life(tm, torch, timer, steps=100, reps=7):
    """Life n = 16384, 100 generations.  The autotuner ranks every map x tile
    (x temporal blocking) candidate on that same schedule (one timed call =
    100 generations, median of 5 calls); lambda and BB then each run at
    their best candidate, timed as the median of `reps` calls of 100
    generations.  The paper's form (one generation per launch, 1-cell halo)
    is timed the same way at each map's best one-generation candidate."""
    from paper_1609_01490_amd import inputs
    n = 16384
    tm.tune_cache_clear()
    _, table = tm.autotune(tm.TUNE_LIFE, n, steps, reps=5, use_cache=False)
    g = inputs.life(n, 0.3)
    g0 = torch.from_numpy(g).cuda()
    cur = g0.clone()
    nxt = torch.zeros_like(cur)
    reset = lambda: cur.copy_(g0)  # every timed call starts from generation 0
    out, one = {}, {}
    one_gen = [c for c in table if not c["flags"] & tm.FLAG_LIFE_TEMPORAL]
    # lambda and BB timed in turn, each call from the same grid
    chs = {m: best_of(table, m) for m in ("lambda", "bb")}
    c1s = {m: best_of(one_gen, m) for m in ("lambda", "bb")}
    plans = {m: tm.Plan(n, chs[m]["tile"], m, flags=chs[m]["flags"]) for m in chs}
    plans1 = {m: tm.Plan(n, c1s[m]["tile"], m, flags=c1s[m]["flags"]) for m in c1s}
    t = timer.interleaved([lambda: plans["lambda"].stencil(cur, nxt, steps),
                           lambda: plans["bb"].stencil(cur, nxt, steps)], reps, 1, reset)
    t1 = timer.interleaved([lambda: plans1["lambda"].stencil(cur, nxt, steps),
                            lambda: plans1["bb"].stencil(cur, nxt, steps)], reps, 1, reset)
    for k, map_name in enumerate(("lambda", "bb")):
        ch, c1 = chs[map_name], c1s[map_name]
        out[map_name] = {"ms": round(t[k], 4), "tile": ch["tile"], "flags": ch["flags"],
                         "tuned_ms_per_generation": round(ch["ms"], 5)}
        one[map_name] = {"ms": round(t1[k], 4), "tile": c1["tile"], "flags": c1["flags"]}
    cells = n * (n + 1) // 2
    del cur, nxt, g0
    torch.cuda.empty_cache()
    lam = out["lambda"]["ms"]
    lam1 = one["lambda"]["ms"]
    copy = same_size_copy(tm, torch, cells)
    return {"n": n, "steps": steps,
            "timing": f"median of {reps} calls of {steps} generations, lambda and BB in turn, "
                      f"each call from the same initial grid",
            "ms_100_steps": out,
            "cell_updates_per_s": round(cells * steps / (lam * 1e-3), 1),
            "generation_work_GBps": round(2 * cells * steps / (lam * 1e-3) / 1e9, 1),
            "I_lambda_vs_bb": round(out["bb"]["ms"] / lam, 4),
            "one_generation_per_launch_ms_100_steps": one,
            "one_generation_I_lambda_vs_bb": round(one["bb"]["ms"] / lam1, 4),
            # one generation per launch moves 2 B per cell (read + write):
            # that is a true HBM figure, unlike the temporal path's
            "one_generation_GBps": round(2 * cells * steps / (lam1 * 1e-3) / 1e9, 1),
            "one_generation_frac_of_hbm": round(2 * cells * steps / (lam1 * 1e-3) / 1e9
                                                / HBM_PEAK_GBS, 4),
            # a plain copy of one generation's bytes, back to back in ping-pong
            # as the generations run: the rate a launch of this size reaches
            "copy_same_size": copy,
            "one_generation_frac_of_same_size_copy": round(
                2 * cells * steps / (lam1 * 1e-3) / 1e9 / copy["best_GBps"], 4),
            "per_generation_ms_by_map_tile": {f"{c['map']}/t{c['tile']}/f{c['flags']}":
                                              round(c["ms"], 5) for c in table}}


def same_size_copy(tm, torch, nbytes, pairs=50):
    """The streaming probe's copy over nbytes (read and written), launched
    back to back in ping-pong (a -> c, c -> a) like the generations of a
    grid, at unroll 1, 256 or 512 threads, cached or non-temporal: the best
    rate, counting 2 nbytes per launch."""
    cnt = nbytes // 4
    a = torch.rand(cnt, device="cuda")
    c = torch.empty_like(a)
    table = {}
    for threads in (256, 512):
        for nt in (False, True):
            def pair():
                tm.stream_probe(tm.PROBE_COPY, c, a, unroll=1, threads=threads, nontemporal=nt)
                tm.stream_probe(tm.PROBE_COPY, a, c, unroll=1, threads=threads, nontemporal=nt)
            for _ in range(5):
                pair()
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(pairs):
                pair()
            e1.record()
            torch.cuda.synchronize()
            us = e0.elapsed_time(e1) * 1e3 / (2 * pairs)
            table[f"t{threads}/{'nt' if nt else 'c'}"] = round(2 * 4 * cnt / (us * 1e-6) / 1e9, 1)
    del a, c
    torch.cuda.empty_cache()
    best = max(table, key=table.get)
    return {"bytes_each_way": 4 * cnt, "best": best, "best_GBps": table[best],
            "best_frac_of_hbm": round(table[best] / HBM_PEAK_GBS, 4), "GBps": table}


def edm_sample_rows(n, pairs):
    """4096 seeded random rows plus the row of every near-duplicate pair."""
    rng = np.random.default_rng(4096)
    return sorted(set(rng.choice(np.arange(1, n), 4096, replace=False).tolist())
                  | set(pairs.max(axis=1).tolist()))


def edm_oracle_rows(X, rows):
    """FP64 oracle distances of whole rows, on the host's threads (the
    oracle's C loop runs without the GIL)."""
    import concurrent.futures as cf
    import oracle
    oracle.lib()
    threads = host_threads()
    chunks = [rows[k::4 * threads] for k in range(4 * threads)]
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(threads) as ex:
        res = list(ex.map(lambda c: oracle.edm_rows(X, c), chunks))
    dt = time.perf_counter() - t0
    exp = {}
    for c, es in zip(chunks, res):
        exp.update(zip(c, es))
    return exp, dt, threads


def edm_rows_error(torch, out, rows, exp):
    """Max and 99.9th-percentile relative error of the device distances of
    the given whole rows against the oracle's."""
    offs = [r * (r - 1) // 2 for r in rows]
    got = torch.cat([out[o:o + r] for o, r in zip(offs, rows)]).cpu().numpy()
    rels, worst, k = [], 0.0, 0
    for r in rows:
        g = got[k:k + r].astype(np.float64)
        k += r
        e = exp[r]
        nz = e > 0
        rel = np.abs(g[nz] - e[nz]) / e[nz]
        if rel.size:
            worst = max(worst, float(rel.max()))
            rels.append(rel.astype(np.float32))
    allrel = np.concatenate(rels)
    return worst, float(np.percentile(allrel, 99.9)), int(allrel.size)


def bench_edm(tm, torch, timer, check=True):
    from paper_1609_01490_amd import inputs
    n, d = 65536, 128
    X, dup_pairs = inputs.points(n, d)
    xd = torch.from_numpy(X).cuda()
    out = torch.empty((n * (n - 1) // 2,), dtype=torch.float32, device="cuda")
    pairs = n * (n - 1) // 2
    res = {}
    p = tm.Plan(n, 128, "lambda", include_diag=False)
    ms = timer.run(lambda: p.edm(xd, out, mode=tm.EDM_FP32), 3, 1)
    res["fp32_tile"] = 128
    res["fp32_ms"] = round(ms, 4)
    res["fp32_pairs_per_s"] = round(pairs / (ms * 1e-3), 1)
    _, table = tune_table(tm, tm.TUNE_EDM_BF16X3, n, d, reps=3)
    best = best_of(table, "lambda")  # the lambda variant (swizzle, order) the autotuner finds fastest
    q = tm.Plan(n, 128, "lambda", include_diag=False, flags=best["flags"])
    res["mfma_map"] = best["map"]
    res["mfma_flags"] = best["flags"]
    # the autotuner's BF16X3 timings of every map at tile 128, and I = t_BB / t_map
    res["bf16x3_tune_ms_by_map"] = {f"{c['map']}/f{c['flags']}": round(c["ms"], 4) for c in table}
    bb = [c["ms"] for c in table if c["map"] == "bb"]
    if bb:
        res["bf16x3_I_vs_bb"] = {k: round(bb[0] / v, 4)
                                 for k, v in res["bf16x3_tune_ms_by_map"].items()}
    rows = exp = None
    if check:
        rows = edm_sample_rows(n, dup_pairs)
        exp, dt, thr = edm_oracle_rows(X, rows)
        res["accuracy_rows"] = (f"{len(rows)} whole rows: 4096 seeded random rows and the row "
                                f"of every one of the {len(dup_pairs)} near-duplicate pairs; "
                                f"FP64 oracle on {thr} host threads, {dt:.1f} s")
    digest = src_digest("edm.hip", "maps.hpp")
    for mode, name in ((tm.EDM_BF16X3, "bf16x3"), (tm.EDM_BF16, "bf16")):
        ws = torch.empty(q.edm_workspace_size(d, mode), dtype=torch.uint8, device="cuda")
        # the GPU idled during the host oracle above: warm up for longer,
        # then the median of single launches
        ms = timer.median(lambda: q.edm(xd, out, mode=mode, fixup_thr=1e-2, ws=ws), 9, 8)
        res[f"{name}_ms"] = round(ms, 4)
        res[f"{name}_pairs_per_s"] = round(pairs / (ms * 1e-3), 1)
        res[f"{name}_write_GBps"] = round(4 * pairs / (ms * 1e-3) / 1e9, 1)
        res[f"{name}_frac_of_hbm_write"] = round(4 * pairs / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)
        res[f"{name}_speedup_vs_fp32"] = round(res["fp32_ms"] / ms, 3)
        if check:
            # the output of the timed launches (the last one is still in out)
            torch.cuda.synchronize()
            worst, p999, cnt = edm_rows_error(torch, out, rows, exp)
            res[f"{name}_max_rel_err"] = worst
            res[f"{name}_p999_rel_err"] = p999
            res[f"{name}_err_pairs"] = cnt
        tag = f"edm_{name}_n{n}_d{d}_lambda_t128_f{best['flags']}"
        res[f"{name}_mfma_busy"] = profile_value(tag, "mfma_busy", digest)
        hb = profile_value(tag, "hbm_bytes_per_launch", digest)
        res[f"{name}_hbm_bytes_per_launch"] = hb
        res[f"{name}_traffic_over_output"] = None if hb is None else round(hb / (4 * pairs), 4)
        del ws
    res["bf16x3_meets_1e-3"] = None if not check else res["bf16x3_max_rel_err"] <= 1e-3
    res["bf16_note"] = ("single BF16 rounds each centred coordinate to 8 significant bits: "
                        "its error is absolute, 2^-8 (|x_i| + |x_j|) per distance, and it is "
                        "not held to the 1e-3 relative target")
    del xd, out
    torch.cuda.empty_cache()
    return {"n": n, "d": d, **res}


def bench_edm4(tm, torch, timer, n=32768):
    """Four-feature distances (the global-memory distance test of Section
    4.1) written to the n x n lower triangle: every map at tiles 16, 32, 64,
    128 (lambda also with the pairs order and the XCD swizzle; UTM has no
    tile), with the improvement factor I = t_BB / t_map at each tile.  HBM-bound: 4 B written per cell; the points (16 B each) stay in
    cache."""
    from paper_1609_01490_amd import inputs
    P = torch.from_numpy(inputs.points4(n)).cuda()
    c = torch.empty((n, n), dtype=torch.float32, device="cuda")
    E = n * (n + 1) // 2
    ms = {}
    for t_ in (16, 32, 64, 128):
        for map_name, fl in (("bb", 0), ("rb", 0), ("rec", 0), ("lambda", 0), ("utm", 0),
                             ("lambda", tm.FLAG_ORDER_PAIRS), ("lambda", tm.FLAG_XCD_SWIZZLE)):
            if map_name == "utm" and t_ != 16:
                continue
            p = tm.Plan(n, t_, map_name, flags=fl)
            key = "utm" if map_name == "utm" else f"{map_name}/t{t_}" + (f"/f{fl}" if fl else "")
            ms[key] = round(timer.run(lambda: p.elementwise(tm.OP_EDM4_F32, P, None, c, ld=n),
                                      5, 2), 4)
    del P, c
    torch.cuda.empty_cache()
    best = min(ms, key=ms.get)
    I = {k: round(ms[f"bb/t{k.split('/t')[1].split('/')[0]}"] / v, 4)
         for k, v in ms.items() if "/t" in k}
    I["utm"] = round(min(v for k, v in ms.items() if k.startswith("bb/")) / ms["utm"], 4)
    return {"n": n, "cells": E, "ms_by_map_tile": ms, "best": best,
            "best_GBps_written": round(4 * E / (ms[best] * 1e-3) / 1e9, 1),
            "I_vs_bb_same_tile": I}


# vector ALU issue rate: 256 CUs x 128 FP32 lanes per clock x 2.4 GHz (the
# published 157.3 TFLOP/s FP32 vector peak counts a fused multiply-add as 2)
VALU_LANE_OPS = 256 * 128 * 2.4e9


def bench_map_study(tm, torch, timer, sizes=(4096, 32768), tile=16):
    """The square-root study of Section 4.1 on the dummy kernel (the map, the
    per-cell test, no stores): BB, RB, REC, UTM and lambda with each square
    root (FP32 root / x rsq / bit-trick + 3 Newton steps / FP64, all with the
    integer correction, and the paper's +1e-4 forms without it), as
    I = t_BB / t_map."""
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    variants = {"X": 0, "R": tm.FLAG_SQRT_RSQ, "N": tm.FLAG_SQRT_NEWTON, "F64": tm.FLAG_SQRT_F64,
                "X_eps": tm.FLAG_SQRT_EPS, "R_eps": tm.FLAG_SQRT_EPS | tm.FLAG_SQRT_RSQ,
                "N_eps": tm.FLAG_SQRT_EPS | tm.FLAG_SQRT_NEWTON}
    out = {"tile": tile}
    for n in sizes:
        us = {}
        for name, mp, fl in ([("bb", "bb", 0), ("rb", "rb", 0), ("rec", "rec", 0),
                              ("utm", "utm", 0)] +
                             [(f"lambda_{k}", "lambda", v) for k, v in variants.items()]):
            p = tm.Plan(n, tile, mp, flags=fl)
            us[name] = round(graph_time(torch, timer, lambda: p.dummy(-1, sink), 50) * 1e3, 3)
        out[f"n{n}"] = {"us_per_launch": us,
                        "I_vs_bb": {k: round(us["bb"] / v, 4) for k, v in us.items()}}
    return out


def bench_collide(tm, torch, timer, n=131072):
    """Sphere collision counts (the shared-memory test of Section 5), 1-D
    and 3-D, every map at tiles 16, 32, 64, 128 (UTM: thread space), with the
    improvement factor over BB at the same tile.  Vector-ALU-bound: 11 VALU
    operations per pair test in 3-D, 5 in 1-D, against 256 CUs x 128 FP32
    lanes x 2.4 GHz."""
    from paper_1609_01490_amd import inputs
    pairs = n * (n - 1) // 2
    out = {"n": n, "pairs": pairs}
    counts = torch.empty(n, dtype=torch.int32, device="cuda")
    for dim, ops in ((3, 11), (1, 5)):
        S = torch.from_numpy(inputs.spheres(n, dim)).cuda()
        ms = {}
        for t_ in (16, 32, 64, 128):
            for map_name in ("bb", "rb", "rec", "lambda", "utm"):
                if map_name == "utm" and t_ != 16:
                    continue
                p = tm.Plan(n, t_, map_name, include_diag=False)
                key = "utm" if map_name == "utm" else f"{map_name}/t{t_}"
                ms[key] = round(timer.run(lambda: p.collide(S, counts, dim=dim), 5, 2), 4)
        best = min(ms, key=ms.get)
        rate = pairs / (ms[best] * 1e-3)
        peak = VALU_LANE_OPS / ops
        I = {k: round(ms[f"bb/t{k.split('/t')[1]}"] / v, 4) for k, v in ms.items() if "/t" in k}
        I["utm"] = round(min(v for k, v in ms.items() if k.startswith("bb/")) / ms["utm"], 4)
        out[f"dim{dim}"] = {"ms_by_map_tile": ms, "best": best, "pairs_per_s": round(rate, 1),
                            "alu_bound_pairs_per_s": round(peak, 1),
                            "frac_of_alu_bound": round(rate / peak, 4),
                            "mean_overlaps_per_sphere": round(float(counts.float().mean()), 3),
                            "I_vs_bb_same_tile": I}
        del S
    del counts
    torch.cuda.empty_cache()
    return out


def bench_tetra(tm, torch, timer, n=8192):
    """The tetrahedral extension (Section 6): triangle counts of the
    neighbour graph of n points (a triplet kernel over the strict
    tetrahedron) and the map-only dummy kernel, 3-D lambda (FP32 / FP64 cube
    root) vs the 3-D bounding box, I = t_BB / t_lambda."""
    from paper_1609_01490_amd import inputs
    P, r2 = inputs.points3(n)
    Pd = torch.from_numpy(P).cuda()
    counts = torch.empty(n, dtype=torch.int32, device="cuda")
    total = torch.zeros(1, dtype=torch.int64, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    tri_ms, dummy_us = {}, {}
    for t_ in (8, 16, 32, 64):
        for name, mp, fl in (("bb", "bb", 0), ("lambda", "lambda", 0),
                             ("lambda_f64", "lambda", tm.FLAG_SQRT_F64)):
            p = tm.TetPlan(n, t_, mp, strict=True, flags=fl)
            tri_ms[f"{name}/t{t_}"] = round(
                timer.run(lambda: p.triangles(Pd, float(r2), counts, total), 5, 2), 4)
            if t_ <= 16:
                q = tm.TetPlan(2048, t_, mp, strict=True, flags=fl)
                dummy_us[f"{name}/t{t_}"] = round(
                    graph_time(torch, timer, lambda: q.dummy(-1, sink), 10) * 1e3, 2)
    tri_total = int(total.cpu()[0])
    del Pd, counts, total, sink
    torch.cuda.empty_cache()
    best = min(tri_ms, key=tri_ms.get)
    triples = n * (n - 1) * (n - 2) // 6
    I = {k: round(tri_ms["bb/" + k.split("/")[1]] / v, 4) for k, v in tri_ms.items()}
    Id = {k: round(dummy_us["bb/" + k.split("/")[1]] / v, 4) for k, v in dummy_us.items()}
    return {"n": n, "triples": triples, "triangles": tri_total,
            "triangles_ms_by_map_tile": tri_ms, "best": best,
            "triples_per_s": round(triples / (tri_ms[best] * 1e-3), 1),
            "I_vs_bb_same_tile": I,
            "dummy_n2048_us_by_map_tile": dummy_us, "dummy_I_vs_bb": Id}


def make_batch(tm, torch, steps=20, d=32, tiles=None):
    """The 512-instance batch (see bench_batch), bound to device buffers."""
    from paper_1609_01490_amd import inputs
    spec = inputs.batch_instances()
    kinds, ns, A, B, init = [], [], [], [], []
    pairs = cells = 0
    for k, (kind, n) in enumerate(spec):
        if kind == "edm":
            X, _ = inputs.points(n, d, dup_frac=0.0, seed=inputs.seed_for(4) * 1000 + k)
            A.append(torch.from_numpy(X).cuda())
            B.append(torch.empty((n * (n - 1) // 2,), dtype=torch.float32, device="cuda"))
            kinds.append(tm.KIND_EDM)
            pairs += n * (n - 1) // 2
            init.append(None)
        else:
            ld = (n + 15) // 16 * 16  # 16-byte rows: the bit-sliced body's vector path
            g = inputs.life(n, 0.3, seed=inputs.seed_for(4) * 1000 + k, ld=ld)
            A.append(torch.from_numpy(g).cuda())
            B.append(torch.zeros_like(A[-1]))
            kinds.append(tm.KIND_LIFE)
            cells += n * (n + 1) // 2
            init.append(g)
        ns.append(n)
    ds = [d] * len(ns)
    tune_ms = None
    if tiles is None:
        te, tl, fl, tune_ms = tm.batch_autotune(kinds, ns, ds, steps, A, B, reps=1)
        for a, g in zip(A, init):  # back to generation 0
            if g is not None:
                a.copy_(torch.from_numpy(g))
    else:
        te, tl, fl = tiles
    b = tm.Batch(kinds, ns, ds, edm_tile=te, life_tile=tl, life_steps=steps, flags=fl)
    b.bind(A, B)
    return spec, kinds, A, B, b, te, tl, fl, tune_ms, pairs, cells


def bench_batch(tm, torch, timer, steps=20, d=32, tiles=None):
    """512 uneven instances (n log-uniform in [64, 8192]), even index distance
    map (d = 32), odd index Life (20 generations).  Tiles from the batch
    autotuner (tri_batch_autotune) unless given; then one hipGraph launch of
    the persistent queue vs the same bodies launched per instance."""
    spec, kinds, A, B, b, te, tl, fl, tune_ms, pairs, cells = make_batch(tm, torch, steps, d, tiles)
    # the graph and the stream form timed in turn after warm-up rounds (the
    # first launches on fresh buffers run slower, and so does whichever
    # launch follows the thousands of small per-instance launches, so those
    # are timed apart, afterwards)
    g_ms, s_ms = timer.interleaved([lambda: b.launch(tm.BATCH_GRAPH),
                                    lambda: b.launch(tm.BATCH_STREAM)], reps=7, warmup=3)
    p_ms = timer.median(lambda: b.launch(tm.BATCH_PER_INSTANCE), 5, 1)
    res = {"graph": round(g_ms, 4), "stream": round(s_ms, 4), "per_instance": round(p_ms, 4)}
    info = b.info
    nodes = info["graph_nodes"]
    n_edm = sum(1 for k in kinds if k == tm.KIND_EDM)
    # per-instance mode: one launch per distance map, and per Life instance
    # one launch per graph node (each node advances Life by its share of the
    # generations: `steps` nodes of one generation, or fewer temporally
    # blocked ones)
    launches = n_edm + (len(kinds) - n_edm) * nodes
    work_bytes = 4 * pairs + 2 * cells * steps
    out = {"instances": len(spec), "edm_tile": te, "life_tile": tl, "flags": fl,
           "graph_nodes": nodes, "tiles_from": (
               "tri_batch_autotune" if tiles is None else "given"),
           "life_steps": steps, "d": d, "edm_pairs": pairs, "life_cells": cells,
           "launches_per_instance_mode": launches,
           "ms": res, "timing": "graph and stream: median of 7 rounds in turn after 3 warm-up "
                                "rounds; per-instance launches: median of 5, timed afterwards",
           "speedup_graph_vs_per_instance": round(res["per_instance"] / res["graph"], 3),
           # 4 B per distance plus 2 B per cell and generation: the work as if
           # every generation went through HBM, not a bandwidth (temporal
           # blocking moves a Life cell through HBM once per node)
           "generation_work_GBps_graph": round(work_bytes / (res["graph"] * 1e-3) / 1e9, 1),
           "persistent_workgroups": info["persistent_workgroups"]}
    b.close()
    del A, B
    torch.cuda.empty_cache()
    return out


def profile_target(tm, torch, args):
    """A few launches of one workload, nothing else, for counter runs."""
    from paper_1609_01490_amd import inputs
    t = args.profile_target
    reps = max(1, args.steps)
    if t == "copy":
        # plain device copy of known size: 1 GiB read + 1 GiB written per launch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(reps):
            b.copy_(a)
    elif t == "elementwise":
        n = 32768
        a, X, Y, _ = inputs.f32_elementwise(n, with_fill=False)
        xd, yd = torch.from_numpy(X).cuda(), torch.from_numpy(Y).cuda()
        c = torch.empty((n, n), dtype=torch.float32, device="cuda")
        p = tm.Plan(n, args.tile or 64, args.map, flags=args.flags)
        for _ in range(reps):
            p.elementwise(tm.OP_AXPYT_F32, xd, yd, c, ld=n, a=float(a))
    elif t in ("edm", "edm_bf16"):
        # BF16X3 (edm) or single BF16 (edm_bf16) on the matrix cores
        mode = tm.EDM_BF16X3 if t == "edm" else tm.EDM_BF16
        n, d = 65536, 128
        X, _ = inputs.points(n, d)
        xd = torch.from_numpy(X).cuda()
        out = torch.empty((n * (n - 1) // 2,), dtype=torch.float32, device="cuda")
        q = tm.Plan(n, 128, "lambda", include_diag=False,
                    flags=args.flags or tm.FLAG_XCD_SWIZZLE)
        ws = torch.empty(q.edm_workspace_size(d, mode), dtype=torch.uint8, device="cuda")
        for _ in range(reps):
            q.edm(xd, out, mode=mode, fixup_thr=1e-2, ws=ws)
    elif t == "edm_fp32":
        n, d = 65536, 128
        X, _ = inputs.points(n, d)
        xd = torch.from_numpy(X).cuda()
        out = torch.empty((n * (n - 1) // 2,), dtype=torch.float32, device="cuda")
        q = tm.Plan(n, args.tile or 128, "lambda", include_diag=False, flags=args.flags)
        for _ in range(reps):
            q.edm(xd, out, mode=tm.EDM_FP32)
    elif t == "life":
        n = 16384
        cur = torch.from_numpy(inputs.life(n, 0.3)).cuda()
        nxt = torch.zeros_like(cur)
        p = tm.Plan(n, args.tile or 64, args.map, flags=args.flags)
        p.stencil(cur, nxt, reps)
    elif t == "batch":
        tiles = (args.tile, args.tile, args.flags) if args.tile else None
        spec, kinds, A, B, b, *_ = make_batch(tm, torch, tiles=tiles)
        torch.cuda.synchronize()
        for _ in range(reps):
            b.launch(tm.BATCH_GRAPH)
        torch.cuda.synchronize()
        b.close()
    elif t == "int":
        n = 2048
        A, B, C0 = inputs.int_elementwise(n)
        ad, bd, cd = (torch.from_numpy(v).cuda() for v in (A, B, C0))
        for map_name in ("lambda", "bb"):
            p = tm.Plan(n, 16, map_name)
            for _ in range(reps):
                p.elementwise(tm.OP_XORMUL_I32, ad, bd, cd, ld=n)
    torch.cuda.synchronize()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--tile", type=int, default=0, help="0: the autotuner's choice")
    ap.add_argument("--map", default="lambda")
    ap.add_argument("--flags", type=int, default=0)
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-target", choices=["elementwise", "edm", "edm_bf16", "edm_fp32", "life",
                                                 "int", "copy", "batch"],
                    help="only launch this workload's kernels a few times (for rocprofv3 runs); "
                         "prints no JSON line")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_1609_01490_amd import trimap as tm
    timer = Timer(torch)
    if args.profile_target:
        profile_target(tm, torch, args)
        return

    n, E, res, cpu, table = bench_elementwise(tm, torch, args, timer)
    ms, tile, flags = res[args.map]
    bytes_per_launch = 12 * E
    achieved = bytes_per_launch / (ms * 1e-3) / 1e9
    digest = src_digest("elementwise.hip", "maps.hpp")
    traffic = traffic_from_profiles(f"axpyt_f32_n{n}_{args.map}_t{tile}_f{flags}", digest)

    extra = {"stream_add_ceiling_GBps": round(res["stream_add_GBps"], 1),
             "frac_of_stream_add": round(achieved / res["stream_add_GBps"], 4),
             "probes": res.get("probes"),
             "frac_of_best_2r1w_probe": (round(achieved / res["probes"]["add_2r1w"]["best_GBps"], 4)
                                         if res.get("probes") else None),
             "I_lambda_vs_bb_elementwise": round(res["bb"][0] / ms, 4),
             "bb_ms": round(res["bb"][0], 4), "bb_tile": res["bb"][1], "src_digest": digest,
             "elementwise_ms_by_map_tile": {f"{c['map']}/t{c['tile']}/f{c['flags']}":
                                            round(c["ms"], 4) for c in table},
             "named_tiles": named_tiles(table, E, achieved)}
    if not args.no_extra:
        for name, fn in (("int32_n2048", lambda: bench_int_elementwise(tm, torch, timer)),
                         ("life_n16384", lambda: bench_life(tm, torch, timer)),
                         ("edm_n65536_d128", lambda: bench_edm(tm, torch, timer)),
                         ("edm4_n32768", lambda: bench_edm4(tm, torch, timer)),
                         ("collide_n131072", lambda: bench_collide(tm, torch, timer)),
                         ("map_study_dummy", lambda: bench_map_study(tm, torch, timer)),
                         ("tetra_n8192", lambda: bench_tetra(tm, torch, timer)),
                         ("batch_512", lambda: bench_batch(tm, torch, timer))):
            log("extra", name)
            try:
                extra[name] = fn()
            except Exception as e:  # keep the main line even if an extra fails
                extra[name] = {"error": str(e)}

    line = {
        "metric": "elements/s + HBM GB/s %peak, λ(ω) vs bounding-box; "
                  "EDM pairs/s BF16 vs FP32",
        "value": E / (ms * 1e-3),
        "unit": "elements/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"triangular elementwise C=a*X+Y^T, n={n} fp32 full storage, "
                               f"lower triangle incl. diagonal ({E} cells), map {args.map}, "
                               f"tile {tile}x{tile} (autotuned), flags {flags}",
                   "n": n, "tile": tile, "map": args.map, "flags": flags},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic},
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
