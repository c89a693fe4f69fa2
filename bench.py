"""Throughput benchmark of the hash table's hot path on one MI355X.

One step = one pass over the presized 16-byte-cell workload at the paper's
headline size (Sec. 8.4: 10^8 operations): clear a 2^28-cell table, insert
10^8 distinct uniform u64 keys (value = index), find 10^8 present keys, find
10^8 absent keys, then clear a second 2^28-cell table and insert-or-increment
10^8 Zipf(s = 1.0) keys over a universe of 10^8.  The value printed is
4 * 10^8 operations divided by the step time, in Mops/s.  Inputs are
generated on the host before timing and are resident in HBM when the timed
region starts.

    python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

N_OPS = 10 ** 8
LOG2C = 28
ZIPF_S = 1.0
ZIPF_N = 10 ** 8
HBM_PEAK_GBS = 8000.0
LINE = 128
CELLS_PER_LINE = 8  # 16-byte cells


TUNING = None  # the autotuner's launch shape, applied to every measured table


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def new_table(**kw):
    from paper_1601_04017_amd import lpht
    t = lpht.Table(**kw)
    if TUNING is not None:
        t.apply_tuning(TUNING)
    return t


def knuth(alpha):
    ls = 0.5 * (1 + 1 / (1 - alpha))
    lu = 0.5 * (1 + 1 / (1 - alpha) ** 2)
    return ls, lu


def lines_per_op(alpha):
    """Expected 128-byte lines a probe run touches at fill alpha (successful,
    unsuccessful): a run of L cells starting at a uniformly random cell
    touches 1 + (L-1)/8 lines."""
    ls, lu = knuth(alpha)
    return 1 + (ls - 1) / CELLS_PER_LINE, 1 + (lu - 1) / CELLS_PER_LINE


def algorithmic_bytes_per_op(alpha):
    """Bytes the method must move per operation at fill alpha, counting the
    random table accesses in whole 128-byte lines.  The timed calls write
    found flags for finds and no flags for inserts."""
    lines_s, lines_u = lines_per_op(alpha)
    return {
        # key in + value out + found flag out
        "find_hit": lines_s * LINE + 17,
        "find_miss": lines_u * LINE + 17,
        # average insertion cost over the fill from 0 to alpha equals the
        # successful-search cost; the line is read and written back; key and
        # value in
        "insert": 2 * lines_s * LINE + 16,
    }


OP_CODE = {"insert": 1, "find_hit": 0, "find_miss": 0}


def phase_widths(tun, op, used0, n, c):
    """The group width of each launch of a call, as the library picks them:
    by the fill quarter (0, c/4], ..., (3c/4, c] of the bound on `used` after
    the launch; inserting calls split where a quarter boundary changes it."""
    key = "g_modify" if op == "insert" else "g_find"

    def pick(used):
        q = 0 if used == 0 else min(3, (min(used, c) - 1) * 4 // c)
        return tun[key][q] or tun["group_width"]

    if op != "insert":
        return [pick(used0)]
    widths, done = [], 0
    while done < n:
        ln = n - done
        if any(tun[key]):
            for q in (1, 2, 3):
                b = q * c // 4
                if (used0 + done < b < used0 + done + ln and b - (used0 + done) >= 1 << 16
                        and used0 + done + ln - b >= 1 << 16 and pick(b) != pick(b + 1)):
                    ln = b - (used0 + done)
        widths.append(pick(used0 + done + ln))
        done += ln
    return widths


def measured_traffic(phase, widths):
    """HBM bytes of the phase's launches (one per width) from the committed
    rocprofv3 counter summary (FETCH_SIZE + WRITE_SIZE, calibrated), or None
    when the summary is missing or was taken with a different kernel source."""
    from paper_1601_04017_amd import profsum

    path = os.path.join(ROOT, "profiles", "k_bulk_kv64_headline_step.traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha") != profsum.kernel_source_sha():
        return None
    total = 0
    for g in widths:
        k = rec.get("per_kernel", {}).get(f"k_bulk<1, {OP_CODE[phase]}, 0, {g}>")
        if k is None:
            return None
        total += k["read_bytes"] + k["write_bytes"]
    return round(total)


def _host_cpu():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return model, os.cpu_count(), len(os.sched_getaffinity(0))


def cpu_baseline(keys, miss, zipf):
    """The oracle (plain sequential C, -O3), one thread pinned to one core, on
    a bounded sample of the same workload: the first n keys of each stream
    into 2^25-cell tables (the fill of 10^8 keys in 2^28 cells), each phase
    timed on its own.  Inputs are prepared before any timing."""
    import oracle
    from paper_1601_04017_amd import inputs

    log2c = 25
    n = int(N_OPS * (1 << log2c) / (1 << LOG2C))
    ins_k = np.ascontiguousarray(keys[:n])
    ins_v = np.arange(n, dtype=np.uint64)
    hit_k = ins_k[inputs.permutation(n, 203)]  # the inserted keys, shuffled
    miss_k = np.ascontiguousarray(miss[:n])
    zipf_k = np.ascontiguousarray(zipf[:n])
    model, ncpu, nallowed = _host_cpu()
    saved = os.sched_getaffinity(0)
    core = max(saved)
    os.sched_setaffinity(0, {core})
    try:
        o = oracle.OracleTable(oracle.KV64, log2c)
        o2 = oracle.OracleTable(oracle.KV64, log2c)
        ph = {}
        for name, fn in (("insert", lambda: o.insert(ins_k, ins_v)),
                         ("find_hit", lambda: o.find(hit_k)),
                         ("find_miss", lambda: o.find(miss_k)),
                         ("upsert_zipf", lambda: o2.insert_or_update(zipf_k, None, oracle.ADD))):
            t0 = time.perf_counter()
            fn()
            ph[name] = time.perf_counter() - t0
    finally:
        os.sched_setaffinity(0, saved)
    el = sum(ph.values())
    return {
        "value": round(4 * n / el / 1e6, 3),
        "unit": "Mops/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{n} inserts + {n} hit finds + {n} miss finds + {n} Zipf(1.0) increments, "
                  f"2^{log2c}-cell tables (same fill as the 2^{LOG2C} workload), {el:.1f} s",
        "phase_mops": {k: round(n / v / 1e6, 3) for k, v in ph.items()},
        "phase_s": {k: round(v, 3) for k, v in ph.items()},
        "pinned_core": core,
        "host_cpu": model,
        "host_nproc": ncpu,
        "host_cpus_allowed": nallowed,
        "build": "gcc -O3 -std=c11",
    }


def _timed(fn, stream):
    import torch
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    fn()
    b.record(stream)
    b.synchronize()
    return a.elapsed_time(b)


SUITE_PARTS = ("ceilings", "packed32", "fill_sweep", "growing", "deletion", "bulk", "async", "strings", "zipf",
               "serving")


def run_suite(dev, reps=3, parts=SUITE_PARTS, serving_requests=2000):
    """The other workloads, each timed on the GPU (mean of `reps` after one
    warm-up): packed 2^21 table; the fill sweep of the 2^28 table; growing
    from 4096 cells in batches of 2^20; the deletion test (sliding window of
    10^7 keys) and shrinking migrations; Zipf insert-or-increment presized and
    growing for s in {0.5, 1, 1.25, 1.5}; and the measured memory ceilings."""
    import torch

    from paper_1601_04017_amd import inputs, lpht, roofline

    stream = torch.cuda.current_stream()
    out = {}

    def up(a):
        return torch.from_numpy(np.ascontiguousarray(a).view(np.int64 if a.dtype == np.uint64 else np.int32)).to(dev)

    if "ceilings" in parts:
        log("suite: ceilings")
        out["ceilings"] = roofline.measure()
    if "packed32" in parts:
        out["packed32_2e21"] = _suite_packed32(dev, up, stream, reps)
    need_keys = any(p in parts for p in ("fill_sweep", "growing", "deletion", "bulk", "async"))
    if need_keys:
        nmax = 201_326_592
        keys = inputs.distinct_keys_u64(nmax, 201)
        dkeys = up(keys)
        dvals = torch.arange(nmax, dtype=torch.int64, device=dev)
        del keys
    if "fill_sweep" in parts:
        out["fill_sweep_2e28"] = _suite_fill_sweep(dev, up, stream, reps, dkeys, dvals)
    if "growing" in parts:
        out["growing_from_4096"] = _suite_growing(stream, reps, dkeys, dvals)
    if "deletion" in parts:
        out["deletion_window_1e7"] = _suite_deletion(stream, dkeys, dvals)
        out["shrink_2e26"] = _suite_shrink(stream, dkeys, dvals)
    if "bulk" in parts:
        out["bulk_build_merge_2e28"] = _suite_bulk(up, stream, reps, dkeys, dvals)
    if "async" in parts:
        out["async_growth_one_call"] = _suite_async(up, reps, dkeys, dvals)
    if need_keys:
        del dkeys, dvals
    if "strings" in parts:
        out["string_keys"] = _suite_strings(stream, reps)
    if "zipf" in parts:
        out["zipf_increment"] = _suite_zipf(up, stream, reps)
    if "serving" in parts:
        out["serving"] = run_serving(nreq=serving_requests)
    return out


def serving_trace(nreq, seed=500, median=16384, lo=1024, hi=1 << 20):
    """64 tables of 2^12..2^26 cells, lognormal requests (median 16384,
    sigma 1.35, clipped to [1024, 2^20]), find / insert-or-increment / erase
    = 60/30/10 %, keys Zipf(1.0) over 10^8 (see inputs.serving_trace)."""
    from paper_1601_04017_amd import inputs

    return inputs.serving_trace(nreq, seed=seed, median=median, lo=lo, hi=hi, universe=ZIPF_N)


def _serve(caps, reqs, total, mode, slots, streams, budget, nclients, keep_results=False):
    from paper_1601_04017_amd import lpht

    srv = lpht.Server(caps, mode=mode, max_inflight=slots, streams=streams, hbm_budget=budget)
    arr, outs, keep = srv.make_requests(reqs)
    done, wall_us = srv.run_closed_loop(arr, nclients)
    lat = np.array([d.done_us - d.submit_us for d in done])
    ok = sum(1 for d in done if d.status == 0)
    st = srv.stats()
    results = [(o[0].numpy().copy(), o[1].numpy().copy()) for o in outs] if keep_results else None
    srv.close()
    del arr, outs, keep
    out = {"mops": round(total / wall_us, 1), "wall_ms": round(wall_us / 1e3, 2),
           "p50_ms": round(float(np.percentile(lat, 50)) / 1e3, 3),
           "p99_ms": round(float(np.percentile(lat, 99)) / 1e3, 3),
           "completed_ok": ok, "launch_groups": st["waves"],
           "admission_waits": st["admission_waits"], "hbm_budget": budget,
           "peak_hbm_bytes": st["peak_hbm_bytes"]}
    return (out, results) if keep_results else out


def _first_true(keys, flags):
    """Flags with each key's single true flag moved to its first occurrence
    (which operation of equal keys wins is unspecified)."""
    f = flags.copy()
    t = f == 1
    if not t.any():
        return f
    order = np.argsort(keys, kind="stable")
    ks, ts = keys[order], t[order]
    starts = np.flatnonzero(np.r_[True, ks[1:] != ks[:-1]])
    has = np.add.reduceat(ts.astype(np.int64), starts)
    f[t] = 0
    f[order[starts][has > 0]] = 1
    return f


def serving_leg(nreq=300, nclients=256):
    """Batched serving on the mixed trace, closed loop: the resident kernel and
    continuous-batching waves against one launch per request, under a budget
    of twice the initial tables.  p50 / p99 request latency (submit to
    completion, host clock) and throughput.  The three runs must agree
    request by request (values, and flags up to which of equal keys won)."""
    from paper_1601_04017_amd import lpht

    caps, reqs, total = serving_trace(nreq)
    budget = 2 * sum(16 << c for c in caps)
    res = {"trace": f"{nreq} requests, {total} ops, 64 tables of 2^12..2^26 cells, {nclients} clients, "
                    "lognormal sizes median 16384 in [1024, 2^20], find/increment/erase 60/30/10, Zipf(1.0) "
                    "keys over 1e8",
           "requests": nreq, "ops": total}
    outs = {}
    for name, mode, streams in (("persistent", lpht.SERVE_PERSISTENT, 1), ("waves", lpht.SERVE_WAVES, 4),
                                ("one_launch_per_request", lpht.SERVE_SINGLE, 4)):
        log(f"serving leg: {name}")
        res[name], outs[name] = _serve(caps, reqs, total, mode, 256, streams, budget, nclients,
                                       keep_results=True)
    ref = outs["one_launch_per_request"]
    agree = True
    for name in ("persistent", "waves"):
        for (tab, keys, kinds), (va, fa), (vb, fb) in zip(reqs, outs[name], ref):
            m0 = kinds == 0
            if not (np.array_equal(va, vb) and np.array_equal(fa[m0], fb[m0])):
                agree = False
            for m in (kinds == 1, kinds == 2):
                if not np.array_equal(_first_true(keys[m], fa[m]), _first_true(keys[m], fb[m])):
                    agree = False
    res["modes_agree"] = agree
    return res


def run_serving(nreq=2000, nclients=256):
    """Closed-loop serving of the mixed trace: continuous batching waves, the
    resident kernel, one launch per request, and waves and the resident
    kernel under a tight HBM budget; then the small-request trace."""
    from paper_1601_04017_amd import lpht

    log(f"suite: serving trace ({nreq} requests)")
    caps, reqs, total = serving_trace(nreq)
    init_bytes = sum(16 << c for c in caps)
    res = {"requests": nreq, "ops": total, "clients": nclients, "tables": len(caps),
           "initial_table_bytes": init_bytes}
    runs = [("waves", lpht.SERVE_WAVES, 256, 4, 2 * init_bytes),
            ("persistent", lpht.SERVE_PERSISTENT, 256, 1, 2 * init_bytes),
            ("one_launch_per_request", lpht.SERVE_SINGLE, 256, 4, 2 * init_bytes),
            ("waves_tight_budget", lpht.SERVE_WAVES, 256, 4, int(1.25 * init_bytes)),
            ("persistent_tight_budget", lpht.SERVE_PERSISTENT, 256, 1, int(1.25 * init_bytes))]
    for name, mode, slots, streams, budget in runs:
        log(f"suite: serving {name}")
        res[name] = _serve(caps, reqs, total, mode, slots, streams, budget, nclients)
    nsmall = 2 * nreq
    caps, reqs, total = serving_trace(nsmall, seed=600, median=1024, lo=64, hi=16384)
    small = {"requests": nsmall, "ops": total, "clients": nclients}
    for name, mode, streams in (("waves", lpht.SERVE_WAVES, 4), ("persistent", lpht.SERVE_PERSISTENT, 1),
                                ("one_launch_per_request", lpht.SERVE_SINGLE, 4)):
        log(f"suite: serving small requests {name}")
        small[name] = _serve(caps, reqs, total, mode, 256, streams, 0, nclients)
    res["small_requests"] = small
    return res


def _suite_packed32(dev, up, stream, reps):
    import torch  # noqa: F401

    from paper_1601_04017_amd import inputs, lpht

    # packed 2^21 cells: 2^20 inserts, 2^20 finds (half absent)
    log("suite: packed32 2^21")
    n = 1 << 20
    k = inputs.distinct_keys_u32(n, 101)
    absent = inputs.distinct_keys_u32(n // 2, 101, absent=True)
    present = k[inputs.permutation(n, 102)[: n // 2]]
    fk, _ = inputs.shuffled_mix(present, absent, 103)
    dk, dv, dfk = up(k), up(np.arange(n, dtype=np.uint32)), up(fk)
    t = lpht.Table(layout=lpht.PACKED32, log2_capacity=21)
    if TUNING is not None:
        t.apply_tuning(lpht.autotune(lpht.PACKED32, 21, reps=2)[0])
    res = []
    for r in range(reps + 1):
        t.clear()
        ti = _timed(lambda: t.insert(dk, dv, flags=False), stream)
        tf = _timed(lambda: t.find(dfk), stream)
        if r:
            res.append((ti, tf))
    ti, tf = np.mean(res, axis=0)
    t.close()
    return {"insert_ms": round(ti, 4), "find_ms": round(tf, 4),
            "insert_mops": round(n / ti / 1e3, 1), "find_mops": round(n / tf / 1e3, 1)}


def _suite_fill_sweep(dev, up, stream, reps, dkeys, dvals):
    import torch

    from paper_1601_04017_amd import inputs, lpht

    # fill sweep on 2^28 cells of 16 bytes
    log("suite: fill sweep")
    sweep = {}
    dmiss = up(inputs.distinct_keys_u64(10 ** 8, 201, absent=True))
    t = new_table(layout=lpht.KV64, log2_capacity=28)
    outv = torch.empty(10 ** 8, dtype=torch.int64, device=dev)
    outf = torch.empty(10 ** 8, dtype=torch.uint8, device=dev)
    for nn in (67_108_864, 10 ** 8, 134_217_728, 201_326_592):
        hit = dkeys[torch.randperm(nn, device=dev)[: 10 ** 8] if nn >= 10 ** 8 else
                    torch.randint(0, nn, (10 ** 8,), device=dev)]
        res = []
        for r in range(reps + 1):
            t.clear()
            ti = _timed(lambda: t.insert(dkeys[:nn], dvals[:nn], flags=False), stream)
            th = _timed(lambda: t.find(hit, outv, outf), stream)
            tm = _timed(lambda: t.find(dmiss, outv, outf), stream)
            if r:
                res.append((ti, th, tm))
        ti, th, tm = np.mean(res, axis=0)
        sweep[f"{nn / (1 << 28):.4f}"] = {"n": nn, "insert_ms": round(ti, 3), "find_hit_ms": round(th, 3),
                                           "find_miss_ms": round(tm, 3),
                                           "insert_mops": round(nn / ti / 1e3, 1),
                                           "find_hit_mops": round(1e8 / th / 1e3, 1),
                                           "find_miss_mops": round(1e8 / tm / 1e3, 1)}
        del hit
    t.close()
    return sweep


def _suite_growing(stream, reps, dkeys, dvals):
    import torch

    from paper_1601_04017_amd import lpht

    # growing from 4096 cells, 10^8 keys in batches of 2^20
    log("suite: growing")
    b = 1 << 20
    res = []
    for r in range(reps + 1):
        t = new_table(layout=lpht.KV64, log2_capacity=12, auto_grow=True)
        t.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for lo in range(0, N_OPS, b):
            hi = min(N_OPS, lo + b)
            t.insert(dkeys[lo:hi], dvals[lo:hi], flags=False)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) * 1e3
        st = t.stats()
        if r:
            res.append((el, st["migrate_ms"], st["migrations"], st["resizes"], t.log2_capacity,
                        st["host_syncs"]))
        assert t.count() == (N_OPS, N_OPS)
        t.close()
    el, mig, nmig, nres, lg, syncs = np.mean(res, axis=0)
    return {"total_ms": round(el, 3), "migrate_ms": round(mig, 3),
            "insert_ms_excl_migration": round(el - mig, 3),
            "mops": round(N_OPS / el / 1e3, 1), "data_migrations": int(nmig),
            "resizes": int(nres), "final_log2_capacity": int(lg), "host_syncs": int(syncs)}


WINDOW = 10 ** 7
ALTERNATIONS = 10 ** 8


def _suite_deletion(stream, dkeys, dvals):
    import torch

    from paper_1601_04017_amd import lpht

    # Deletion test: a table created for 1.5e7 elements (2^24 cells, auto
    # growth) prefilled with 10^7 keys, then 10^8 alternations of inserting
    # the next key and erasing the key 10^7 before it, in batches of b
    # inserts followed by the b matching erases; one alternation counts as
    # one operation.  Tombstones are reclaimed by the cleanup migrations.
    out = {}
    for b in (1 << 16, 1 << 20):
        log(f"suite: deletion window, batches of {b}")
        t = new_table(layout=lpht.KV64, log2_capacity=24, auto_grow=True)
        t.set_timing(True)
        for lo in range(0, WINDOW, 1 << 20):
            hi = min(WINDOW, lo + (1 << 20))
            t.insert(dkeys[lo:hi], dvals[lo:hi], flags=False)
        st0 = t.stats()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for lo in range(0, ALTERNATIONS, b):
            hi = min(ALTERNATIONS, lo + b)
            t.insert(dkeys[WINDOW + lo:WINDOW + hi], dvals[WINDOW + lo:WINDOW + hi], flags=False)
            t.erase(dkeys[lo:hi], flags=False)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) * 1e3
        st = t.stats()
        assert t.count()[1] == WINDOW, t.count()
        assert t.status() == 0
        out[str(b)] = {"total_ms": round(el, 3), "mops": round(ALTERNATIONS / el / 1e3, 1),
                       "cleanup_migrations": int(st["resizes"] - st0["resizes"]),
                       "cleanup_ms": round(st["migrate_ms"] - st0["migrate_ms"], 3),
                       "shrinks": int(st["shrinks"]), "final_log2_capacity": int(t.log2_capacity),
                       "host_syncs": int(st["host_syncs"] - st0["host_syncs"])}
        t.close()
    return out


def _suite_shrink(stream, dkeys, dvals):
    import torch

    from paper_1601_04017_amd import lpht

    # Shrinking migrations of a 2^26-cell KV64 table holding 2^22 live keys
    # (and 2^22 tombstones) into 2^25 and 2^23 cells; algorithmic bytes = the
    # old cells read once plus the new cells written once.
    out = {}
    n = 1 << 23
    for log2_new in (25, 23):
        res = []
        for r in range(3):
            t = new_table(layout=lpht.KV64, log2_capacity=26)
            t.insert(dkeys[:n], dvals[:n], flags=False)
            t.erase(dkeys[:n:2].contiguous(), flags=False)
            t.set_timing(True)
            t.grow(log2_new)
            torch.cuda.synchronize()
            st = t.stats()
            assert t.count() == (n // 2, n // 2) and st["shrinks"] == 1
            if r:
                res.append(st["migrate_ms"])
            t.close()
        ms = float(np.mean(res))
        nbytes = (1 << 26) * 16 + (1 << log2_new) * 16
        out[f"to_2e{log2_new}"] = {"ms": round(ms, 4), "algorithmic_gbs": round(nbytes / ms / 1e6, 1)}
    return out


def _suite_bulk(up, stream, reps, dkeys, dvals):
    import torch

    from paper_1601_04017_amd import inputs, lpht

    # Sort-based bulk build / merge into a 2^28-cell KV64 table: 10^8
    # distinct keys (the headline insert's workload), 10^8 Zipf(1.0) keys
    # aggregated with add, and a merge of 10^7 new keys into the 10^8.
    log("suite: bulk build and merge")
    out = {}
    t = new_table(layout=lpht.KV64, log2_capacity=28)
    res = [_timed(lambda: t.build(dkeys[:N_OPS], dvals[:N_OPS]), stream) for _ in range(reps + 1)][1:]
    assert t.count() == (N_OPS, N_OPS)
    out["build_1e8_distinct_ms"] = round(float(np.mean(res)), 3)
    out["build_1e8_distinct_mops"] = round(N_OPS / np.mean(res) / 1e3, 1)
    m = 10 ** 7
    res = []
    for r in range(reps + 1):
        t.build(dkeys[:N_OPS], dvals[:N_OPS])
        torch.cuda.synchronize()
        tm = _timed(lambda: t.merge(dkeys[N_OPS:N_OPS + m], dvals[N_OPS:N_OPS + m]), stream)
        if r:
            res.append(tm)
    assert t.count() == (N_OPS + m, N_OPS + m)
    out["merge_1e7_into_1e8_ms"] = round(float(np.mean(res)), 3)
    z = up(inputs.zipf_keys_u64(N_OPS, ZIPF_N, ZIPF_S, seed=404))
    res = [_timed(lambda: t.build(z, None, op=lpht.ADD), stream) for _ in range(reps + 1)][1:]
    out["build_zipf1_add_1e8_ms"] = round(float(np.mean(res)), 3)
    out["build_zipf1_add_distinct"] = int(t.count()[1])
    t.close()
    del z
    return out


def _suite_async(up, reps, dkeys, dvals):
    import torch

    from paper_1601_04017_amd import inputs, lpht

    # One call of 10^8 operations into a table created with 4096 cells:
    # growth inside the kernel (lpht_insert_async) against growth by the
    # host before the call (pre-growth by the call's length), for distinct
    # keys and for Zipf(1.0) insert-or-increment.
    log("suite: async growth")
    z = up(inputs.zipf_keys_u64(N_OPS, ZIPF_N, ZIPF_S, seed=404))
    out = {}
    for name, keys, vals, add in (("distinct", dkeys[:N_OPS], dvals[:N_OPS], False), ("zipf1_add", z, None, True)):
        row = {}
        for mode in ("async", "async_presized", "host"):
            res = []
            for r in range(reps + 1):
                t = new_table(layout=lpht.KV64, log2_capacity=28 if mode == "async_presized" else 12,
                              auto_grow=True)
                t.set_timing(True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                if mode.startswith("async"):
                    t.insert_async(keys, vals, add=add, flags=False)
                elif add:
                    t.insert_or_update(keys, None, op=lpht.ADD, flags=False)
                else:
                    t.insert(keys, vals, flags=False)
                torch.cuda.synchronize()
                el = (time.perf_counter() - t0) * 1e3
                st = t.stats()
                if not add:
                    assert t.count() == (N_OPS, N_OPS), t.count()
                if r:
                    res.append((el, t.log2_capacity, st["async_growths"], st["async_fallbacks"]))
                t.close()
            el, lg, ng, nf = np.mean(res, axis=0)
            row[mode] = {"ms": round(el, 3), "final_log2_capacity": int(lg), "in_kernel_growths": int(ng),
                         "fallback_growths": round(float(nf), 2)}
        out[name] = row
    del z
    return out


def _suite_strings(stream, reps):
    import torch

    from paper_1601_04017_amd import lpht

    # String keys: 10^7 distinct keys of 8..40 random bytes into a table of
    # 2^25 cells (alpha = 1/2 leaves it at fill 0.3), then 10^7 successful
    # and 10^7 unsuccessful finds.
    log("suite: string keys")
    n = 10 ** 7
    rng = np.random.default_rng(77)
    lens = rng.integers(8, 41, 2 * n)
    offs = np.zeros(2 * n + 1, dtype=np.int64)
    offs[1:] = np.cumsum(lens)
    raw = rng.integers(0, 256, int(offs[-1]), dtype=np.uint8)
    # make every key distinct: its index in its first 8 bytes
    view = np.arange(2 * n, dtype=np.uint64).view(np.uint8).reshape(-1, 8)
    for b in range(8):
        raw[offs[:-1] + b] = view[:, b]
    dbytes = torch.from_numpy(raw).cuda()
    doffs = torch.from_numpy(offs).cuda()
    L = lpht._str_lib()
    res = []
    for r in range(reps + 1):
        t = lpht.StrTable(log2_capacity=25, pool_bytes=int(offs[n]) + 12 * n + 64)
        flags = torch.zeros(n, dtype=torch.uint8, device="cuda")
        vout = torch.zeros(n, dtype=torch.int64, device="cuda")
        torch.cuda.synchronize()
        ins = _timed(lambda: L.lpht_str_insert(t._h, lpht._ptr(dbytes), lpht._ptr(doffs), n, None,
                                               lpht._ptr(flags), None), stream)
        hit = _timed(lambda: L.lpht_str_find(t._h, lpht._ptr(dbytes), lpht._ptr(doffs), n, lpht._ptr(vout),
                                             lpht._ptr(flags), None), stream)
        miss_offs = doffs[n:]
        miss = _timed(lambda: L.lpht_str_find(t._h, lpht._ptr(dbytes), lpht._ptr(miss_offs), n,
                                              lpht._ptr(vout), lpht._ptr(flags), None), stream)
        assert t.count() == (n, n)
        if r:
            res.append((ins, hit, miss))
        t.close()
    ins, hit, miss = np.mean(res, axis=0)
    return {"keys": n, "mean_key_bytes": round(float(lens[:n].mean()), 1), "insert_ms": round(ins, 3),
            "find_hit_ms": round(hit, 3), "find_miss_ms": round(miss, 3),
            "insert_mops": round(n / ins / 1e3, 1), "find_hit_mops": round(n / hit / 1e3, 1)}


def _suite_zipf(up, stream, reps):
    import torch

    from paper_1601_04017_amd import inputs, lpht

    # Zipf insert-or-increment, presized 2^28 and growing from 4096
    b = 1 << 20
    zres = {}
    for sx in (0.5, 1.0, 1.25, 1.5):
        log(f"suite: zipf s={sx}")
        z = up(inputs.zipf_keys_u64(N_OPS, ZIPF_N, sx, seed=400 + int(sx * 4)))
        t = new_table(layout=lpht.KV64, log2_capacity=28)
        res = []
        for r in range(reps + 1):
            t.clear()
            tp = _timed(lambda: t.insert_or_update(z, None, op=lpht.ADD, flags=False), stream)
            if r:
                res.append(tp)
        distinct = t.count()[1]
        t.close()
        gres = []
        for r in range(2):
            g = new_table(layout=lpht.KV64, log2_capacity=12, auto_grow=True)
            g.set_timing(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for lo in range(0, N_OPS, b):
                g.insert_or_update(z[lo:lo + b], None, op=lpht.ADD, flags=False)
            torch.cuda.synchronize()
            el = (time.perf_counter() - t0) * 1e3
            st = g.stats()
            if r:
                gres.append((el, st["migrate_ms"], g.log2_capacity))
            assert g.count()[1] == distinct
            g.close()
        zres[str(sx)] = {"presized_ms": round(float(np.mean(res)), 3),
                         "presized_mops": round(N_OPS / np.mean(res) / 1e3, 1),
                         "growing_ms": round(gres[0][0], 3), "growing_migrate_ms": round(gres[0][1], 3),
                         "growing_mops": round(N_OPS / gres[0][0] / 1e3, 1),
                         "growing_final_log2_capacity": int(gres[0][2]), "distinct": int(distinct)}
        del z
    return zres


def _stats(xs):
    xs = [float(x) for x in xs]
    return {"mean": round(float(np.mean(xs)), 3), "min": round(min(xs), 3), "max": round(max(xs), 3)}


def control_zipf_scrambled(t2, d_zscr, reps, stream):
    """The Zipf insert-or-increment with the keys renamed by a seeded
    bijection: the same histogram, without the consecutive ranks that the CRC
    pair spreads over distinct cells (the control for that artefact)."""
    from paper_1601_04017_amd import lpht
    ms = []
    for r in range(reps + 1):
        t2.clear()
        x = _timed(lambda: t2.insert_or_update(d_zscr, None, op=lpht.ADD, flags=False), stream)
        if r:
            ms.append(x)
    return ms


def control_growing(d_keys, d_vals, reps):
    """10^8 distinct keys inserted in batches of 2^20 into a table that starts
    at 4096 cells and doubles by block-parallel migration when the fill would
    pass 1/2: total and migration time (HIP events around each migration)."""
    import torch
    from paper_1601_04017_amd import lpht
    b = 1 << 20
    tot, mig = [], []
    for r in range(reps + 1):
        g = new_table(layout=lpht.KV64, log2_capacity=12, auto_grow=True)
        g.set_timing(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for lo in range(0, N_OPS, b):
            g.insert(d_keys[lo:lo + b], d_vals[lo:lo + b], flags=False)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) * 1e3
        st = g.stats()
        assert g.count() == (N_OPS, N_OPS) and g.log2_capacity == 28
        g.close()
        if r:
            tot.append(el)
            mig.append(st["migrate_ms"])
    return tot, mig, st


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the controls, ceilings and the serving leg (profiling runs)")
    ap.add_argument("--group-width", type=int, default=None)
    ap.add_argument("--aggregate", type=int, default=None)
    ap.add_argument("--suite", action="store_true", help="also measure the other workloads")
    ap.add_argument("--parts", default=",".join(SUITE_PARTS), help="suite parts to run")
    ap.add_argument("--suite-only", action="store_true", help="skip the headline step")
    ap.add_argument("--serving-requests", type=int, default=2000,
                    help="requests of the suite's serving trace (fewer under a tracing profiler)")
    ap.add_argument("--no-autotune", action="store_true",
                    help="use the library's default launch shape instead of the autotuner's")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path (tables shard by hash "
              "prefix in the design only); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1601_04017_amd import inputs, lpht, roofline

    lpht.load()
    assert torch.cuda.is_available()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    global TUNING
    tune_info = None
    if not args.no_autotune:
        # launch shape for 16-byte cells, tuned on scratch tables of the
        # headline capacity (2^28 cells, 4 GiB), outside every timed region
        log("autotune")
        t0 = time.perf_counter()
        TUNING, _ = lpht.autotune(lpht.KV64, LOG2C, reps=2)
        tune_info = {"shape": TUNING, "scratch_log2_capacity": LOG2C,
                     "seconds": round(time.perf_counter() - t0, 2)}
    if args.suite_only:
        print(json.dumps({"tuning": tune_info,
                          "suite": run_suite(dev, parts=tuple(args.parts.split(",")),
                                                           serving_requests=args.serving_requests)}), flush=True)
        return

    log("generating inputs")
    keys = inputs.distinct_keys_u64(N_OPS, 201)
    miss = inputs.distinct_keys_u64(N_OPS, 201, absent=True)
    perm = inputs.permutation(N_OPS, 203)
    hit = keys[perm]
    zipf = inputs.zipf_keys_u64(N_OPS, ZIPF_N, ZIPF_S, seed=402)
    zscr = None if args.no_extras else inputs.scramble_keys_u64(zipf, 409)
    log("uploading")

    def up(a):
        return torch.from_numpy(a.view(np.int64)).to(dev)

    d_keys, d_vals = up(keys), torch.arange(N_OPS, dtype=torch.int64, device=dev)
    d_hit, d_miss, d_zipf = up(hit), up(miss), up(zipf)
    d_out = torch.empty(N_OPS, dtype=torch.int64, device=dev)
    d_flags = torch.empty(N_OPS, dtype=torch.uint8, device=dev)
    d_found = torch.empty(N_OPS, dtype=torch.uint8, device=dev)

    t1 = new_table(layout=lpht.KV64, log2_capacity=LOG2C)
    t2 = new_table(layout=lpht.KV64, log2_capacity=LOG2C)
    if args.group_width or args.aggregate is not None:
        tun = t1.get_tuning()
        if args.group_width:
            tun["group_width"] = args.group_width
        if args.aggregate is not None:
            tun["aggregate"] = args.aggregate
        t1.set_tuning(**tun)
        t2.set_tuning(**tun)
    stream = torch.cuda.current_stream()
    phases = ["clear1", "insert", "find_hit", "find_miss", "clear2", "upsert_zipf"]

    def step(ev=None):
        def mark(i):
            if ev is not None:
                ev[i].record(stream)
        mark(0)
        t1.clear()
        mark(1)
        t1.insert(d_keys, d_vals, flags=False)
        mark(2)
        t1.find(d_hit, d_out, d_found)
        mark(3)
        t1.find(d_miss, d_out, d_found)
        mark(4)
        t2.clear()
        mark(5)
        t2.insert_or_update(d_zipf, None, op=lpht.ADD, flags=False)
        mark(6)

    log(f"warmup x{args.warmup}")
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    if args.warmup < 1:
        step()
        torch.cuda.synchronize()
    # correctness spot check of the last warmup pass (on device)
    hv, hf = t1.find(d_hit[:1 << 20])
    assert bool((hf == 1).all()), "present keys not found"
    assert bool((hv == torch.from_numpy(perm[:1 << 20].astype(np.int64)).to(dev)).all()), "values"
    mv, mf = t1.find(d_miss[:1 << 20])
    assert not bool(mf.any()), "absent keys found"
    used, live = t1.count()
    assert used == live == N_OPS, (used, live)
    zipf_distinct = t2.count()[1]

    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(7)] for _ in range(args.steps)]
    log(f"timed x{args.steps}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        step(evs[k])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1000 / args.steps
    ph_all = {p: [evs[k][i].elapsed_time(evs[k][i + 1]) for k in range(args.steps)] for i, p in enumerate(phases)}
    ph_ms = {p: float(np.mean(v)) for p, v in ph_all.items()}
    ops_per_step = 4 * N_OPS
    value = ops_per_step / (wall / args.steps) / 1e6

    alpha = N_OPS / (1 << LOG2C)
    bpo = algorithmic_bytes_per_op(alpha)
    ach = {
        "insert": bpo["insert"] * N_OPS / (ph_ms["insert"] / 1e3) / 1e9,
        "find_hit": bpo["find_hit"] * N_OPS / (ph_ms["find_hit"] / 1e3) / 1e9,
        "find_miss": bpo["find_miss"] * N_OPS / (ph_ms["find_miss"] / 1e3) / 1e9,
    }
    dominant = max(("insert", "find_hit", "find_miss"), key=lambda p: ph_ms[p])
    # the group widths each phase's launches ran with
    tun = t1.get_tuning()
    width = {"insert": phase_widths(tun, "insert", 0, N_OPS, 1 << LOG2C),
             "find_hit": phase_widths(tun, "find", N_OPS, 0, 1 << LOG2C),
             "find_miss": phase_widths(tun, "find", N_OPS, 0, 1 << LOG2C)}
    traffic = measured_traffic(dominant, width[dominant])
    roofline_out = {
        "bound": "hbm",
        "kernel": " + ".join(f"k_bulk<KV64,{dominant},G={g}>" for g in width[dominant]),
        "launches": len(width[dominant]),
        "achieved": round(ach[dominant], 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(ach[dominant] / HBM_PEAK_GBS, 4),
        "traffic": traffic,
        # the phase's launches together (one per group width), timed with
        # HIP events on the stream they run on
        "algorithmic_bytes_per_phase": round(bpo[dominant] * N_OPS),
    }
    if traffic:
        roofline_out["traffic_GBs"] = round(traffic / (ph_ms[dominant] / 1e3) / 1e9, 1)

    out = {
        "metric": "Mops/s insert/find/Zipf-increment at 1e8 ops; % HBM roofline; batch p99",
        "value": round(value, 2),
        "unit": "Mops/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {
            "workload": "presized 2^28 KV64 table: 1e8 uniform inserts, 1e8 hit finds, "
                        "1e8 miss finds; 2^28 table: 1e8 Zipf(1.0) insert-or-increment",
            "capacity": 1 << LOG2C,
            "ops": N_OPS,
            "fill": round(alpha, 4),
            "zipf_s": ZIPF_S,
            "group_width": width,
            "block_threads": tun["block_threads"],
            "aggregate": t2.get_tuning()["aggregate"],
        },
        "tuning": tune_info,
        "phases_ms": {k: round(v, 3) for k, v in ph_ms.items()},
        "phases_ms_min_max": {k: [round(min(v), 3), round(max(v), 3)] for k, v in ph_all.items()},
        "phase_mops": {p: round(N_OPS / (ph_ms[p] / 1e3) / 1e6, 1)
                       for p in ("insert", "find_hit", "find_miss", "upsert_zipf")},
        "phase_gbs_algorithmic": {k: round(v, 1) for k, v in ach.items()},
        "zipf_distinct_keys": int(zipf_distinct),
        "roofline": roofline_out,
    }
    if not args.no_extras:
        # outside the timed steps: controls, measured ceilings, serving
        log("control: scrambled Zipf keys")
        d_zscr = up(zscr)
        zs = control_zipf_scrambled(t2, d_zscr, max(3, min(args.steps, 10)), stream)
        assert t2.count()[1] == zipf_distinct  # a bijection keeps the distinct count
        out["control_zipf_scrambled"] = {
            "ms": _stats(zs), "mops": round(N_OPS / (np.mean(zs) / 1e3) / 1e6, 1),
            "keys": "the Zipf(1.0) keys mapped through a seeded 64-bit Feistel bijection (seed 409)"}
        del d_zscr
        log("control: growing from 4096 cells")
        t1.close()
        t2.close()
        gt, gm, gst = control_growing(d_keys, d_vals, 3)
        out["growing_from_4096"] = {
            "total_ms": _stats(gt), "migrate_ms": _stats(gm),
            "mops": round(N_OPS / (np.mean(gt) / 1e3) / 1e6, 1),
            "data_migrations": int(gst["migrations"]), "final_log2_capacity": LOG2C,
            "batches": -(-N_OPS // (1 << 20))}
        del d_out, d_flags, d_found
        log("ceilings")
        ceil = roofline.measure()
        out["ceilings"] = ceil
        lines_s, lines_u = lines_per_op(alpha)
        r_line = ceil["gather16_Gps"]  # every random access fetches one whole line
        bound_mops = {"insert": min(r_line / (2 * lines_s), ceil["cas_Gps"]) * 1e3,
                      "find_hit": r_line / lines_s * 1e3, "find_miss": r_line / lines_u * 1e3}
        roofline_out["measured_random_access"] = {
            "R_line_G_per_s": r_line, "R_cas_G_per_s": ceil["cas_Gps"],
            "bound_mops": {k: round(v, 1) for k, v in bound_mops.items()},
            "frac": {k: round(out["phase_mops"][k] / v, 4) for k, v in bound_mops.items()}}
        out["serving"] = serving_leg()
    if args.suite:
        del d_keys, d_vals, d_hit, d_miss, d_zipf
        t1.close()
        t2.close()
        out["suite"] = run_suite(dev, parts=tuple(args.parts.split(",")),
                                                           serving_requests=args.serving_requests)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle, 1 thread pinned)")
        out["cpu_baseline"] = cpu_baseline(keys, miss, zipf)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
