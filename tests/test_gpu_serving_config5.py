"""The serving workload at its stated shape, against the oracle.

64 auto-growing tables of 2^12..2^26 cells (16-byte cells), 300 requests from
256 closed-loop clients to uniformly random tables, lognormal sizes (median
16384 operations) clipped to [1024, 2^20] with three requests of at least
2^19 operations, operations find / insert-or-increment / erase = 60/30/10 %
over keys Zipf(1.0) ranks over 10^8 (plus one).  One 2^26-cell table is first
filled to 200 cells below its growth trigger (2^25 distinct keys far outside
the Zipf range), so its first request grows it to 2^27 cells while the server
runs: growth under serving at the largest size.

Every mode (continuous-batching waves, the resident kernel, one launch per
request with many in flight, and strictly one request at a time) runs the
same trace under the default budget (twice the initial tables) and under a
tight one (the least that admits every request when it is alone in
flight: the other tables at their largest capacity, its own table, the new
table of its growth and its staging, plus 16 MiB), and must give, request by request,
the oracle's values and canonical flags (the oracle replays each table's
requests in submission order, phase by phase: finds, then
insert-or-increments, then erases), and, table by table, the oracle's
occupied cells, each live key in the same run with the same count, the same
capacity and the same exact counts.  Results alone equal results in the mix.
"""
import time

import numpy as np
import pytest

import oracle
from paper_1601_04017_amd import inputs
from tests import helpers as H
from tests.gpu_util import to_dev

pytestmark = pytest.mark.gpu

NREQ = 300
NCLIENTS = 256
PREFILL_GAP = 200
I64_MIN = -(1 << 63)


def _say(msg):
    print(f"[config5] {msg}", flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"


def _canon_dev(cells):
    """Canonical form of a 16-byte-cell table held on the device (int64
    words): the occupancy bitmap, and the live keys in unsigned order with
    the start of the run of non-empty cells holding each and its value.  Two
    tables with equal forms hold the same keys in the same runs with the same
    values; only the order inside a run may differ."""
    import torch
    keys, vals = cells[0::2], cells[1::2]
    c = keys.numel()
    occ = keys != 0
    idx = torch.arange(c, device=cells.device)
    le = torch.cummax(torch.where(occ, torch.full_like(idx, -1), idx), 0).values
    empties = torch.nonzero(~occ).flatten()
    assert empties.numel() > 0
    le = torch.where(le < 0, empties[-1] - c, le)
    rs = (le + 1) % c
    live = occ & (keys != 1)
    k, r, v = keys[live], rs[live], vals[live]
    order = torch.argsort(k ^ I64_MIN)  # unsigned order by flipping the sign bit
    return (occ.cpu().numpy(), k[order].cpu().numpy().view(np.uint64), r[order].cpu().numpy(),
            v[order].cpu().numpy().view(np.uint64))


def _same_canon(a, b, what):
    for x, y, name in zip(a, b, ("occupancy", "keys", "run starts", "values")):
        if not np.array_equal(x, y):
            raise AssertionError(f"{what}: {name} differ")


class _World:
    pass


@pytest.fixture(scope="module")
def world():
    """The trace, the prefill, the oracle's replay and its canonical tables."""
    import torch
    w = _World()
    t0 = time.time()
    w.caps, w.reqs, w.total = inputs.serving_trace(NREQ)
    sizes = np.array([k.size for _, k, _ in w.reqs])
    assert sizes.min() >= 1024 and sizes.max() <= 1 << 20 and (sizes >= 1 << 19).sum() >= 1
    assert min(w.caps) == 12 and max(w.caps) == 26 and len(w.caps) == 64
    tabs = [t for t, _, _ in w.reqs]
    # the first 2^26-cell table with requests, prefilled just below its trigger
    w.big = next(t for t in tabs if w.caps[t] == 26)
    first = next(j for j, t in enumerate(tabs) if t == w.big)
    assert int((w.reqs[first][2] == 1).sum()) > PREFILL_GAP
    w.pk = inputs.distinct_keys_u64((1 << 25) - PREFILL_GAP, 511)
    assert w.pk.min() > 10 ** 8 + 1  # disjoint from the Zipf keys 2..10^8+1
    w.pv = np.arange(w.pk.size, dtype=np.uint64) + 7
    _say(f"trace {w.total} ops, prefill table {w.big}: {time.time() - t0:.1f} s")

    orcs = [oracle.OracleTable(oracle.KV64, c, auto_grow=True) for c in w.caps]
    orcs[w.big].insert(w.pk, w.pv)
    # admission accounting (tables, the new table of a growth, staging); in
    # the concurrent run other tables may be ahead of the sequential replay,
    # so the feasible bound uses each table's largest capacity
    most = [16 << c for c in w.caps]
    alone = []  # per request: its table before it, its growth, its staging
    w.ref = []
    for tab, keys, kinds in w.reqs:
        o = orcs[tab]
        m0, m1, m2 = kinds == 0, kinds == 1, kinds == 2
        vals = np.zeros(keys.size, np.uint64)
        flags = np.zeros(keys.size, np.uint8)
        before = o.capacity
        v, f = o.find(keys[m0])
        vals[m0], flags[m0] = v, f
        flags[m1] = o.insert_or_update(keys[m1], None, oracle.ADD)
        flags[m2] = o.erase(keys[m2])
        staging = 2 * (-(-8 * keys.size // 256) * 256) + 2 * (-(-keys.size // 256) * 256)
        alone.append((tab, 16 * before, 16 * o.capacity if o.capacity != before else 0, staging))
        most[tab] = max(most[tab], 16 * o.capacity)
        w.ref.append((vals, flags))
    assert orcs[w.big].log2c == 27  # it grew under serving
    w.final_log2 = [o.log2c for o in orcs]
    w.counts = [o.counts() for o in orcs]
    w.init_bytes = sum(16 << c for c in w.caps)
    w.budget_default = 2 * w.init_bytes
    # the least budget that admits every request when it is alone in flight,
    # whatever the other tables have grown to by then (at most their largest
    # size), plus 16 MiB
    total_most = sum(most)
    w.budget_tight = max(total_most - most[t] + cur + grow + stg for t, cur, grow, stg in alone) + (16 << 20)
    _say(f"oracle replay done: {time.time() - t0:.1f} s; tight budget {w.budget_tight / 1e9:.2f} GB "
         f"({w.budget_tight / w.init_bytes:.2f}x the initial tables)")
    w.canon = []
    for i, o in enumerate(orcs):
        w.canon.append(_canon_dev(to_dev(o.cells())))
    del orcs
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    _say(f"oracle canonical tables: {time.time() - t0:.1f} s")
    return w


def test_canonical_form_agrees_with_host_helper():
    # the device canonicaliser against the plain numpy helper, on a table
    # with a wrapping run, tombstones and erased values
    o = oracle.OracleTable(oracle.KV64, 12)
    keys = inputs.distinct_keys_u64(2500, 3)
    o.insert(keys, keys + np.uint64(1))
    o.erase(keys[::7])
    cells = o.cells()
    occ, k, r, v = _canon_dev(to_dev(cells))
    hk, hr, hv = H.key_run_starts(cells, oracle.KV64)
    assert np.array_equal(occ, H.occupancy(cells, oracle.KV64))
    assert np.array_equal(k, hk) and np.array_equal(r, hr) and np.array_equal(v, hv)


def _serve(w, mode, slots, clients, budget, streams):
    import torch
    from paper_1601_04017_amd import lpht
    srv = lpht.Server(w.caps, mode=mode, max_inflight=slots, streams=streams, hbm_budget=budget)
    pre = srv.table(w.big)
    pre.insert(to_dev(w.pk), to_dev(w.pv), flags=False)
    torch.cuda.synchronize()
    arr, outs, keep = srv.make_requests(w.reqs)
    t0 = time.time()
    done, wall = srv.run_closed_loop(arr, clients)
    _say(f"served in {time.time() - t0:.2f} s ({w.total / wall:.0f} Mops/s)")
    status = [d.status for d in done]
    res = [(o[0].numpy().view(np.uint64).copy(), o[1].numpy().copy()) for o in outs]
    tables = []
    for i in range(len(w.caps)):
        t = srv.table(i)
        tables.append((t.capacity, t.count(), _canon_dev(t.export_cells())))
    stats = srv.stats()
    srv.close()
    del arr, outs, keep
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return status, res, tables, stats


def _check(w, status, res, tables, what):
    assert all(s == 0 for s in status), what
    for j, ((tab, keys, kinds), (gv, gf), (ov, of)) in enumerate(zip(w.reqs, res, w.ref)):
        m0 = kinds == 0
        assert np.array_equal(gv, ov), f"{what}: request {j} values"
        assert np.array_equal(gf[m0], of[m0]), f"{what}: request {j} find flags"
        for m in (kinds == 1, kinds == 2):
            assert np.array_equal(H.canonical_flags(keys[m], gf[m]), of[m]), f"{what}: request {j} flags"
    for i, (cap, cnt, canon) in enumerate(tables):
        assert cap == 1 << w.final_log2[i], f"{what}: table {i} capacity"
        assert cnt == w.counts[i], f"{what}: table {i} counts"
        _same_canon(canon, w.canon[i], f"{what}: table {i}")


MODES = [("waves", "SERVE_WAVES", NREQ, NCLIENTS, 4),
         ("persistent", "SERVE_PERSISTENT", NREQ, NCLIENTS, 1),
         ("one_launch_per_request", "SERVE_SINGLE", NREQ, NCLIENTS, 4)]


@pytest.mark.parametrize("budget", ["default", "tight"])
@pytest.mark.parametrize("name,mode,slots,clients,streams", MODES, ids=[m[0] for m in MODES])
def test_config5_trace_matches_oracle(world, name, mode, slots, clients, streams, budget):
    from paper_1601_04017_amd import lpht
    b = world.budget_default if budget == "default" else world.budget_tight
    _say(f"{name}, {budget} budget {b / 1e9:.2f} GB")
    status, res, tables, stats = _serve(world, getattr(lpht, mode), slots, clients, b, streams)
    _check(world, status, res, tables, f"{name}/{budget}")
    assert stats["completed"] == NREQ
    assert stats["peak_hbm_bytes"] <= b
    if budget == "tight":
        assert stats["admission_waits"] > 0, stats
    if name != "one_launch_per_request":
        assert stats["waves"] < NREQ  # requests shared launches


def test_config5_alone_equals_mix(world):
    # strictly one request at a time, and the full mix; the oracle checks each
    # on its own above, this compares the two runs directly
    from paper_1601_04017_amd import lpht
    _say("alone")
    sa, ra, ta, st_a = _serve(world, lpht.SERVE_SINGLE, 1, 1, world.budget_default, 1)
    assert st_a["waves"] == NREQ
    _say("mix")
    sm, rm, tm, st_m = _serve(world, lpht.SERVE_WAVES, NREQ, NCLIENTS, world.budget_default, 4)
    assert all(s == 0 for s in sa) and all(s == 0 for s in sm)
    for j, ((tab, keys, kinds), (va, fa), (vm, fm)) in enumerate(zip(world.reqs, ra, rm)):
        assert np.array_equal(va, vm), f"request {j} values"
        assert np.array_equal(fa[kinds == 0], fm[kinds == 0]), f"request {j} find flags"
        for m in (kinds == 1, kinds == 2):
            assert np.array_equal(H.canonical_flags(keys[m], fa[m]), H.canonical_flags(keys[m], fm[m]))
    for i, ((ca, na, xa), (cm, nm, xm)) in enumerate(zip(ta, tm)):
        assert ca == cm and na == nm, f"table {i}"
        _same_canon(xa, xm, f"table {i}")
