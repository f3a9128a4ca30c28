"""Batches and the serving loop (workloads of queries, Problem 2): every
result is bit-identical to the CPU oracle's (and so to the same query
evaluated alone), whatever the lanes, fusion, memory admission, cache and
arrival order; fused chains that overflow fall back to one query at a time."""
import numpy as np
import pytest

from synth import configs, workload
from synth.hin import HIN, Constraint, Query, add_bipartite

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def atp():
    import paper_2201_04058_amd as atp
    atp.lib()
    return atp


@pytest.fixture(scope="module")
def net():
    hin, _ = configs.make_hin("scholarly", 0.01)
    return hin


def host(res):
    rp, col, val = res.to_host()
    return rp, col, val


def same(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def mixed_queries(hin):
    """Session queries (single start entity, fusable) and random walks with
    their own start sets and windows."""
    qs = workload.sessions(hin, 21, 40, ["A", "T"], restart_p=0.1, entities=6,
                           type_predicates={"P": ("year", 2012, 32767)})
    qs += workload.random_walk_batch(hin, 3, 24, lengths=(3, 6), start_sizes=(5, 200))
    rng = np.random.default_rng(0)
    order = rng.permutation(len(qs))
    return [qs[i] for i in order]


def alone_results(atp, hin, qs):
    ctx = atp.Context(device=0)
    ctx.load_hin(hin)
    out = []
    for q in qs:
        r = ctx.eval_query(q)
        out.append(host(r))
        r.free()
    ctx.close()
    return out


@pytest.fixture(scope="module")
def mixed(atp, oracle_mod, net):
    """The mixed queries and their oracle results; each query evaluated alone
    on the GPU equals its oracle result, so every comparison with ``ref``
    below is a comparison with the oracle."""
    qs = mixed_queries(net)
    ref = []
    for q in qs:
        rp, col, val, st = oracle_mod.eval_full(net, q, nthreads=8)
        assert st == oracle_mod.ORC_OK, q.name
        ref.append((rp, col, val.astype(np.int64)))
    for z, got in enumerate(alone_results(atp, net, qs)):
        assert same(got, ref[z]), (z, qs[z].name)
    return qs, ref


@pytest.mark.parametrize("lanes,max_batch,budget", [(1, 1, 0), (1, 16, 0), (4, 16, 0), (4, 64, 1 << 20),
                                                    (3, 4, 0)])
def test_batch_equals_oracle(atp, net, mixed, lanes, max_batch, budget):
    qs, ref = mixed
    ctx = atp.Context(device=0)
    ctx.load_hin(net)
    res = ctx.eval_batch(qs, lanes=lanes, max_batch=max_batch, mem_budget_bytes=budget)
    for z, (r, want) in enumerate(zip(res, ref)):
        assert not isinstance(r, Exception), (z, r)
        assert same(host(r), want), (z, qs[z].name)
        if max_batch > 1 and z < 3:
            assert r.stats()["n_products"] >= 1
        r.free()
    ctx.close()


def test_batch_fuses_and_matches_oracle(atp, oracle_mod, net):
    """Queries that differ only in their start set (overlapping ones too) run
    as one chain; each gets exactly its own rows."""
    rng = np.random.default_rng(5)
    yr = ("year", 2010, 32767)
    qs = []
    for z in range(12):
        ids = np.sort(rng.choice(net.counts["A"], size=int(rng.integers(1, 40)), replace=False)).astype(np.int32)
        if z == 3:
            ids = np.concatenate([qs[0].constraints[0].ids[:5], ids[:3]])
            ids = np.unique(ids).astype(np.int32)
        qs.append(Query("A-P-T-P-A", ["A", "P", "T", "P", "A"],
                        [Constraint(0, "idset", ids=ids), Constraint(1, "range", prop=yr[0], lo=yr[1], hi=yr[2]),
                         Constraint(3, "range", prop=yr[0], lo=yr[1], hi=yr[2])]))
    ctx = atp.Context(device=0)
    ctx.load_hin(net)
    res = ctx.eval_batch(qs, lanes=2, max_batch=16)
    for q, r in zip(qs, res):
        want = oracle_mod.eval_full(net, q)
        got = host(r)
        assert np.array_equal(got[0], want[0]) and np.array_equal(got[1], want[1])
        assert np.array_equal(got[2], want[2].astype(np.int64))
    ctx.close()


def test_empty_and_invalid_members(atp, oracle_mod, net):
    """An empty start set and a malformed query inside a batch."""
    ctx = atp.Context(device=0)
    ctx.load_hin(net)
    good = Query("A-P-A", ["A", "P", "A"], [Constraint(0, "idset", ids=np.array([1, 2, 3], np.int32))])
    empty = Query("A-P-A", ["A", "P", "A"], [Constraint(0, "idset", ids=np.zeros(0, np.int32))])
    bad = Query("A-P-A", ["A", "P", "A"], [Constraint(7, "idset", ids=np.array([1], np.int32))])
    res = ctx.eval_batch([good, empty, bad, good], lanes=2, max_batch=8)
    assert isinstance(res[2], atp.AtpError) and res[2].status == atp.ATP_EINVAL
    rp, col, val = host(res[1])
    assert rp[-1] == 0
    assert same(host(res[0]), host(res[3]))
    alone = ctx.eval_query(good)
    assert same(host(res[0]), host(alone))
    orp, ocol, oval, st = oracle_mod.eval_full(net, good)
    assert st == oracle_mod.ORC_OK and same(host(res[0]), (orp, ocol, oval.astype(np.int64)))
    ctx.close()


def _overflow_net():
    """A: node 0 reaches all 2^16 B nodes, node 1 only B node 0; counts along
    A-B-A-B-A-B-A-B-A from node 0 reach 2^64, from node 1 stay below 2^52."""
    nb = 1 << 16
    pairs = [(0, j) for j in range(nb)] + [(1, 0)]
    src = np.array([p[0] for p in pairs], np.int64)
    dst = np.array([p[1] for p in pairs], np.int64)
    hin = HIN(counts={"A": 2, "B": nb})
    add_bipartite(hin, "A", "B", src, dst)
    return hin


def test_fused_overflow_falls_back_to_each_query(atp, oracle_mod):
    hin = _overflow_net()
    types = ["A", "B"] * 4 + ["A"]
    q0 = Query("hub", types, [Constraint(0, "idset", ids=np.array([0], np.int32))])
    q1 = Query("leaf", types, [Constraint(0, "idset", ids=np.array([1], np.int32))])
    ctx = atp.Context(device=0)
    ctx.load_hin(hin)
    with pytest.raises(atp.AtpError) as e:
        ctx.eval_query(q0)
    assert e.value.status == atp.ATP_EOVERFLOW
    alone = host(ctx.eval_query(q1))
    res = ctx.eval_batch([q0, q1], lanes=1, max_batch=2)
    assert isinstance(res[0], atp.AtpError) and res[0].status == atp.ATP_EOVERFLOW
    assert same(host(res[1]), alone)
    assert oracle_mod.eval_full(hin, q0)[3] == oracle_mod.ORC_OVERFLOW
    orp, ocol, oval, st = oracle_mod.eval_full(hin, q1)
    assert st == oracle_mod.ORC_OK and same(alone, (orp, ocol, oval.astype(np.int64)))
    ctx.close()


@pytest.mark.parametrize("cache", [False, True])
def test_server_results_equal_oracle(atp, net, mixed, cache):
    """Continuous batching: requests submitted while others run are fused and
    overlapped; each completion equals the oracle's result (and the query
    alone)."""
    qs, ref = mixed
    ctx = atp.Context(device=0)
    ctx.load_hin(net)
    if cache:
        ctx.cache_configure(atp.ATP_CACHE_OTREE, 1 << 30)
    ctx.server_start(lanes=4, max_batch=16, mem_budget_bytes=1 << 30)
    for z, q in enumerate(qs):
        ctx.submit(q, tag=z)
    got = {}
    while len(got) < len(qs):
        for cp in ctx.poll(64, wait_ms=2000):
            assert cp["tag"] not in got
            got[cp["tag"]] = cp
    assert ctx.server_pending() == 0
    batches = []
    for z, q in enumerate(qs):
        cp = got[z]
        assert cp["status"] == atp.ATP_OK, (z, cp["status"])
        assert same(host(cp["result"]), ref[z]), (z, q.name)
        assert cp["t_submit"] <= cp["t_start"] <= cp["t_done"]
        batches.append(cp["batch"])
        cp["result"].free()
    assert max(batches) > 1  # queued requests were fused
    ctx.server_stop()
    with pytest.raises(atp.AtpError):
        ctx.server_stop()
    ctx.close()


def test_heavy_products_run_alone_and_equal_oracle(atp, net, mixed, monkeypatch):
    """With every product counted as heavy (a threshold of one product), each
    product's numeric phase holds the device alone across the server's four
    lanes (the others wait at the gate), so the lanes take turns; every
    request still completes with the oracle's result, and so does a batch on
    four lanes afterwards."""
    monkeypatch.setenv("ATP_HEAVY_OPS", "1")
    qs, ref = mixed
    ctx = atp.Context(device=0)
    ctx.load_hin(net)
    ctx.server_start(lanes=4, max_batch=4)
    for z, q in enumerate(qs):
        ctx.submit(q, tag=z)
    got = {}
    while len(got) < len(qs):
        for cp in ctx.poll(64, wait_ms=2000):
            got[cp["tag"]] = cp
    for z in range(len(qs)):
        assert got[z]["status"] == atp.ATP_OK, (z, got[z]["status"])
        assert same(host(got[z]["result"]), ref[z]), (z, qs[z].name)
        got[z]["result"].free()
    ctx.server_stop()
    res = ctx.eval_batch(qs, lanes=4, max_batch=1)
    for z, (r, want) in enumerate(zip(res, ref)):
        assert not isinstance(r, Exception), (z, r)
        assert same(host(r), want), (z, qs[z].name)
        r.free()
    ctx.close()


def test_server_submit_during_run_and_stop_drains(atp, net, mixed):
    qs, ref = mixed
    ctx = atp.Context(device=0)
    ctx.load_hin(net)
    ctx.server_start(lanes=2, max_batch=8)
    with pytest.raises(atp.AtpError) as e:
        ctx.eval_batch(qs[:2])
    assert e.value.status == atp.ATP_ESTATE
    got = {}
    for z, q in enumerate(qs[:20]):
        ctx.submit(q, tag=z)
        for cp in ctx.poll(64):
            got[cp["tag"]] = cp
    while len(got) < 20:
        for cp in ctx.poll(64, wait_ms=2000):
            got[cp["tag"]] = cp
    for z in range(20):
        assert same(host(got[z]["result"]), ref[z])
    for z, q in enumerate(qs[20:30]):
        ctx.submit(q, tag=100 + z)
    ctx.server_stop()  # finishes the queue; unpolled completions are freed
    assert ctx.server_pending() == 0
    ctx.close()


def test_tuning_get_set_and_autotune(atp, net, mixed):
    """Tunables change kernels, never results; the autotuner keeps a setting
    from its grid and refuses to run with a cache configured."""
    qs, ref = mixed
    ctx = atp.Context(device=0)
    ctx.load_hin(net)
    t0 = ctx.tuning()
    assert t0["bucket_pct"] == 400 and t0["part_hash_cap"] == 4096
    for bad in ({"part_target": 0}, {"part_hash_cap": 4097}, {"bucket_pct": -1}, {"split_ops": 10},
                {"bucket_chunk": 8}):
        with pytest.raises(atp.AtpError) as e:
            ctx.set_tuning(**bad)
        assert e.value.status == atp.ATP_EINVAL
    assert ctx.tuning() == t0
    ctx.set_tuning(bucket_pct=0, part_target=64, split_ops=1024, task_ops=1, bucket_chunk=64)
    for q, want in zip(qs[:20], ref[:20]):
        assert same(host(ctx.eval_query(q)), want)
    ctx.set_tuning(**t0)
    got = ctx.autotune(qs[:10], rounds=1)
    assert got["bucket_pct"] in (25, 50, 100, 200, 400, 800)
    assert got["part_target"] in (600, 1200, 2400, 3600)
    assert got["part_hash_cap"] in (1024, 2048, 4096)
    assert got["bucket_chunk"] in (1024, 2048, 4096, 8192)
    assert got["ms_after"] <= got["ms_before"] * 1.0001
    assert {k: ctx.tuning()[k] for k in atp.TUNABLES} == {k: got[k] for k in atp.TUNABLES}
    for q, want in zip(qs, ref):
        assert same(host(ctx.eval_query(q)), want)
    ctx.cache_configure(atp.ATP_CACHE_OTREE, 1 << 30)
    with pytest.raises(atp.AtpError) as e:
        ctx.autotune(qs[:2])
    assert e.value.status == atp.ATP_ESTATE
    ctx.close()


def test_cost_model_calibration_keeps_results(atp, net, mixed):
    """Eq. 2 refit on timed multiplications: non-negative coefficients,
    installed in the planner, results unchanged."""
    qs, ref = mixed
    ctx = atp.Context(device=0)
    ctx.load_hin(net)
    start = ctx.cost_model()
    assert all(v >= 0 for v in start)
    with pytest.raises(atp.AtpError) as e:
        ctx.set_cost_model((-1.0, 1.0, 1.0, 0.0))
    assert e.value.status == atp.ATP_EINVAL
    with pytest.raises(atp.AtpError):
        ctx.set_cost_model((0.0, 0.0, 0.0, 1.0))
    fit = ctx.calibrate_cost_model(qs[:24])
    assert fit["products"] >= 4
    assert all(v >= 0 for v in fit["coeffs"]) and sum(fit["coeffs"][:3]) > 0
    assert ctx.cost_model() == pytest.approx(fit["coeffs"])
    for q, want in zip(qs, ref):
        assert same(host(ctx.eval_query(q)), want)
    ctx.set_cost_model(start)
    assert ctx.cost_model() == pytest.approx(start)
    ctx.close()


def test_fused_members_are_cached_as_whole_queries(atp, oracle_mod, net):
    """With a cache, each fused member's rows are offered as that query's own
    whole result; repeating the batch is answered from the cache."""
    rng = np.random.default_rng(9)
    qs = []
    for z in range(8):
        ids = np.array([int(rng.integers(net.counts["A"]))], np.int32)
        qs.append(Query("A-P-V", ["A", "P", "V"],
                        [Constraint(0, "idset", ids=ids), Constraint(1, "range", prop="year", lo=2010, hi=32767)]))
    ctx = atp.Context(device=0)
    ctx.load_hin(net)
    ctx.cache_configure(atp.ATP_CACHE_OTREE, 1 << 30)
    first = [host(r) for r in ctx.eval_batch(qs, lanes=1, max_batch=8)]
    st1 = ctx.cache_stats()
    assert st1["inserts"] >= len({int(q.constraints[0].ids[0]) for q in qs})
    again = [host(r) for r in ctx.eval_batch(qs, lanes=2, max_batch=8)]
    st2 = ctx.cache_stats()
    assert st2["whole_hits"] - st1["whole_hits"] == len(qs)
    for q, a, b in zip(qs, first, again):
        want = oracle_mod.eval_full(net, q)
        assert same(a, b)
        assert np.array_equal(a[0], want[0]) and np.array_equal(a[1], want[1])
        assert np.array_equal(a[2], want[2].astype(np.int64))
    ctx.close()
