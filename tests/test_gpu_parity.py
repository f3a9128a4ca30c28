"""GPU parity: every result of the HIP library (through the C-ABI) must equal
the CPU oracle's canonical CSR byte for byte (int64 row pointers, int32
columns, int64 counts).  Integer work: the bar is bit-exactness."""
import itertools

import numpy as np
import pytest

from synth import configs
from synth import tiny as tinygen
from synth.hin import HIN, Constraint, Query, Relation
from tests._nets import _csr_rel, _narrow_and_wide

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def atp():
    import paper_2201_04058_amd as atp
    atp.lib()
    return atp


def make_ctx(atp, hin, **kw):
    ctx = atp.Context(device=0, **kw)
    ctx.load_hin(hin)
    return ctx


def assert_same(res, ref, what=""):
    rp, col, val = res.to_host()
    orp, ocol, oval, st = ref
    assert st == 0, what
    assert np.array_equal(rp, orp), f"row_ptr differs {what}"
    assert np.array_equal(col, ocol), f"col differs {what}"
    assert np.array_equal(val, oval.astype(np.int64)), f"val differs {what}"


def all_plans(i, j):
    if i == j:
        yield str(i)
        return
    for k in range(i, j):
        for a in all_plans(i, k):
            for b in all_plans(k + 1, j):
                yield f"({a},{b})"


# ---------------------------------------------------------------------------

def test_tiny_config_every_plan(atp, oracle_mod, tiny_cfg):
    hin, qs = tiny_cfg
    q = qs[0]
    ref = oracle_mod.eval_full(hin, q)
    ctx = make_ctx(atp, hin)
    res = ctx.eval_query(q)
    assert_same(res, ref, "planner")
    for plan in all_plans(0, len(q.types) - 2):
        assert_same(ctx.eval_query(q, plan=plan), ref, plan)
    ctx.close()


@pytest.mark.parametrize("block", range(8))
def test_random_tiny_networks(atp, oracle_mod, block):
    """Random schemas (self-relations, empty relations, degenerate masks)."""
    for seed in range(block * 40, block * 40 + 40):
        hin = tinygen.random_hin(seed, max_nodes=20)
        rng = np.random.default_rng(50_000 + seed)
        ctx = make_ctx(atp, hin)
        for _ in range(3):
            q = tinygen.random_query(hin, rng, max_len=6)
            if q is None:
                continue
            ref = oracle_mod.eval_full(hin, q)
            assert_same(ctx.eval_query(q), ref, f"seed {seed} {q.name}")
            plans = list(all_plans(0, len(q.types) - 2))
            assert_same(ctx.eval_query(q, plan=plans[-1]), ref, f"seed {seed} {q.name} {plans[-1]}")
        ctx.close()


@pytest.mark.parametrize("no_restrict", [False, True])
@pytest.mark.parametrize("name,scale", [("scholarly", 0.002), ("scholarly", 0.02), ("news", 0.005),
                                        ("news", 0.03)])
def test_scaled_configs_every_plan(atp, oracle_mod, name, scale, no_restrict):
    hin, rng = configs.make_hin(name, scale)
    qs = configs.make_queries(name, hin, rng)
    ctx = make_ctx(atp, hin, no_restrict=no_restrict)
    for q in qs:
        ref = oracle_mod.eval_full(hin, q, nthreads=8)
        assert_same(ctx.eval_query(q), ref, q.name)
        plans = list(all_plans(0, len(q.types) - 2))
        if len(plans) > 8:
            plans = plans[::len(plans) // 8]
        for plan in plans:
            assert_same(ctx.eval_query(q, plan=plan), ref, f"{q.name} {plan}")
    ctx.close()


# ---------------------------------------------------------------------------
# edge cases

def _bip(hin, a, b, pairs):
    na, nb = hin.counts[a], hin.counts[b]
    m = np.zeros((na, nb), bool)
    for i, j in pairs:
        m[i, j] = True
    rp = np.zeros(na + 1, np.int64)
    np.cumsum(m.sum(1), out=rp[1:])
    hin.relations[(a, b)] = Relation(a, b, rp, np.nonzero(m)[1].astype(np.int32))
    t = m.T
    rp2 = np.zeros(nb + 1, np.int64)
    np.cumsum(t.sum(1), out=rp2[1:])
    hin.relations[(b, a)] = Relation(b, a, rp2, np.nonzero(t)[1].astype(np.int32))


@pytest.mark.parametrize("n_out", [1, 31, 32, 33, 63, 64, 65, 127, 128, 129, 255, 256, 257, 511, 512, 513,
                                   1023, 1024, 1025, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192, 8193,
                                   20000])
@pytest.mark.parametrize("ncols", [8191, 8192, 8193, 40000])
def test_row_size_at_every_bin_threshold(atp, oracle_mod, n_out, ncols):
    """Rows whose upper bound sits exactly at each hash-table / tile limit."""
    if n_out > ncols:
        pytest.skip("more outputs than columns")
    rng = np.random.default_rng(n_out * 7 + ncols)
    hin = HIN(counts={"A": 3, "B": 4, "C": ncols})
    _csr_rel(hin, "A", "B", [[0, 1], [2], [0, 1, 2, 3]])
    cols = np.sort(rng.choice(ncols, size=n_out, replace=False))
    half = n_out // 2
    # B0 and B1 overlap on half the columns, B2 hits the last column and column 0, B3 empty
    rows = [cols[: max(1, half + 1)], cols[half:], np.array(sorted({0, ncols - 1})), np.array([], np.int64)]
    _csr_rel(hin, "B", "C", [np.asarray(r, np.int64) for r in rows])
    q = Query("A-B-C", ["A", "B", "C"], [])
    ref = oracle_mod.eval_full(hin, q)
    ctx = make_ctx(atp, hin)
    assert_same(ctx.eval_query(q), ref)
    ctx.close()


@pytest.mark.parametrize("ncols", [100_000, 8193, 1 << 24])
def test_hub_rows_bucketed_by_tile(atp, oracle_mod, ncols):
    """A left-operand row with 20k entries, each expanding to 1-3 products over
    many column tiles (the tile-bucket path), pattern-only and valued."""
    rng = np.random.default_rng(ncols)
    nb = 20_000
    hin = HIN(counts={"Z": 2, "A": 3, "B": nb, "C": ncols})
    _csr_rel(hin, "Z", "A", [[0, 1, 2], [1]])
    _csr_rel(hin, "A", "B", [list(range(nb)), list(range(0, nb, 7)), [3]])
    rows = []
    for b in range(nb):
        k = int(rng.integers(1, 4))
        rows.append(np.sort(rng.choice(ncols, size=k, replace=False)))
    _csr_rel(hin, "B", "C", rows)
    ctx = make_ctx(atp, hin)
    for q, plans in [(Query("A-B-C", ["A", "B", "C"], []), [None]),
                     (Query("Z-A-B-C", ["Z", "A", "B", "C"], []), [None, "((0,1),2)", "(0,(1,2))"]),
                     (Query("A-B-C", ["A", "B", "C"], [Constraint(1, "idset", ids=np.arange(0, nb, 3, dtype=np.int32))]),
                      [None])]:
        ref = oracle_mod.eval_full(hin, q)
        for plan in plans:
            assert_same(ctx.eval_query(q, plan=plan), ref, f"{q.name} {plan}")
    ctx.close()


def test_colliding_hash_keys(atp, oracle_mod):
    """Columns that share low bits and hash-step patterns (multiples of 2^k)."""
    hin = HIN(counts={"A": 4, "B": 64, "C": 1 << 22})
    rows = []
    for b in range(64):
        stride = 1 << (b % 12 + 8)
        rows.append(np.arange(0, min(1 << 22, stride * 300), stride, dtype=np.int64)[:300])
    _csr_rel(hin, "B", "C", rows)
    _csr_rel(hin, "A", "B", [list(range(0, 64, 2)), list(range(64)), [5], list(range(1, 64, 3))])
    q = Query("A-B-C", ["A", "B", "C"], [])
    ref = oracle_mod.eval_full(hin, q)
    ctx = make_ctx(atp, hin)
    assert_same(ctx.eval_query(q), ref)
    ctx.close()


def test_degenerate_constraints(atp, oracle_mod, tiny_cfg):
    hin, qs = tiny_cfg
    q = qs[0]
    ctx = make_ctx(atp, hin)
    cases = {
        "empty start": q.constraints + [Constraint(0, "idset", ids=np.zeros(0, np.int32))],
        "empty middle": q.constraints + [Constraint(1, "idset", ids=np.zeros(0, np.int32))],
        "empty end": q.constraints + [Constraint(4, "idset", ids=np.zeros(0, np.int32))],
        "single start": q.constraints + [Constraint(0, "idset", ids=np.array([7], np.int32))],
        "duplicate ids": q.constraints + [Constraint(0, "idset", ids=np.array([9, 3, 9, 3, 1], np.int32))],
        "all ids": [Constraint(i, "idset", ids=np.arange(hin.counts[t], dtype=np.int32))
                    for i, t in enumerate(q.types)],
        "two idsets one position": q.constraints + [Constraint(0, "idset", ids=np.arange(0, 3000, 2, dtype=np.int32)),
                                                     Constraint(0, "idset", ids=np.arange(0, 3000, 3, dtype=np.int32))],
        "unconstrained": [],
    }
    for name, cons in cases.items():
        qq = Query(q.name, q.types, cons)
        ref = oracle_mod.eval_full(hin, qq)
        for plan in [None, "(((0,1),2),3)", "(0,(1,(2,3)))"]:
            assert_same(ctx.eval_query(qq, plan=plan), ref, f"{name} {plan}")
    ctx.close()


def test_two_type_metapath(atp, oracle_mod, tiny_cfg):
    hin, _ = tiny_cfg
    ctx = make_ctx(atp, hin)
    for cons in ([], [Constraint(1, "idset", ids=np.arange(0, 2000, 5, dtype=np.int32))],
                 [Constraint(0, "idset", ids=np.arange(0, 3000, 7, dtype=np.int32))]):
        q = Query("A-P", ["A", "P"], cons)
        assert_same(ctx.eval_query(q), oracle_mod.eval_full(hin, q))
    ctx.close()


def test_range_constraints_every_dtype(atp, oracle_mod):
    hin, rng = configs.make_hin("scholarly", 0.002)
    year = hin.props[("P", "year")]
    hin.props[("P", "y32")] = year.astype(np.int32)
    hin.props[("P", "y64")] = year.astype(np.int64) - 3000
    ctx = make_ctx(atp, hin)
    for prop, lo, hi in [("year", 2015, 2021), ("y32", 1990, 1995), ("y64", -1000, -990), ("year", 3000, 4000),
                         ("y64", -(1 << 40), 1 << 40)]:
        q = Query("A-P-T-P-A", ["A", "P", "T", "P", "A"],
                  [Constraint(1, "range", prop=prop, lo=lo, hi=hi), Constraint(3, "range", prop=prop, lo=lo, hi=hi)])
        assert_same(ctx.eval_query(q), oracle_mod.eval_full(hin, q, nthreads=8), prop)
    ctx.close()


# ---------------------------------------------------------------------------
# counts beyond int64

def layered_complete(widths):
    names = [f"L{i}" for i in range(len(widths))]
    hin = HIN(counts=dict(zip(names, widths)))
    for i in range(len(widths) - 1):
        a, b = widths[i], widths[i + 1]
        rp = np.arange(a + 1, dtype=np.int64) * b
        col = np.tile(np.arange(b, dtype=np.int32), a)
        hin.relations[(names[i], names[i + 1])] = Relation(names[i], names[i + 1], rp, col)
    return hin, Query("-".join(names), names, [])


@pytest.mark.parametrize("widths,over", [
    ([1] + [128] * 9 + [1], True),       # exactly 2^63
    ([1] + [127] * 9 + [1], False),      # 127^9 < 2^63
    ([1] + [128] * 8 + [64, 1], False),  # 2^62
    ([2] + [128] * 9 + [3], True),
    ([1] + [256] * 9 + [1], True),       # 2^72: intermediate products wrap 64 bits
])
def test_overflow_is_detected_for_every_plan(atp, oracle_mod, widths, over):
    hin, q = layered_complete(widths)
    ref = oracle_mod.eval_full(hin, q)
    assert ref[3] == (oracle_mod.ORC_OVERFLOW if over else oracle_mod.ORC_OK)
    ctx = make_ctx(atp, hin)
    plans = list(all_plans(0, len(q.types) - 2))
    for plan in [None] + plans[:: max(1, len(plans) // 12)] + [plans[-1]]:
        if over:
            with pytest.raises(atp.AtpError) as e:
                ctx.eval_query(q, plan=plan)
            assert e.value.status == atp.ATP_EOVERFLOW, plan
        else:
            assert_same(ctx.eval_query(q, plan=plan), ref, str(plan))
    ctx.close()


@pytest.mark.parametrize("w,over", [(128, True), (127, False)])
def test_counts_beyond_int64_in_sparse_parts(atp, oracle_mod, w, over):
    """The last product of the left-deep plan is one start row (w entries of
    2^56 paths each) times a 60,000-column relation in which every one of
    the w nodes reaches the same 40 columns spread over eight column tiles:
    few products per tile, so the row is accumulated in sparse parts by
    column rank.  Each column receives w contributions of 2^56: 128 reach
    exactly 2^63 (ATP_EOVERFLOW, as the oracle reports), 127 stay exact."""
    k = 9
    names = [f"L{i}" for i in range(k + 2)]
    counts = {names[0]: 1, names[k]: w, names[k + 1]: 60000}
    for i in range(1, k):
        counts[names[i]] = 128
    hin = HIN(counts=counts)
    for i in range(k):
        a, b = counts[names[i]], counts[names[i + 1]]
        _csr_rel(hin, names[i], names[i + 1], [list(range(b))] * a)
    cols = [c * 1500 + 7 for c in range(40)]
    _csr_rel(hin, names[k], names[k + 1], [cols] * w)
    q = Query("-".join(names), names, [])
    ref = oracle_mod.eval_full(hin, q)
    assert ref[3] == (oracle_mod.ORC_OVERFLOW if over else oracle_mod.ORC_OK)
    ctx = make_ctx(atp, hin)
    ld = "0"
    for i in range(1, k + 1):
        ld = f"({ld},{i})"
    for plan in [ld, None]:
        if over:
            with pytest.raises(atp.AtpError) as e:
                ctx.eval_query(q, plan=plan)
            assert e.value.status == atp.ATP_EOVERFLOW, plan
        else:
            assert_same(ctx.eval_query(q, plan=plan), ref, str(plan))
    ctx.close()


def test_dead_intermediate_may_exceed_int64(atp, oracle_mod):
    """Suffix products hold counts of 2^63 on rows the start never reaches;
    the final count is 1, so every plan returns the exact result."""
    hin, q = _narrow_and_wide()
    ref = oracle_mod.eval_full(hin, q)
    assert ref[3] == oracle_mod.ORC_OK and list(ref[2]) == [1]
    ctx = make_ctx(atp, hin)
    p = len(q.types) - 1
    rd = str(p - 1)
    for i in range(p - 2, -1, -1):
        rd = f"({i},{rd})"
    for plan in [None, rd]:
        assert_same(ctx.eval_query(q, plan=plan), ref, str(plan))
    ctx.close()


# ---------------------------------------------------------------------------
# errors

def test_wait_limit_turns_a_stalled_read_into_a_device_error(atp, oracle_mod, monkeypatch):
    """The host waits for a product's posted sizes at most ATP_WAIT_LIMIT_S
    seconds; past it the query ends with ATP_EDEVICE (the context is then
    unusable, as documented) instead of spinning.  The limit is forced tiny
    from the host; the kernels themselves finish normally, and a context
    created with the default limit returns the oracle's result."""
    hin, rng = configs.make_hin("scholarly", 0.01)
    q = [x for x in configs.make_queries("scholarly", hin, rng) if x.name == "T-P-A-P-T"][0]
    monkeypatch.setenv("ATP_WAIT_LIMIT_S", "1e-9")
    ctx = make_ctx(atp, hin)
    for _ in range(2):
        with pytest.raises(atp.AtpError) as e:
            ctx.eval_query(q)
        assert e.value.status == atp.ATP_EDEVICE
    ctx.close()
    monkeypatch.delenv("ATP_WAIT_LIMIT_S")
    ctx = make_ctx(atp, hin)
    assert_same(ctx.eval_query(q), oracle_mod.eval_full(hin, q, nthreads=8))
    ctx.close()


def test_error_paths_leave_the_context_usable(atp, oracle_mod, tiny_cfg):
    hin, qs = tiny_cfg
    q = qs[0]
    ctx = make_ctx(atp, hin)
    ref = oracle_mod.eval_full(hin, q)
    with pytest.raises(atp.AtpError) as e:
        ctx.eval(["A", "T"])  # no relation A->T
    assert e.value.status == atp.ATP_ESCHEMA
    for bad in ["((0,1),(2,3)", "((0,1),(3,2))", "(0,1,2,3)", "((0,1),2)", "x"]:
        with pytest.raises(atp.AtpError) as e:
            ctx.eval_query(q, plan=bad)
        assert e.value.status == atp.ATP_EINVAL, bad
    with pytest.raises(atp.AtpError) as e:
        ctx.eval(q.types, [Constraint(0, "idset", ids=np.array([10 ** 6], np.int32))])
    assert e.value.status == atp.ATP_EINVAL
    with pytest.raises(atp.AtpError) as e:
        ctx.add_relation(0, 1, np.array([0, 2, 1] + [1] * (hin.counts["A"] - 2), np.int64), np.array([0], np.int32))
    assert e.value.status == atp.ATP_EINVAL
    assert_same(ctx.eval_query(q), ref)
    ctx.close()


def test_memory_budget(atp, oracle_mod, tiny_cfg):
    hin, qs = tiny_cfg
    q = qs[0]
    ref = oracle_mod.eval_full(hin, q)
    ctx = atp.Context(device=0, budget_bytes=1 << 20)
    with pytest.raises(atp.AtpError) as e:
        ctx.load_hin(hin)
        ctx.eval_query(q)
    assert e.value.status == atp.ATP_EBUDGET
    ctx.close()
    ctx = atp.Context(device=0, budget_bytes=256 << 20)
    ctx.load_hin(hin)
    assert_same(ctx.eval_query(q), ref)
    ctx.close()


@pytest.mark.parametrize("tune", [{"ATP_SPLIT_OPS": "1024"}, {"ATP_PART_HASH_CAP": "0"}, {"ATP_PART_TARGET": "1"},
                                  {"ATP_PART_TARGET": "100000", "ATP_TASK_OPS": "1"}, {"ATP_BUCKET_PCT": "0"},
                                  {"ATP_SPLIT_OPS": "1024", "ATP_PART_TARGET": "64", "ATP_BUCKET_PCT": "100"},
                                  {"ATP_TILE_INDEX_CAP": "0"}, {"ATP_TILE_INDEX_CAP": "0", "ATP_PART_TARGET": "1"},
                                  {"ATP_BUCKET_PCT": "0", "ATP_BUCKET_CHUNK": "64"}, {"ATP_SERIAL_BINS": "1"},
                                  {"ATP_BUCKET_PCT": "0", "ATP_CHUNK_HIST_CAP": "0"}, {"ATP_NO_MAILBOX": "1"},
                                  {"ATP_PART_TARGET": "4000"}, {"ATP_PART_TARGET": "4000", "ATP_BUCKET_PCT": "0"}])
def test_every_kernel_path_under_forced_tunings(atp, oracle_mod, tune, monkeypatch):
    """The binning thresholds only move rows between kernels (rank-accumulated
    sparse parts, dense tiles, split tiles, tile buckets) and segment bounds between the tile
    index and searches, the bins run on one stream or beside each other, and
    step totals come back through the mapped mailbox or by copies; results
    must not change."""
    for k, v in tune.items():
        monkeypatch.setenv(k, v)
    for name, scale in [("scholarly", 0.02), ("news", 0.03)]:
        hin, rng = configs.make_hin(name, scale)
        qs = configs.make_queries(name, hin, rng)
        ctx = make_ctx(atp, hin)
        for q in qs:
            ref = oracle_mod.eval_full(hin, q, nthreads=8)
            assert_same(ctx.eval_query(q), ref, f"{tune} {q.name}")
            assert_same(ctx.eval_query(q, plan="(((" + ",".join(str(i) for i in range(2)) + "),2),3)"
                                       if len(q.types) == 5 else None), ref, f"{tune} {q.name} left-deep")
        ctx.close()
    hin, qs = configs.load("tiny", use_cache=False)
    ctx = make_ctx(atp, hin)
    assert_same(ctx.eval_query(qs[0]), oracle_mod.eval_full(hin, qs[0]), f"{tune} tiny")
    ctx.close()


@pytest.mark.parametrize("tune", [{}, {"ATP_PART_TARGET": "4000"}, {"ATP_PART_HASH_CAP": "0"},
                                  {"ATP_TILE_INDEX_CAP": "0"}])
def test_masks_at_the_junction_and_the_end(atp, oracle_mod, tune, monkeypatch):
    """Id-set constraints on the middle type and on the last type of
    A-P-X-P-A (a column mask on the root's left operand and on its right
    operand, so a dense row's slots number fewer than its products and fewer
    than the columns): sparse parts, dense tiles and rows without the tile
    index must skip exactly the masked columns and keep their output ranges
    apart."""
    for k, v in tune.items():
        monkeypatch.setenv(k, v)
    hin, rng = configs.make_hin("scholarly", 0.02)
    ctx = make_ctx(atp, hin)
    for mid in ("V", "T"):
        types = ["A", "P", mid, "P", "A"]
        n_a, n_m = hin.counts["A"], hin.counts[mid]
        start = np.sort(rng.choice(n_a, size=min(300, n_a), replace=False)).astype(np.int32)
        keep_m = np.sort(rng.choice(n_m, size=max(1, n_m // 2), replace=False)).astype(np.int32)
        keep_a = np.sort(rng.choice(n_a, size=n_a // 3, replace=False)).astype(np.int32)
        q = Query("-".join(types), types, [Constraint(0, "idset", ids=start), Constraint(2, "idset", ids=keep_m),
                                            Constraint(4, "idset", ids=keep_a),
                                            Constraint(1, "range", prop="year", lo=2005, hi=32767)])
        ref = oracle_mod.eval_full(hin, q, nthreads=8)
        for plan in (None, "((0,1),(2,3))", "(((0,1),2),3)"):
            assert_same(ctx.eval_query(q, plan=plan), ref, f"{tune} {q.name} {plan}")
    ctx.close()


def test_profiling_one_kernel(atp, oracle_mod):
    """Timing every launch, then only one kernel's, leaves results as they
    are; the restricted table names only that kernel."""
    hin, rng = configs.make_hin("scholarly", 0.02)
    qs = configs.make_queries("scholarly", hin, rng)
    ctx = make_ctx(atp, hin)
    q = qs[3]
    ref = oracle_mod.eval_full(hin, q, nthreads=8)
    ctx.set_flags(profile=True)
    ctx.kernel_times_reset()
    assert_same(ctx.eval_query(q), ref, "profile all")
    every = {k: v for k, v in ctx.kernel_times().items() if v[1] > 0}
    assert "symbolic" in every and len(every) > 3
    name = max(every, key=lambda k: every[k][0])
    ctx.set_profile_kernel(name)
    ctx.kernel_times_reset()
    assert_same(ctx.eval_query(q), ref, f"profile {name}")
    only = {k: v for k, v in ctx.kernel_times().items() if v[1] > 0}
    assert set(only) == {name} and only[name][1] == every[name][1]
    ctx.set_profile_kernel(None)
    ctx.kernel_times_reset()
    ctx.eval_query(q).free()
    assert {k for k, v in ctx.kernel_times().items() if v[1] > 0} == set(every)
    ctx.close()
