"""Workload evaluation with the intermediate-result cache (Sec. 3.3-3.4):
every query's result equals the oracle's whatever the policy and budget, and
the cache is actually used (hits) and replaced (evictions)."""
import numpy as np
import pytest

from synth import configs, workload
from synth.hin import Constraint, Query
from tests._nets import _narrow_and_wide

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def atp():
    import paper_2201_04058_amd as atp
    atp.lib()
    return atp


@pytest.fixture(scope="module")
def scholarly_small():
    hin, _ = configs.make_hin("scholarly", 0.01)
    qs = workload.sessions(hin, 11, 60, "A", restart_p=0.1, entities=12,
                           type_predicates={"P": ("year", 2012, 32767)})
    return hin, qs


def same(res, ref):
    rp, col, val = res.to_host()
    return (np.array_equal(rp, ref[0]) and np.array_equal(col, ref[1])
            and np.array_equal(val, ref[2].astype(np.int64)))


POLICIES = ["ATP_CACHE_OTREE", "ATP_CACHE_PGDS", "ATP_CACHE_LRU", "ATP_CACHE_CBS1", "ATP_CACHE_CBS2"]


@pytest.mark.parametrize("budget", [1 << 17, 1 << 30])
@pytest.mark.parametrize("policy", POLICIES)
def test_workload_results_equal_oracle(atp, oracle_mod, scholarly_small, policy, budget):
    hin, qs = scholarly_small
    ctx = atp.Context(device=0)
    ctx.load_hin(hin)
    ctx.cache_configure(getattr(atp, policy), budget)
    refs = {}
    for z, q in enumerate(qs):
        key = (q.name, int(q.constraints[0].ids[0]))
        if key not in refs:
            refs[key] = oracle_mod.eval_full(hin, q)
        res = ctx.eval_query(q)
        assert same(res, refs[key]), f"{policy} query {z} {q.name}"
        res.free()
    st = ctx.cache_stats()
    assert st["queries"] == len(qs)
    assert st["insert_attempts"] > 0
    if budget == 1 << 30:
        assert st["whole_hits"] + st["sub_hits"] > 0, st
        assert st["evictions"] == 0
    else:
        assert st["bytes"] <= budget
    if policy != "ATP_CACHE_CBS1":
        assert st["otree_leaves"] == sum(len(q.types) for q in qs)
    ctx.close()


def test_repeated_query_is_a_whole_hit_and_sub_results_are_reused(atp, oracle_mod, scholarly_small):
    hin, _ = scholarly_small
    ctx = atp.Context(device=0)
    ctx.load_hin(hin)
    ctx.cache_configure(atp.ATP_CACHE_OTREE, 1 << 30)
    ent = np.array([5], np.int32)
    yr = Constraint(1, "range", prop="year", lo=2012, hi=32767)
    q1 = Query("A-P-T-P-A", ["A", "P", "T", "P", "A"],
               [Constraint(0, "idset", ids=ent), yr, Constraint(3, "range", prop="year", lo=2012, hi=32767)])
    ref = oracle_mod.eval_full(hin, q1)
    assert same(ctx.eval_query(q1), ref)
    assert same(ctx.eval_query(q1), ref)
    st = ctx.cache_stats()
    assert st["whole_hits"] == 1
    # a longer query sharing the cached prefix reuses it
    q2 = Query("A-P-T-P-A-P-V", ["A", "P", "T", "P", "A", "P", "V"],
               q1.constraints + [Constraint(5, "range", prop="year", lo=2012, hi=32767)])
    assert same(ctx.eval_query(q2), oracle_mod.eval_full(hin, q2))
    st2 = ctx.cache_stats()
    assert st2["sub_hits"] >= 1
    # a plan token for a block that is cached is accepted, an uncached one is not
    r = ctx.eval_query(q2, plan="([0-3],(4,5))")
    assert same(r, oracle_mod.eval_full(hin, q2))
    with pytest.raises(atp.AtpError) as e:
        ctx.eval_query(q2, plan="(0,[1-5])")
    assert e.value.status == atp.ATP_EINVAL
    ctx.close()


def test_cached_block_as_restricted_left_operand(atp, oracle_mod, scholarly_small):
    """A cached sub-chain that is the left operand of a product whose rows are
    restricted (its left neighbour picks few columns) multiplies only the
    listed rows: same result, fewer products than over all its rows."""
    hin, _ = scholarly_small
    ctx = atp.Context(device=0)
    ctx.load_hin(hin)
    ctx.cache_configure(atp.ATP_CACHE_OTREE, 1 << 30)
    # one publication year keeps the co-authorship block small (about 0.6M entries)
    yr = lambda pos: Constraint(pos, "range", prop="year", lo=2015, hi=2015)
    sub = Query("P-A-P", ["P", "A", "P"], [yr(0), yr(2)])
    for _ in range(2):
        ctx.eval_query(sub).free()
    assert ctx.cache_stats()["whole_hits"] == 1
    q = Query("A-P-A-P-V", ["A", "P", "A", "P", "V"],
              [Constraint(0, "idset", ids=np.array([20], np.int32)), yr(1), yr(3)])
    ref = oracle_mod.eval_full(hin, q)
    r = ctx.eval_query(q, plan="(0,([1-2],3))")
    assert same(r, ref)
    n_op_restricted = r.stats()["n_op"]
    ctx.set_flags(no_restrict=True)
    r2 = ctx.eval_query(q, plan="(0,([1-2],3))")
    assert same(r2, ref)
    assert n_op_restricted < r2.stats()["n_op"]
    ctx.close()


def test_out_of_memory_with_the_cache_retries_restricted(atp, oracle_mod, scholarly_small):
    """P-T-P-A seen before makes the cache compute that right sub-chain on all
    its rows (about 8e7 entries) so it can be kept; under a 256 MiB budget that
    fails, and the query is evaluated again restricted to one author's papers."""
    hin, _ = scholarly_small
    ctx = atp.Context(device=0, budget_bytes=256 << 20)
    ctx.load_hin(hin)
    ctx.cache_configure(atp.ATP_CACHE_OTREE, 1 << 30)
    yr = lambda pos: Constraint(pos, "range", prop="year", lo=2012, hi=32767)
    seen = Query("P-T-P-A", ["P", "T", "P", "A"],
                 [Constraint(0, "idset", ids=np.array([24806], np.int32)), yr(0), yr(2)])
    ctx.eval_query(seen).free()
    q = Query("A-P-T-P-A", ["A", "P", "T", "P", "A"],
              [Constraint(0, "idset", ids=np.array([1], np.int32)), yr(1), yr(3)])
    r = ctx.eval_query(q, plan="(0,((1,2),3))")
    assert same(r, oracle_mod.eval_full(hin, q))
    r.free()
    assert ctx.cache_stats()["queries"] == 2
    ctx.close()


def test_cache_off_again_matches(atp, oracle_mod, scholarly_small):
    hin, qs = scholarly_small
    ctx = atp.Context(device=0)
    ctx.load_hin(hin)
    ctx.cache_configure(atp.ATP_CACHE_OTREE, 1 << 30)
    for q in qs[:10]:
        ctx.eval_query(q).free()
    ctx.cache_configure(atp.ATP_CACHE_OFF, 0)
    for q in qs[10:20]:
        assert same(ctx.eval_query(q), oracle_mod.eval_full(hin, q))
    assert ctx.cache_stats()["queries"] == 0
    ctx.close()


@pytest.mark.parametrize("policy", ["ATP_CACHE_CBS2", "ATP_CACHE_OTREE"])
def test_saturated_intermediate_is_not_served_from_the_cache(atp, oracle_mod, policy):
    """A sub-chain whose counts reach 2^63 on rows the query's start never
    reaches (a dead intermediate): the query itself is exact, and a later
    query equal to that sub-chain must still report ATP_EOVERFLOW, as the
    oracle does (Problem 1 with int64 counts), not a cached saturated copy."""
    hin, q = _narrow_and_wide()
    ref = oracle_mod.eval_full(hin, q)
    assert ref[3] == oracle_mod.ORC_OK
    suffix = Query("-".join(q.types[1:]), q.types[1:], [])
    assert oracle_mod.eval_full(hin, suffix)[3] == oracle_mod.ORC_OVERFLOW
    ctx = atp.Context(device=0)
    ctx.load_hin(hin)
    ctx.set_flags(no_restrict=True)  # suffix products on all their rows: cache candidates
    ctx.cache_configure(getattr(atp, policy), 1 << 30)
    p = len(q.types) - 1
    rd = str(p - 1)
    for i in range(p - 2, -1, -1):
        rd = f"({i},{rd})"
    for _ in range(3):  # the suffix recurs: every policy considers it
        res = ctx.eval_query(q, plan=rd)
        assert same(res, ref)
        res.free()
    for _ in range(2):
        with pytest.raises(atp.AtpError) as e:
            ctx.eval_query(suffix)
        assert e.value.status == atp.ATP_EOVERFLOW
    ctx.close()
