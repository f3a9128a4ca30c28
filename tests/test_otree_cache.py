"""Host-only pins of the Overlap Tree (Sec. 3.3) and the cache replacement
policies (Sec. 3.4, Algorithm 1), through the library's C-ABI."""
import numpy as np
import pytest


@pytest.fixture(scope="module")
def atp():
    import os
    import paper_2201_04058_amd as atp
    if not os.path.exists(atp.LIB_PATH):
        from paper_2201_04058_amd import build
        build.build()
    atp.lib()
    return atp


def occurrences(strings, sub):
    n = 0
    for s in strings:
        for i in range(len(s) - len(sub) + 1):
            if list(s[i:i + len(sub)]) == list(sub):
                n += 1
    return n


@pytest.mark.parametrize("seed", range(40))
def test_overlap_tree_shape_and_frequencies(atp, seed):
    rng = np.random.default_rng(seed)
    alpha = int(rng.integers(2, 6))
    strings = [list(rng.integers(0, alpha, size=int(rng.integers(1, 8)))) for _ in range(int(rng.integers(1, 25)))]
    t = atp.OverlapTree()
    for s in strings:
        t.insert(s)
    sh = t.shape()
    lam = sum(len(s) for s in strings)
    # one leaf per suffix; internal nodes branch; leaves have f = 1 (Sec. 3.3)
    assert sh["lambda"] == lam
    assert sh["leaves"] == lam
    assert sh["thin_internal"] == 0
    assert sh["leaves_f_not_1"] == 0
    assert sh["nodes"] - 1 <= 2 * lam - 1  # space bound, root excluded
    subs = {tuple(s[i:j]) for s in strings for i in range(len(s)) for j in range(i + 1, len(s) + 1)}
    for sub in subs:
        assert t.frequency(sub) == occurrences(strings, sub), sub
    for _ in range(20):
        sub = tuple(rng.integers(0, alpha + 1, size=int(rng.integers(1, 5))))
        assert t.frequency(sub) == occurrences(strings, sub)


def test_overlap_tree_repeated_and_prefix_queries(atp):
    t = atp.OverlapTree()
    for s in ([1, 2, 3, 4], [1, 2, 3, 4], [1, 2], [2, 3, 4, 5]):
        t.insert(s)
    assert t.frequency([1, 2]) == 3
    assert t.frequency([2, 3, 4]) == 3
    assert t.frequency([1, 2, 3, 4]) == 2
    assert t.frequency([4, 5]) == 1
    assert t.frequency([5, 1]) == 0
    assert t.shape()["leaves"] == 14


# ---------------------------------------------------------------------------
# Algorithm 1 and its baselines, replayed independently

def replay(policy, budget, size, cost, parent, req):
    """PGDS with inflation L (utility h = f*c/s + L); the Overlap-Tree variant
    moves an item's cost into / out of the cached items in its subtree on
    eviction / insertion; LRU evicts the least recently requested.  Items over
    80% of the budget are never admitted."""
    n = len(size)
    desc = [[] for _ in range(n)]
    for i in range(n):
        p = parent[i]
        while p >= 0:
            desc[p].append(i)
            p = parent[p]
    c = [float(x) for x in cost]
    f = [0] * n
    lval = [0.0] * n
    h = [0.0] * n
    last = [0] * n
    cached = [False] * n
    L = 0.0
    used = 0.0
    clock = 0
    hits, after = [], []

    def util(i):
        h[i] = (f[i] * c[i] / size[i] if size[i] > 0 else 0.0) + lval[i]

    for i in req:
        f[i] += 1
        clock += 1
        last[i] = clock
        hits.append(cached[i])
        if cached[i]:
            lval[i] = L
            util(i)
            after.append(True)
            continue
        if size[i] > 0.8 * budget:
            after.append(False)
            continue
        ok = True
        while used + size[i] > budget:
            live = [k for k in range(n) if cached[k]]
            if not live:
                ok = False
                break
            if policy == "lru":
                q = min(live, key=lambda k: (last[k], k))
            else:
                q = min(live, key=lambda k: (h[k], k))
                L = h[q]
            cached[q] = False
            used -= size[q]
            if policy == "otree":
                for e in desc[q]:
                    if cached[e]:
                        c[e] += c[q]
                        util(e)
        if not ok:
            after.append(False)
            continue
        cached[i] = True
        used += size[i]
        lval[i] = L
        util(i)
        if policy == "otree":
            for e in desc[i]:
                if cached[e]:
                    c[e] -= c[i]
                    util(e)
        after.append(True)
    return np.array(hits), np.array(after), np.array(cached)


@pytest.mark.parametrize("seed", range(60))
@pytest.mark.parametrize("policy", ["otree", "pgds", "lru"])
def test_policy_matches_replay(atp, policy, seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2, 25))
    size = rng.integers(1, 50, size=n).astype(np.float64)
    cost = rng.integers(1, 100, size=n).astype(np.float64)
    parent = np.full(n, -1, np.int32)
    for i in range(1, n):  # a forest: parents have smaller ids
        if rng.random() < 0.6:
            parent[i] = int(rng.integers(0, i))
    budget = float(rng.integers(20, 200))
    req = rng.integers(0, n, size=int(rng.integers(1, 200))).astype(np.int32)
    pid = {"otree": atp.ATP_CACHE_OTREE, "pgds": atp.ATP_CACHE_PGDS, "lru": atp.ATP_CACHE_LRU}[policy]
    got = atp.cache_simulate(pid, budget, size, cost, parent, req)
    ref = replay(policy, budget, size, cost, parent, req)
    for g, r in zip(got, ref):
        assert np.array_equal(g, r)


def test_policy_worked_cases(atp):
    # LRU evicts the least recently used; PGDS keeps the costly-per-byte item
    size = [10, 10, 10]
    cost = [100, 1, 1]
    parent = [-1, -1, -1]
    req = [0, 1, 2]
    _, _, fin = atp.cache_simulate(atp.ATP_CACHE_LRU, 20, size, cost, parent, req)
    assert list(fin) == [False, True, True]
    _, _, fin = atp.cache_simulate(atp.ATP_CACHE_PGDS, 20, size, cost, parent, req)
    assert fin[0] and fin[2] and not fin[1]
    # an item over 80% of the budget is never cached
    hit, after, fin = atp.cache_simulate(atp.ATP_CACHE_OTREE, 100, [81, 10], [1, 1], [-1, -1], [0, 0, 1])
    assert not after[0] and not after[1] and after[2]
