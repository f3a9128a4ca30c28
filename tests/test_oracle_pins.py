"""Pins of the CPU oracle against facts fixed outside it: brute-force
enumeration of instances (Def. 2), scipy.sparse products, closed forms, the
associativity the planner relies on (Sec. 3.1), symmetry and row sums."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

from synth import tiny as tinygen
from synth.hin import HIN, Constraint, Query, Relation
from tests._brute import count_instances


def csr_to_dict(rp, col, val):
    out = {}
    for u in range(len(rp) - 1):
        for e in range(rp[u], rp[u + 1]):
            out[(u, int(col[e]))] = int(val[e])
    return out


def check_canonical(rp, col, val, n_cols):
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0)
    assert rp[-1] == len(col) == len(val)
    for u in range(len(rp) - 1):
        c = col[rp[u]:rp[u + 1]]
        assert np.all(np.diff(c) > 0)
        assert np.all((c >= 0) & (c < n_cols))
    assert np.all(val > 0)


@pytest.mark.parametrize("seed", range(300))
def test_oracle_equals_bruteforce_random(oracle_mod, seed):
    hin = tinygen.random_hin(seed, max_nodes=8)
    rng = np.random.default_rng(10_000 + seed)
    q = tinygen.random_query(hin, rng, max_len=5)
    if q is None:
        pytest.skip("schema without a walk")
    rp, col, val, st = oracle_mod.eval_full(hin, q)
    assert st == oracle_mod.ORC_OK
    check_canonical(rp, col, val, hin.counts[q.types[-1]])
    assert csr_to_dict(rp, col, val) == count_instances(hin, q)


def _random_case(seed):
    hin = tinygen.random_hin(seed, max_nodes=8)
    rng = np.random.default_rng(10_000 + seed)
    return hin, tinygen.random_query(hin, rng, max_len=5)


def _doubled_positions(q):
    pos = [c.position for c in q.constraints]
    return {p for p in pos if pos.count(p) > 1}


def test_random_cases_reach_anded_constraints():
    """The brute-force cases above include positions with two constraints
    (Def. 3 allows one per position; several are read as their conjunction),
    with both kinds mixed and with two id sets."""
    kinds = set()
    n_doubled = 0
    for seed in range(300):
        hin, q = _random_case(seed)
        if q is None:
            continue
        for p in _doubled_positions(q):
            n_doubled += 1
            kinds.add(tuple(sorted(c.kind for c in q.constraints if c.position == p)))
    assert n_doubled >= 40
    assert {("idset", "range"), ("idset", "idset"), ("range", "range")} <= kinds


def test_last_constraint_wins_mistake_is_caught(oracle_mod, monkeypatch):
    """Plant a plausible mistake in the oracle (the last constraint at a
    position replaces the earlier ones instead of being ANDed with them): the
    brute-force pin must reject it on some random case."""
    def last_wins(hin, query):
        masks = [None] * len(query.types)
        for c in query.constraints:
            masks[c.position] = oracle_mod.constraint_mask(hin, query.types[c.position], c)
        return masks

    monkeypatch.setattr(oracle_mod, "query_masks", last_wins)
    caught = 0
    for seed in range(300):
        hin, q = _random_case(seed)
        if q is None or not _doubled_positions(q):
            continue
        rp, col, val, st = oracle_mod.eval_full(hin, q)
        if csr_to_dict(rp, col, val) != count_instances(hin, q):
            caught += 1
    assert caught >= 5


def test_oracle_equals_bruteforce_tiny_config(oracle_mod, tiny_cfg):
    """The whole tiny scholarly query (A-P-T-P-A, 10% of topics), every pair."""
    hin, qs = tiny_cfg
    q = qs[0]
    rp, col, val, st = oracle_mod.eval_full(hin, q)
    assert st == oracle_mod.ORC_OK
    check_canonical(rp, col, val, hin.counts["A"])
    brute = count_instances(hin, q)
    assert csr_to_dict(rp, col, val) == brute
    assert len(brute) > 1000  # not a vacuous check


def _scipy_chain(hin, q, masks):
    mats = []
    for i in range(len(q.types) - 1):
        r = hin.rel(q.types[i], q.types[i + 1])
        mats.append(sp.csr_matrix((np.ones(r.nnz, np.int64), r.col, r.row_ptr),
                                  shape=(r.n_rows, hin.counts[q.types[i + 1]])))
    diag = [sp.diags(np.ones(hin.counts[t], np.int64) if m is None else m.astype(np.int64),
                     format="csr", dtype=np.int64) for t, m in zip(q.types, masks)]
    z = diag[0]
    for i, a in enumerate(mats):
        z = (z @ a) @ diag[i + 1]
    z = sp.csr_matrix(z)
    z.eliminate_zeros()
    z.sort_indices()
    return z


def test_oracle_equals_scipy_tiny_config(oracle_mod, tiny_cfg):
    hin, qs = tiny_cfg
    q = qs[0]
    masks = oracle_mod.query_masks(hin, q)
    rp, col, val, st = oracle_mod.eval_full(hin, q, nthreads=4)
    z = _scipy_chain(hin, q, masks)
    assert np.array_equal(rp, z.indptr.astype(np.int64))
    assert np.array_equal(col, z.indices.astype(np.int32))
    assert np.array_equal(val.astype(np.int64), z.data)


@pytest.mark.parametrize("scale", [0.002, 0.01])
@pytest.mark.parametrize("name", ["scholarly", "news"])
def test_oracle_equals_scipy_scaled_configs(oracle_mod, name, scale):
    """Every query of the scholarly and news workloads on shrunken networks."""
    from synth import configs
    hin, rng = configs.make_hin(name, scale)
    qs = configs.make_queries(name, hin, rng)
    for q in qs:
        masks = oracle_mod.query_masks(hin, q)
        rp, col, val, st = oracle_mod.eval_full(hin, q, nthreads=4)
        assert st == oracle_mod.ORC_OK
        z = _scipy_chain(hin, q, masks)
        assert np.array_equal(rp, z.indptr.astype(np.int64)), q.name
        assert np.array_equal(col, z.indices.astype(np.int32)), q.name
        assert np.array_equal(val.astype(np.int64), z.data), q.name


def test_thread_count_does_not_change_result(oracle_mod, tiny_cfg):
    hin, qs = tiny_cfg
    a = oracle_mod.eval_full(hin, qs[0], nthreads=1)
    b = oracle_mod.eval_full(hin, qs[0], nthreads=7)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)


# ---------------------------------------------------------------------------
# closed forms

def _one_venue_hin(n_p=50, n_v=7, seed=3):
    rng = np.random.default_rng(seed)
    venue = rng.integers(0, n_v, size=n_p)
    year = rng.integers(1990, 2022, size=n_p).astype(np.int16)
    hin = HIN(counts={"P": n_p, "V": n_v})
    pv_rp = np.arange(n_p + 1, dtype=np.int64)
    hin.relations[("P", "V")] = Relation("P", "V", pv_rp, venue.astype(np.int32))
    order = np.argsort(venue, kind="stable")
    vp_rp = np.zeros(n_v + 1, np.int64)
    np.cumsum(np.bincount(venue, minlength=n_v), out=vp_rp[1:])
    hin.relations[("V", "P")] = Relation("V", "P", vp_rp, order.astype(np.int32))
    hin.props[("P", "year")] = year
    return hin, venue, year


def test_vpv_is_diagonal_with_masked_paper_counts(oracle_mod):
    """With exactly one venue per paper, V-P-V is diagonal and its entry is
    the number of (constrained) papers of the venue."""
    hin, venue, year = _one_venue_hin()
    q = Query("V-P-V", ["V", "P", "V"], [Constraint(1, "range", prop="year", lo=2000, hi=2010)])
    rp, col, val, st = oracle_mod.eval_full(hin, q)
    keep = (year >= 2000) & (year <= 2010)
    expect = np.bincount(venue[keep], minlength=7)
    got = np.zeros(7, np.int64)
    for v in range(7):
        for e in range(rp[v], rp[v + 1]):
            assert col[e] == v
            got[v] = val[e]
    assert np.array_equal(got, expect)


def test_all_true_mask_equals_unconstrained(oracle_mod, tiny_cfg):
    hin, qs = tiny_cfg
    q = qs[0]
    plain = Query(q.name, q.types, [])
    full = Query(q.name, q.types, [Constraint(i, "idset", ids=np.arange(hin.counts[t], dtype=np.int32))
                                   for i, t in enumerate(q.types)])
    a = oracle_mod.eval_full(hin, plain)
    b = oracle_mod.eval_full(hin, full)
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)


def test_all_false_mask_gives_empty(oracle_mod, tiny_cfg):
    hin, qs = tiny_cfg
    q = qs[0]
    for pos in range(len(q.types)):
        qq = Query(q.name, q.types, q.constraints + [Constraint(pos, "idset", ids=np.zeros(0, np.int32))])
        rp, col, val, st = oracle_mod.eval_full(hin, qq)
        assert rp[-1] == 0 and rp.shape[0] == hin.counts["A"] + 1


def test_single_start_node_is_one_row_of_unrestricted(oracle_mod, tiny_cfg):
    hin, qs = tiny_cfg
    q = qs[0]
    rp, col, val, _ = oracle_mod.eval_full(hin, q)
    nonempty = np.nonzero(np.diff(rp))[0]
    for u in nonempty[:5]:
        qq = Query(q.name, q.types, q.constraints + [Constraint(0, "idset", ids=np.array([u], np.int32))])
        rp2, col2, val2, _ = oracle_mod.eval_full(hin, qq)
        assert np.array_equal(np.nonzero(np.diff(rp2))[0], [u])
        assert np.array_equal(col2, col[rp[u]:rp[u + 1]])
        assert np.array_equal(val2, val[rp[u]:rp[u + 1]])


def test_palindromic_query_is_symmetric(oracle_mod, tiny_cfg):
    """A-P-T-P-A with the reverse relations stored as exact transposes and
    the same constraint at mirrored positions gives R = R^T."""
    hin, qs = tiny_cfg
    rp, col, val, _ = oracle_mod.eval_full(hin, qs[0])
    n = hin.counts["A"]
    r = sp.csr_matrix((val.astype(np.int64), col, rp), shape=(n, n))
    assert (r != r.T).nnz == 0


def test_reversed_metapath_gives_transpose(oracle_mod):
    hin = tinygen.random_hin(77, max_nodes=10)
    rng = np.random.default_rng(5)
    for _ in range(20):
        q = tinygen.random_query(hin, rng, max_len=5)
        if q is None:
            continue
        if not all((q.types[i + 1], q.types[i]) in hin.relations for i in range(len(q.types) - 1)):
            continue
        # build the reverse network with exact transposes so the reverse walk exists
        rev = HIN(counts=dict(hin.counts), props=dict(hin.props))
        for (s, d), r in hin.relations.items():
            m = sp.csr_matrix((np.ones(r.nnz, np.int64), r.col, r.row_ptr), shape=(hin.counts[s], hin.counts[d]))
            t = sp.csr_matrix(m.T)
            t.sort_indices()
            rev.relations[(d, s)] = Relation(d, s, t.indptr.astype(np.int64), t.indices.astype(np.int32))
        n = len(q.types)
        qr = Query("rev", q.types[::-1], [Constraint(n - 1 - c.position, c.kind, c.prop, c.lo, c.hi, c.ids)
                                         for c in q.constraints])
        a = oracle_mod.eval_full(hin, q)
        b = oracle_mod.eval_full(rev, qr)
        ma = sp.csr_matrix((a[2].astype(np.int64), a[1], a[0]),
                           shape=(hin.counts[q.types[0]], hin.counts[q.types[-1]]))
        mb = sp.csr_matrix((b[2].astype(np.int64), b[1], b[0]),
                           shape=(hin.counts[q.types[-1]], hin.counts[q.types[0]]))
        assert (ma != mb.T).nnz == 0


def test_row_sums_equal_spmv_chain(oracle_mod, tiny_cfg):
    """R * 1 = M_1 A_1 M_2 ... A_{n-1} M_n 1, evaluated right to left as
    dense matrix-vector products (no sparse product)."""
    hin, qs = tiny_cfg
    q = qs[0]
    masks = oracle_mod.query_masks(hin, q)
    rp, col, val, _ = oracle_mod.eval_full(hin, q)
    x = np.ones(hin.counts[q.types[-1]], dtype=np.int64)
    if masks[-1] is not None:
        x = x * masks[-1]
    for i in range(len(q.types) - 2, -1, -1):
        r = hin.rel(q.types[i], q.types[i + 1])
        deg_w = np.add.reduceat(np.concatenate([x[r.col], [0]]), r.row_ptr[:-1]) \
            if r.nnz else np.zeros(r.n_rows, np.int64)
        deg_w = np.where(np.diff(r.row_ptr) > 0, deg_w, 0)
        x = deg_w if masks[i] is None else deg_w * masks[i]
    rows = np.add.reduceat(np.concatenate([val.astype(np.int64), [0]]), rp[:-1])
    rows = np.where(np.diff(rp) > 0, rows, 0)
    assert np.array_equal(rows, x)
    assert x.sum() > 0


def test_two_type_row_sum_is_masked_degree(oracle_mod, tiny_cfg):
    hin, _ = tiny_cfg
    keep = np.arange(0, hin.counts["P"], 3, dtype=np.int32)
    q = Query("A-P", ["A", "P"], [Constraint(1, "idset", ids=keep)])
    rp, col, val, _ = oracle_mod.eval_full(hin, q)
    r = hin.rel("A", "P")
    m = np.zeros(hin.counts["P"], bool)
    m[keep] = True
    deg = np.array([m[r.col[r.row_ptr[u]:r.row_ptr[u + 1]]].sum() for u in range(r.n_rows)])
    assert np.array_equal(np.diff(rp), deg)
    assert np.all(val == 1)


# ---------------------------------------------------------------------------
# associativity: every parenthesisation of the masked chain agrees (Sec. 3.1)

def _paren_trees(i, j):
    if i == j:
        yield i
        return
    for k in range(i, j):
        for left in _paren_trees(i, k):
            for right in _paren_trees(k + 1, j):
                yield (left, right)


def _masked_relation(hin, q, masks, i):
    r = hin.rel(q.types[i], q.types[i + 1])
    m = sp.csr_matrix((np.ones(r.nnz, np.int64), r.col, r.row_ptr),
                      shape=(r.n_rows, hin.counts[q.types[i + 1]]))
    if masks[i] is not None:
        m = sp.diags(masks[i].astype(np.int64)) @ m
    if masks[i + 1] is not None:
        m = m @ sp.diags(masks[i + 1].astype(np.int64))
    m = sp.csr_matrix(m)
    m.eliminate_zeros()
    m.sort_indices()
    return m.indptr.astype(np.int64), m.indices.astype(np.int32), None, m.shape


def test_every_parenthesisation_agrees(oracle_mod):
    """orc_spgemm over all Catalan(n-2) orders equals the row-chain result."""
    hin = tinygen.random_hin(11, max_nodes=12, p_rel=1.0)
    rng = np.random.default_rng(12)
    done = 0
    while done < 6:
        q = tinygen.random_query(hin, rng, max_len=6)
        if q is None or len(q.types) < 4:
            continue
        masks = oracle_mod.query_masks(hin, q)
        ref = oracle_mod.eval_full(hin, q)
        leaves = [_masked_relation(hin, q, masks, i) for i in range(len(q.types) - 1)]

        def ev(t):
            if isinstance(t, int):
                rp, col, val, shape = leaves[t]
                return rp, col, val, shape
            a, b = ev(t[0]), ev(t[1])
            rp, col, val, st = oracle_mod.spgemm(a[3][0], b[3][1], a[0], a[1], a[2], b[0], b[1], b[2])
            return rp, col, val.astype(np.int64), (a[3][0], b[3][1])

        n_trees = 0
        for t in _paren_trees(0, len(q.types) - 2):
            rp, col, val, _ = ev(t)
            assert np.array_equal(rp, ref[0]) and np.array_equal(col, ref[1])
            assert np.array_equal(val, ref[2].astype(np.int64))
            n_trees += 1
        catalan = [1, 1, 2, 5, 14, 42][len(q.types) - 2]
        assert n_trees == catalan
        done += 1


def test_spgemm_valued_matches_scipy(oracle_mod):
    rng = np.random.default_rng(3)
    for _ in range(20):
        m, k, n = rng.integers(1, 40, size=3)
        x = sp.random(m, k, density=0.2, random_state=rng, format="csr",
                      data_rvs=lambda s: rng.integers(1, 1000, size=s)).astype(np.int64)
        y = sp.random(k, n, density=0.2, random_state=rng, format="csr",
                      data_rvs=lambda s: rng.integers(1, 1000, size=s)).astype(np.int64)
        x.sort_indices(); y.sort_indices()
        rp, col, val, st = oracle_mod.spgemm(m, n, x.indptr, x.indices, x.data, y.indptr, y.indices, y.data)
        z = sp.csr_matrix(x @ y)
        z.eliminate_zeros(); z.sort_indices()
        assert np.array_equal(rp, z.indptr) and np.array_equal(col, z.indices)
        assert np.array_equal(val.astype(np.int64), z.data)


def _python_product(m, n, x, y):
    """Exact Z = X * Y with Python integers (no fixed width), as a dict."""
    out = {}
    for i in range(m):
        for e in range(x.indptr[i], x.indptr[i + 1]):
            k, a = int(x.indices[e]), int(x.data[e])
            for f in range(y.indptr[k], y.indptr[k + 1]):
                j = int(y.indices[f])
                out[(i, j)] = out.get((i, j), 0) + a * int(y.data[f])
    return out


def _large_value_case(oracle_mod, seed):
    """Valued operands between 2^31 and 2^62: each entry of the oracle's
    product is the exact sum (Python integers) when below 2^63 and 2^63
    otherwise, and the status says overflow exactly when some entry reached
    2^63 (the int64 reading of the counts)."""
    rng = np.random.default_rng(100 + seed)
    m, k, n = (int(v) for v in rng.integers(2, 12, size=3))
    # X entries of b bits, b in [31, 62]; Y entries of about 61 - b bits, so
    # that products and their sums straddle 2^63
    bx = int(rng.integers(31, 63))
    by = max(1, 61 - bx)

    def vals_of(bits):
        def draw(size):
            b = np.clip(bits + rng.integers(-2, 2, size=size), 1, 62)
            return np.array([int(rng.integers(1 << (int(v) - 1), 1 << int(v))) for v in b], dtype=np.int64)
        return draw

    x = sp.random(m, k, density=0.5, random_state=rng, format="csr", data_rvs=vals_of(bx), dtype=np.int64)
    y = sp.random(k, n, density=0.5, random_state=rng, format="csr", data_rvs=vals_of(by), dtype=np.int64)
    assert x.data.dtype == np.int64 and y.data.dtype == np.int64
    x.sort_indices(); y.sort_indices()
    exact = _python_product(m, n, x, y)
    rp, col, val, st = oracle_mod.spgemm(m, n, x.indptr, x.indices, x.data.astype(np.int64),
                                         y.indptr, y.indices, y.data.astype(np.int64))
    got = csr_to_dict(rp, col, val)
    assert set(got) == {ij for ij, v in exact.items() if v != 0}
    for ij, v in exact.items():
        assert got[ij] == min(v, 1 << 63), ij
    over = any(v >= (1 << 63) for v in exact.values())
    assert st == (oracle_mod.ORC_OVERFLOW if over else oracle_mod.ORC_OK)
    return sum(1 for v in exact.values() if v >= (1 << 63)), sum(1 for v in exact.values() if 0 < v < (1 << 63))


@pytest.mark.parametrize("seed", range(12))
def test_spgemm_large_values_saturate_exactly(oracle_mod, seed):
    _large_value_case(oracle_mod, seed)


def test_large_value_cases_straddle_the_bound(oracle_mod):
    """The random large-value cases hold entries on both sides of 2^63 and
    cases with and without overflow."""
    stats = [_large_value_case(oracle_mod, s) for s in range(12)]
    assert sum(a for a, _ in stats) > 20 and sum(b for _, b in stats) > 20
    assert any(a == 0 for a, _ in stats) and any(a > 0 for a, _ in stats)


@pytest.mark.parametrize("terms,total", [
    ([(7, 1317624576693539401)], (1 << 63) - 1),                   # 7 * (2^63 - 1) / 7
    ([(1 << 32, 1 << 31)], 1 << 63),                               # exactly 2^63
    ([(1 << 31, 1 << 31), (1 << 62, 1)], (1 << 62) + (1 << 62)),   # two terms reaching 2^63
    ([(3, 1 << 61), (1, (1 << 61) - 1)], (1 << 63) - 1),            # two terms just below
    ([((1 << 62) + 1, 3)], 3 * ((1 << 62) + 1)),                     # one product far above
])
def test_spgemm_saturation_boundary(oracle_mod, terms, total):
    """One output entry made of the given products x*y (1 x t times t x 1):
    below 2^63 it is exact, at or above it reads 2^63 with ORC_OVERFLOW."""
    t = len(terms)
    xrp = np.array([0, t], np.int64)
    xcol = np.arange(t, dtype=np.int32)
    xval = np.array([a for a, _ in terms], np.int64)
    yrp = np.arange(t + 1, dtype=np.int64)
    ycol = np.zeros(t, np.int32)
    yval = np.array([b for _, b in terms], np.int64)
    assert sum(a * b for a, b in terms) == total
    rp, col, val, st = oracle_mod.spgemm(1, 1, xrp, xcol, xval, yrp, ycol, yval)
    assert list(rp) == [0, 1] and list(col) == [0]
    assert int(val[0]) == min(total, 1 << 63)
    assert st == (oracle_mod.ORC_OVERFLOW if total >= (1 << 63) else oracle_mod.ORC_OK)


# ---------------------------------------------------------------------------
# overflow: counts are exact, a final count >= 2^63 is reported

def layered_complete(widths):
    """Types L0..Lk with complete bipartite relations L_i -> L_{i+1}; the
    number of instances between the end nodes is prod(widths[1:-1])."""
    names = [f"L{i}" for i in range(len(widths))]
    hin = HIN(counts=dict(zip(names, widths)))
    for i in range(len(widths) - 1):
        a, b = widths[i], widths[i + 1]
        rp = np.arange(a + 1, dtype=np.int64) * b
        col = np.tile(np.arange(b, dtype=np.int32), a)
        hin.relations[(names[i], names[i + 1])] = Relation(names[i], names[i + 1], rp, col)
    return hin, Query("-".join(names), names, [])


@pytest.mark.parametrize("widths,count,over", [
    ([1] + [128] * 9 + [1], 1 << 63, True),            # exactly 2^63
    ([1] + [128] * 8 + [64, 1], 1 << 62, False),       # 2^62 fits
    ([2] + [128] * 9 + [3], 1 << 63, True),
    ([1] + [127] * 9 + [1], 127 ** 9, False),          # just below 2^63
])
def test_overflow_boundary(oracle_mod, widths, count, over):
    hin, q = layered_complete(widths)
    rp, col, val, st = oracle_mod.eval_full(hin, q)
    assert st == (oracle_mod.ORC_OVERFLOW if over else oracle_mod.ORC_OK)
    assert np.all(val == np.uint64(min(count, 1 << 63)))
    assert len(val) == widths[0] * widths[-1]
