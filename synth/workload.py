"""Seeded metapath query workloads.

Sessions as in the paper's workloads (Sec. 4.1, "Query Workloads"): a data
scientist explores one entity of interest, fixed by an equality constraint
(here: an id-set of one node at the first position), with consecutive
metapath queries; at each step a new session (new entity and metapath) starts
with restart probability p, otherwise the session continues with the same
entity and a different metapath.  Metapaths are schema walks of 3..5 node
types starting at the entity's type; the queries are shuffled at the end.
Selections are uniform (default) or Zipf.  Type-level property predicates
(e.g. P.year >= 2015) can be added at every position of their type.
"""
from __future__ import annotations

import numpy as np

from .hin import HIN, Constraint, Query


def schema_walks(hin: HIN, start: str, lengths=(3, 4, 5)) -> list:
    """Every walk on the relation schema of the given lengths from `start`."""
    out = {}
    for (s, d) in hin.relations:
        out.setdefault(s, []).append(d)
    walks = []

    def rec(path):
        if len(path) in lengths:
            walks.append(list(path))
        if len(path) >= max(lengths):
            return
        for nb in sorted(out.get(path[-1], [])):
            rec(path + [nb])

    rec([start])
    return walks


def sessions(hin: HIN, seed: int, n_queries: int, start_type, restart_p: float = 0.08,
             lengths=(3, 4, 5), zipf: float = 0.0, entities: int = 200, type_predicates=None) -> list:
    """The shuffled query list of a session workload.

    ``start_type`` is a node type or a list of them (each session picks one
    uniformly).  ``type_predicates`` maps a node type to (prop, lo, hi): a
    range constraint added at every position of that type.  Entities are drawn
    from a seeded pool of ``entities`` random nodes per start type.
    """
    rng = np.random.default_rng(seed)
    starts = [start_type] if isinstance(start_type, str) else list(start_type)
    walks = {t: schema_walks(hin, t, lengths) for t in starts}
    pools = {t: rng.choice(hin.counts[t], size=min(entities, hin.counts[t]), replace=False) for t in starts}

    def pick(n):
        if zipf > 0:
            w = np.arange(1, n + 1, dtype=np.float64) ** (-zipf)
            return int(rng.choice(n, p=w / w.sum()))
        return int(rng.integers(n))

    def new_session():
        t = starts[int(rng.integers(len(starts)))]
        return t, int(pools[t][pick(len(pools[t]))])

    qs = []
    stype, entity = new_session()
    last = -1
    for z in range(n_queries):
        if z > 0 and rng.random() < restart_p:
            stype, entity = new_session()
            last = -1
        ws = walks[stype]
        wi = pick(len(ws))
        if wi == last and len(ws) > 1:
            wi = (wi + 1) % len(ws)
        last = wi
        types = ws[wi]
        cons = [Constraint(0, "idset", ids=np.array([entity], dtype=np.int32))]
        for i, t in enumerate(types):
            if type_predicates and t in type_predicates:
                prop, lo, hi = type_predicates[t]
                cons.append(Constraint(i, "range", prop=prop, lo=lo, hi=hi))
        qs.append(Query("-".join(types), types, cons))
    order = rng.permutation(len(qs))
    return [qs[i] for i in order]


# ---------------------------------------------------------------------------
# batched and streamed workloads

# the range property of the type that carries the workload's predicate
WINDOW_PROPS = {"P": ("year", 1990, 2021), "D": ("day", 0, 1095)}


def _neighbours(hin: HIN) -> dict:
    nb = {}
    for (s, d) in hin.relations:
        nb.setdefault(s, []).append(d)
    return {k: sorted(v) for k, v in nb.items()}


def _window(rng, sel: float, lo: int, hi: int) -> tuple:
    """A window of max(1, round(span * sel)) consecutive values of [lo, hi]."""
    span = hi - lo + 1
    w = max(1, int(round(span * sel)))
    a = lo + int(rng.integers(0, span - w + 1))
    return a, a + w - 1


def _start_set(rng, n_nodes: int, size: int) -> np.ndarray:
    return np.sort(rng.choice(n_nodes, size=min(size, n_nodes), replace=False)).astype(np.int32)


def _query(types, ids, window) -> Query:
    cons = [Constraint(0, "idset", ids=ids)]
    for i, t in enumerate(types):
        if t in WINDOW_PROPS and window is not None:
            cons.append(Constraint(i, "range", prop=WINDOW_PROPS[t][0], lo=window[0], hi=window[1]))
    return Query("-".join(types), list(types), cons)


def random_walk_batch(hin: HIN, seed: int = 3, n: int = 256, lengths=(3, 7), start_sizes=(100, 5000),
                      selectivity=(0.01, 0.20)) -> list:
    """Random schema walks: start type uniform, each next type uniform over
    the schema neighbours, length uniform in ``lengths``; a seeded start set of
    uniform size in ``start_sizes``; a window predicate of selectivity uniform
    in ``selectivity`` at every position of the predicate's type."""
    rng = np.random.default_rng(seed)
    nb = _neighbours(hin)
    types = list(hin.counts)
    wtype = [t for t in types if t in WINDOW_PROPS]
    out = []
    for _ in range(n):
        k = int(rng.integers(lengths[0], lengths[1] + 1))
        walk = [types[int(rng.integers(len(types)))]]
        while len(walk) < k:
            cand = nb[walk[-1]]
            walk.append(cand[int(rng.integers(len(cand)))])
        ids = _start_set(rng, hin.counts[walk[0]], int(rng.integers(start_sizes[0], start_sizes[1] + 1)))
        win = None
        if wtype:
            _, lo, hi = WINDOW_PROPS[wtype[0]]
            win = _window(rng, float(rng.uniform(*selectivity)), lo, hi)
        out.append(_query(walk, ids, win))
    return out


def serving_stream(hin: HIN, seed: int = 4, n: int = 20000, qps: float = 200.0, n_base: int = 500,
                   base_lengths=(3, 5), affix=(0, 2), zipf: float = 1.0, start_sizes=(100, 5000),
                   selectivity=(0.01, 0.20), pool: int = 16) -> tuple:
    """An open-loop query stream: (arrival times in s, queries).

    Each query is a base walk drawn Zipf(``zipf``) over ``n_base`` seeded
    schema walks of ``base_lengths`` types, extended by a random walk prefix
    and suffix of ``affix`` steps each.  Constraints come from finite seeded
    pools so that overlaps recur as in session workloads: ``pool`` start sets
    per node type (sizes uniform in ``start_sizes``) and ``pool`` windows
    (selectivity uniform in ``selectivity``) applied at every position of the
    predicate's type.  Arrivals are Poisson at ``qps``."""
    rng = np.random.default_rng(seed)
    nb = _neighbours(hin)
    types = list(hin.counts)
    bases = []
    for _ in range(n_base):
        k = int(rng.integers(base_lengths[0], base_lengths[1] + 1))
        walk = [types[int(rng.integers(len(types)))]]
        while len(walk) < k:
            cand = nb[walk[-1]]
            walk.append(cand[int(rng.integers(len(cand)))])
        bases.append(walk)
    starts = {t: [_start_set(rng, hin.counts[t], int(rng.integers(start_sizes[0], start_sizes[1] + 1)))
                  for _ in range(pool)] for t in types}
    wtype = [t for t in types if t in WINDOW_PROPS]
    windows = []
    if wtype:
        _, lo, hi = WINDOW_PROPS[wtype[0]]
        windows = [_window(rng, float(rng.uniform(*selectivity)), lo, hi) for _ in range(pool)]
    w = np.arange(1, n_base + 1, dtype=np.float64) ** (-zipf)
    w /= w.sum()
    ranks = rng.choice(n_base, size=n, p=w)
    gaps = rng.exponential(1.0 / qps, size=n)
    arrivals = np.cumsum(gaps) - gaps[0]
    out = []
    for z in range(n):
        walk = list(bases[ranks[z]])
        for _ in range(int(rng.integers(affix[0], affix[1] + 1))):  # prefix: walk backwards
            cand = nb[walk[0]]
            walk.insert(0, cand[int(rng.integers(len(cand)))])
        for _ in range(int(rng.integers(affix[0], affix[1] + 1))):
            cand = nb[walk[-1]]
            walk.append(cand[int(rng.integers(len(cand)))])
        ids = starts[walk[0]][int(rng.integers(pool))]
        win = windows[int(rng.integers(len(windows)))] if windows else None
        out.append(_query(walk, ids, win))
    return arrivals, out
