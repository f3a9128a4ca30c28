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
