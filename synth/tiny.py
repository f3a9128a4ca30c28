"""Small random HINs and constrained metapaths for exhaustive checks.

Random schemas (2-4 node types, self-relations allowed, relations directed
and independent), one small integer property per type, and random schema
walks with random per-position constraints, including the degenerate ones:
empty id sets, ranges that keep nothing or everything, empty relations, and
positions that carry two constraints at once.
"""
from __future__ import annotations

import numpy as np

from .hin import HIN, Constraint, Query, Relation


def random_hin(seed: int, max_nodes: int = 12, max_types: int = 4,
               p_rel: float = 0.7) -> HIN:
    rng = np.random.default_rng(seed)
    nt = int(rng.integers(2, max_types + 1))
    names = [f"t{i}" for i in range(nt)]
    counts = {n: int(rng.integers(1, max_nodes + 1)) for n in names}
    hin = HIN(counts=counts)
    for a in names:
        for b in names:
            if rng.random() >= p_rel:
                continue
            dens = float(rng.choice([0.0, 0.1, 0.3, 0.6, 1.0]))
            dense = rng.random((counts[a], counts[b])) < dens
            rp = np.zeros(counts[a] + 1, dtype=np.int64)
            np.cumsum(dense.sum(axis=1), out=rp[1:])
            col = np.nonzero(dense)[1].astype(np.int32)
            hin.relations[(a, b)] = Relation(a, b, rp, col)
    for n in names:
        hin.props[(n, "p")] = rng.integers(0, 10, size=counts[n]).astype(np.int32)
    return hin


def random_query(hin: HIN, rng: np.random.Generator, max_len: int = 6,
                 p_double: float = 0.25) -> Query | None:
    outs = {}
    for (s, d) in hin.relations:
        outs.setdefault(s, []).append(d)
    starts = sorted(outs)
    if not starts:
        return None
    n = int(rng.integers(2, max_len + 1))
    t = starts[int(rng.integers(len(starts)))]
    types = [t]
    while len(types) < n:
        nb = sorted(outs.get(types[-1], []))
        if not nb:
            break
        types.append(nb[int(rng.integers(len(nb)))])
    if len(types) < 2:
        return None
    cons = []

    def draw(i, ty, u):
        if u < 0.3:
            lo = int(rng.integers(-1, 10))
            hi = int(rng.integers(lo - 1, 11))
            cons.append(Constraint(i, "range", prop="p", lo=lo, hi=hi))
        elif u < 0.45:
            k = int(rng.integers(0, hin.counts[ty] + 1))
            ids = np.sort(rng.choice(hin.counts[ty], size=k, replace=False)).astype(np.int32)
            cons.append(Constraint(i, "idset", ids=ids))

    for i, ty in enumerate(types):
        draw(i, ty, rng.random())
        if rng.random() < p_double:
            # a second constraint at the same position (range and id set, two
            # id sets or two ranges): the position keeps what passes both
            draw(i, ty, 0.45 * rng.random())
    return Query("-".join(types), types, cons)
