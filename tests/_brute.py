"""Brute-force enumeration of metapath instances (Def. 2): walk every typed
path and count arrivals.  Independent of the oracle's sparse-product code."""
from collections import defaultdict


def node_ok(hin, query, pos, v):
    for c in query.constraints:
        if c.position != pos:
            continue
        t = query.types[pos]
        if c.kind == "range":
            x = int(hin.props[(t, c.prop)][v])
            if not (c.lo <= x <= c.hi):
                return False
        elif c.kind == "idset":
            if v not in set(int(i) for i in c.ids):
                return False
    return True


def count_instances(hin, query):
    """dict (u, v) -> number of instances of the constrained metapath."""
    types = query.types
    n = len(types)
    adj = []
    for i in range(n - 1):
        r = hin.rel(types[i], types[i + 1])
        rp, col = r.row_ptr, r.col
        adj.append([[int(c) for c in col[rp[k]:rp[k + 1]]] for k in range(r.n_rows)])
    ok = [[node_ok(hin, query, i, v) for v in range(hin.counts[types[i]])] for i in range(n)]
    out = defaultdict(int)

    def walk(pos, v, start):
        if pos == n - 1:
            out[(start, v)] += 1
            return
        for w in adj[pos][v]:
            if ok[pos + 1][w]:
                walk(pos + 1, w, start)

    for u in range(hin.counts[types[0]]):
        if ok[0][u]:
            walk(0, u, u)
    return dict(out)
