"""Small hand-built networks shared by several GPU test files."""
import numpy as np

from synth.hin import HIN, Query, Relation


def _csr_rel(hin, a, b, rows):
    """relation a->b from per-row sorted column lists"""
    rp = np.zeros(len(rows) + 1, np.int64)
    np.cumsum([len(r) for r in rows], out=rp[1:])
    col = np.concatenate([np.asarray(r, np.int32) for r in rows]) if rows else np.zeros(0, np.int32)
    hin.relations[(a, b)] = Relation(a, b, rp, col.astype(np.int32))


def _narrow_and_wide(n_wide_layers=10, width=128):
    """L0 (1 node) -> L1..Lk (node 0 = a narrow lane, nodes 1..width = a wide
    lane of complete bipartite layers) -> L_{k+1} (1 node).  The start only
    enters the narrow lane, so R = [[1]], but suffix products reach width^(k-1)
    paths from every wide node."""
    k = n_wide_layers
    names = [f"L{i}" for i in range(k + 2)]
    counts = {names[0]: 1, names[-1]: 1}
    for i in range(1, k + 1):
        counts[names[i]] = width + 1
    hin = HIN(counts=counts)
    _csr_rel(hin, names[0], names[1], [[0]])
    wide = list(range(1, width + 1))
    for i in range(1, k):
        _csr_rel(hin, names[i], names[i + 1], [[0]] + [wide] * width)
    _csr_rel(hin, names[k], names[k + 1], [[0]] * (width + 1))
    return hin, Query("-".join(names), names, [])
