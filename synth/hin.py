"""Seeded synthetic heterogeneous information networks (HINs).

This module only *draws inputs*: node counts, typed edges, property columns
and constraint specifications.  It holds none of the path-count arithmetic;
both the CPU oracle and the GPU library receive the same arrays from here.

Data model (paper Sec. 2, Def. 1 and the adjacency-matrix paragraph that
follows it): each node type has a count; every node is identified by its
index inside its type; each edge type between two node types is a 0/1
adjacency matrix, stored as CSR with int64 row pointers and int32 column
indices sorted ascending within each row.  Both directions of a relation are
stored; the reverse is the exact transpose.

Generation rules (fixed, so every consumer sees identical bytes):
  * RNG: numpy ``default_rng(seed)`` (PCG64).  Draw order: one rank->id
    permutation per node type (declared order), then relations (declared
    order), then property columns, then query constraints (query order).
  * Zipf(s) over N items: P(rank r) proportional to r**-s for r = 1..N, drawn
    by inverse-CDF search on float64 cumulative weights; rank r is mapped to
    a node id through the type's permutation so hubs are scattered.
  * Each source node draws k targets with k capped at N; duplicate targets of
    one source are redrawn (first occurrence kept) until all k are distinct.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class Relation:
    src: str
    dst: str
    row_ptr: np.ndarray  # int64[n_src + 1]
    col: np.ndarray      # int32[nnz], ascending within each row

    @property
    def nnz(self) -> int:
        return int(self.col.shape[0])

    @property
    def n_rows(self) -> int:
        return int(self.row_ptr.shape[0] - 1)


@dataclass
class HIN:
    counts: dict                                     # type -> node count (ordered)
    relations: dict = field(default_factory=dict)    # (src, dst) -> Relation
    props: dict = field(default_factory=dict)        # (type, name) -> ndarray

    def rel(self, src: str, dst: str) -> Relation:
        return self.relations[(src, dst)]


@dataclass
class Constraint:
    """One per-position constraint of a constrained metapath (Def. 3).

    kind "range": lo <= prop[v] <= hi (inclusive) on property ``prop``.
    kind "idset": v is one of ``ids`` (sorted, unique int32 node ids).
    ``position`` is 0-based within the metapath's type sequence.
    """
    position: int
    kind: str
    prop: str | None = None
    lo: int = 0
    hi: int = 0
    ids: np.ndarray | None = None


@dataclass
class Query:
    name: str
    types: list
    constraints: list


class ZipfSampler:
    """Inverse-CDF Zipf(s) sampler over ranks 0..n-1 (rank 0 = most likely)."""

    def __init__(self, n: int, s: float):
        w = np.arange(1, n + 1, dtype=np.float64) ** (-float(s))
        cdf = np.cumsum(w)
        cdf /= cdf[-1]
        self.cdf = cdf
        self.n = n

    def __call__(self, rng: np.random.Generator, size: int) -> np.ndarray:
        u = rng.random(size)
        r = np.searchsorted(self.cdf, u, side="right")
        return np.minimum(r, self.n - 1).astype(np.int64)


class UniformSampler:
    def __init__(self, n: int):
        self.n = n

    def __call__(self, rng: np.random.Generator, size: int) -> np.ndarray:
        return rng.integers(0, self.n, size=size, dtype=np.int64)


def _segment_positions(starts: np.ndarray, lens: np.ndarray) -> np.ndarray:
    """Concatenation of arange(starts[i], starts[i]+lens[i])."""
    total = int(lens.sum())
    if total == 0:
        return np.zeros(0, dtype=np.int64)
    seg_begin = np.repeat(np.cumsum(lens) - lens, lens)
    return np.repeat(starts, lens) + (np.arange(total, dtype=np.int64) - seg_begin)


def draw_distinct_targets(rng, counts: np.ndarray, n_dst: int, sampler) -> tuple:
    """Per source i draw counts[i] (capped at n_dst) distinct target ranks.

    Returns (src, dst_rank) int64 arrays, grouped by source in source order.
    """
    counts = np.minimum(counts.astype(np.int64), n_dst)
    n_src = counts.shape[0]
    total = int(counts.sum())
    src = np.repeat(np.arange(n_src, dtype=np.int64), counts)
    dst = sampler(rng, total)
    off = np.zeros(n_src + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    check = np.arange(total, dtype=np.int64)
    while check.size:
        key = src[check] * n_dst + dst[check]
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = ks[1:] == ks[:-1]
        if not dup.any():
            break
        bad = np.sort(check[order[1:][dup]])
        dst[bad] = sampler(rng, bad.size)
        dirty = np.unique(src[bad])
        check = _segment_positions(off[dirty], counts[dirty])
    return src, dst


def csr_from_pairs(src: np.ndarray, dst: np.ndarray, n_src: int, n_dst: int) -> Relation:
    """Build a CSR 0/1 matrix from unique (src, dst) pairs."""
    key = src.astype(np.int64) * np.int64(n_dst) + dst.astype(np.int64)
    order = np.argsort(key, kind="stable")
    s = src[order]
    d = dst[order]
    row_ptr = np.zeros(n_src + 1, dtype=np.int64)
    if s.size:
        np.cumsum(np.bincount(s, minlength=n_src), out=row_ptr[1:])
    return row_ptr, d.astype(np.int32)


def add_bipartite(hin: HIN, a: str, b: str, src: np.ndarray, dst: np.ndarray) -> None:
    """Store relation a->b and its exact transpose b->a from pairs (a_id, b_id)."""
    na, nb = hin.counts[a], hin.counts[b]
    rp, c = csr_from_pairs(src, dst, na, nb)
    hin.relations[(a, b)] = Relation(a, b, rp, c)
    rp2, c2 = csr_from_pairs(dst, src, nb, na)
    hin.relations[(b, a)] = Relation(b, a, rp2, c2)


def schema_neighbours(hin: HIN, t: str) -> list:
    return sorted({d for (s, d) in hin.relations if s == t})
