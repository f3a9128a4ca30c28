"""The synthetic workloads: HINs shaped like the paper's Scholarly and News
networks (Sec. 4.1, Tables 1-2) and their metapath queries.

  tiny      seed 0  A 3,000  P 2,000  V 40  T 120; one query A-P-T-P-A keeping
                    a seeded 10% of T.
  scholarly seed 1  A 4M  P 6M  V 10k  T 60k; P.year int16 in [1990, 2021];
                    queries A-P-V-P-A, A-P-T-P-A, V-P-T-P-V, T-P-A-P-T, each
                    with a seeded 1,000-node start set and P.year >= 2015 at
                    every P position.
  news      seed 2  D 3M  R 500k  O 200k  L 100k  H 2k; D.day int32 in
                    [0, 1095]; queries O-D-H-D-O, R-D-L-D-R, R-D-O-D-H-D-R,
                    each with a seeded 2,000-node start set and a 110-day
                    window (10% of D) at every D position.

Every network is a star around its core type (papers / articles): each core
node draws its neighbours of each other type independently.
"""
from __future__ import annotations

import hashlib
import json
import os

import numpy as np

from .hin import (HIN, Constraint, Query, UniformSampler, ZipfSampler,
                  add_bipartite, draw_distinct_targets)

# (other type, count law, lambda, target law, zipf s) in draw order
SPECS = {
    "tiny": dict(
        seed=0,
        types=[("A", 3000), ("P", 2000), ("V", 40), ("T", 120)],
        core="P",
        rels=[("V", "one", 0.0, "uniform", 0.0),
              ("A", "1+pois", 2.0, "zipf", 1.1),
              ("T", "1+pois", 1.5, "zipf", 1.0)],
        props=[],
    ),
    "scholarly": dict(
        seed=1,
        types=[("A", 4_000_000), ("P", 6_000_000), ("V", 10_000), ("T", 60_000)],
        core="P",
        rels=[("A", "1+pois", 2.5, "zipf", 1.05),
              ("T", "1+pois", 3.0, "zipf", 0.9),
              ("V", "one", 0.0, "zipf", 1.2)],
        props=[("P", "year", np.int16, 1990, 2021)],
    ),
    "news": dict(
        seed=2,
        types=[("D", 3_000_000), ("R", 500_000), ("O", 200_000), ("L", 100_000), ("H", 2_000)],
        core="D",
        rels=[("R", "pois", 3.0, "zipf", 1.1),
              ("O", "pois", 2.0, "zipf", 1.2),
              ("L", "pois", 2.0, "zipf", 1.3),
              ("H", "1+pois", 4.0, "zipf", 1.3)],
        props=[("D", "day", np.int32, 0, 1095)],
    ),
}

QUERIES = {
    "tiny": ["A-P-T-P-A"],
    "scholarly": ["A-P-V-P-A", "A-P-T-P-A", "V-P-T-P-V", "T-P-A-P-T"],
    "news": ["O-D-H-D-O", "R-D-L-D-R", "R-D-O-D-H-D-R"],
}


def _scaled_spec(name: str, scale: float) -> dict:
    spec = dict(SPECS[name])
    if scale != 1.0:
        spec["types"] = [(t, max(2, int(round(n * scale)))) for t, n in spec["types"]]
    return spec


def make_hin(name: str, scale: float = 1.0) -> tuple:
    """Return (HIN, rng) for a named network; ``rng`` continues the stream
    for the query constraints.  ``scale`` shrinks every node count (tests)."""
    spec = _scaled_spec(name, scale)
    rng = np.random.default_rng(spec["seed"])
    counts = dict(spec["types"])
    hin = HIN(counts=counts)
    perms = {t: rng.permutation(n).astype(np.int64) for t, n in spec["types"]}
    core = spec["core"]
    n_core = counts[core]
    for other, law, lam, tlaw, s in spec["rels"]:
        if law == "one":
            k = np.ones(n_core, dtype=np.int64)
        elif law == "1+pois":
            k = 1 + rng.poisson(lam, size=n_core).astype(np.int64)
        elif law == "pois":
            k = rng.poisson(lam, size=n_core).astype(np.int64)
        else:
            raise ValueError(law)
        n_o = counts[other]
        sampler = UniformSampler(n_o) if tlaw == "uniform" else ZipfSampler(n_o, s)
        src, rank = draw_distinct_targets(rng, k, n_o, sampler)
        dst = perms[other][rank]
        add_bipartite(hin, core, other, src, dst)
    for t, pname, dt, lo, hi in spec["props"]:
        hin.props[(t, pname)] = rng.integers(lo, hi + 1, size=counts[t]).astype(dt)
    return hin, rng


def make_queries(name: str, hin: HIN, rng: np.random.Generator) -> list:
    out = []
    for qs in QUERIES[name]:
        types = qs.split("-")
        cons = []
        if name == "tiny":
            n_t = hin.counts["T"]
            keep = np.sort(rng.choice(n_t, size=max(1, n_t // 10), replace=False)).astype(np.int32)
            for i, t in enumerate(types):
                if t == "T":
                    cons.append(Constraint(i, "idset", ids=keep))
        elif name == "scholarly":
            n0 = hin.counts[types[0]]
            start = np.sort(rng.choice(n0, size=min(1000, n0), replace=False)).astype(np.int32)
            cons.append(Constraint(0, "idset", ids=start))
            for i, t in enumerate(types):
                if t == "P":
                    cons.append(Constraint(i, "range", prop="year", lo=2015, hi=32767))
        elif name == "news":
            d0 = int(rng.integers(0, 1096 - 110 + 1))
            n0 = hin.counts[types[0]]
            start = np.sort(rng.choice(n0, size=min(2000, n0), replace=False)).astype(np.int32)
            cons.append(Constraint(0, "idset", ids=start))
            for i, t in enumerate(types):
                if t == "D":
                    cons.append(Constraint(i, "range", prop="day", lo=d0, hi=d0 + 109))
        out.append(Query(qs, types, cons))
    return out


# ---------------------------------------------------------------------------
# on-disk cache (plain .npy files + JSON manifest; nothing is unpickled)

def _cache_dir() -> str:
    return os.environ.get("ATP_SYNTH_CACHE", "/tmp/atp_synth_cache")


def load(name: str, scale: float = 1.0, use_cache: bool = True) -> tuple:
    """(HIN, [Query]) for a named workload, cached under $ATP_SYNTH_CACHE."""
    tag = f"{name}_s{scale:g}_v1"
    d = os.path.join(_cache_dir(), tag)
    man = os.path.join(d, "manifest.json")
    if use_cache and os.path.exists(man):
        return _read(d)
    hin, rng = make_hin(name, scale)
    qs = make_queries(name, hin, rng)
    if use_cache:
        _write(d, hin, qs)
    return hin, qs


def _write(d: str, hin: HIN, qs: list) -> None:
    tmp = d + f".tmp{os.getpid()}"
    os.makedirs(tmp, exist_ok=True)
    m = {"counts": list(hin.counts.items()), "relations": [], "props": [], "queries": []}
    for (s, t), r in hin.relations.items():
        base = f"rel_{s}_{t}"
        np.save(os.path.join(tmp, base + "_rp.npy"), r.row_ptr)
        np.save(os.path.join(tmp, base + "_col.npy"), r.col)
        m["relations"].append([s, t, base])
    for (t, p), v in hin.props.items():
        base = f"prop_{t}_{p}"
        np.save(os.path.join(tmp, base + ".npy"), v)
        m["props"].append([t, p, base])
    for qi, q in enumerate(qs):
        cl = []
        for ci, c in enumerate(q.constraints):
            e = {"position": c.position, "kind": c.kind, "prop": c.prop, "lo": int(c.lo), "hi": int(c.hi)}
            if c.ids is not None:
                base = f"q{qi}_c{ci}_ids"
                np.save(os.path.join(tmp, base + ".npy"), c.ids)
                e["ids"] = base
            cl.append(e)
        m["queries"].append({"name": q.name, "types": q.types, "constraints": cl})
    with open(os.path.join(tmp, "manifest.json"), "w") as f:
        json.dump(m, f)
    try:
        os.rename(tmp, d)
    except OSError:
        pass  # another process won the race; its copy is identical


def _read(d: str) -> tuple:
    with open(os.path.join(d, "manifest.json")) as f:
        m = json.load(f)
    hin = HIN(counts={t: int(n) for t, n in m["counts"]})
    from .hin import Relation
    for s, t, base in m["relations"]:
        rp = np.load(os.path.join(d, base + "_rp.npy"))
        col = np.load(os.path.join(d, base + "_col.npy"))
        hin.relations[(s, t)] = Relation(s, t, rp, col)
    for t, p, base in m["props"]:
        hin.props[(t, p)] = np.load(os.path.join(d, base + ".npy"))
    qs = []
    for q in m["queries"]:
        cl = []
        for e in q["constraints"]:
            ids = np.load(os.path.join(d, e["ids"] + ".npy")) if "ids" in e else None
            cl.append(Constraint(e["position"], e["kind"], e["prop"], e["lo"], e["hi"], ids))
        qs.append(Query(q["name"], q["types"], cl))
    return hin, qs


def digest(hin: HIN) -> str:
    """SHA-256 over every array of the network (stable identity of inputs)."""
    h = hashlib.sha256()
    for (s, t), r in sorted(hin.relations.items()):
        h.update(f"{s}>{t}".encode())
        h.update(r.row_ptr.tobytes())
        h.update(r.col.tobytes())
    for (t, p), v in sorted(hin.props.items()):
        h.update(f"{t}.{p}".encode())
        h.update(v.tobytes())
    return h.hexdigest()
