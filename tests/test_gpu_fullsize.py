"""Parity at the full workload sizes (scholarly: 4M authors / 6M papers;
news: 3M articles), in the configuration bench.py times (planner's plan,
one context, default pool).

For every query of both workloads:

* the whole result -- row pointers, columns and counts of every row -- is
  compared element by element with the CPU oracle (Problem 1 defines the
  whole matrix), the oracle running row-parallel on the host's cores;
* independently of both sides, row sums equal the right-to-left SpMV chain
  M_1 A_1 ... M_n 1 (numpy) and the CSR is canonical.
"""
import os

import numpy as np
import pytest

from synth import configs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

QUERIES = [("scholarly", i) for i in range(len(configs.QUERIES["scholarly"]))] + \
          [("news", i) for i in range(len(configs.QUERIES["news"]))]


@pytest.fixture(scope="module")
def atp():
    import paper_2201_04058_amd as atp
    atp.lib()
    return atp


_ctx = {}


@pytest.fixture(scope="module")
def workloads(atp):
    """One context per workload with the network loaded (as in bench.py)."""
    yield _ctx
    for hin, qs, ctx in _ctx.values():
        ctx.close()
    _ctx.clear()


def _get(atp, name):
    if name not in _ctx:
        hin, qs = configs.load(name)
        ctx = atp.Context(device=0)
        ctx.load_hin(hin)
        _ctx[name] = (hin, qs, ctx)
    return _ctx[name]


def host_threads() -> int:
    return max(1, min(len(os.sched_getaffinity(0)), 32))


def spmv_row_sums(hin, q, masks):
    x = np.ones(hin.counts[q.types[-1]], dtype=np.int64)
    if masks[-1] is not None:
        x = x * masks[-1]
    for i in range(len(q.types) - 2, -1, -1):
        r = hin.rel(q.types[i], q.types[i + 1])
        y = np.zeros(r.n_rows, dtype=np.int64)
        nz = np.diff(r.row_ptr) > 0
        if r.nnz:
            y[nz] = np.add.reduceat(x[r.col], r.row_ptr[:-1][nz])
        x = y if masks[i] is None else y * masks[i]
    return x


@pytest.mark.parametrize("name,qi", QUERIES, ids=[f"{n}-{configs.QUERIES[n][i]}" for n, i in QUERIES])
def test_full_size_query_equals_oracle(atp, oracle_mod, workloads, name, qi):
    hin, qs, ctx = _get(atp, name)
    q = qs[qi]
    res = ctx.eval_query(q)
    stats = res.stats()
    rp, col, val = res.to_host()
    res.free()
    n0, n1 = hin.counts[q.types[0]], hin.counts[q.types[-1]]
    # canonical CSR
    assert rp.shape == (n0 + 1,) and rp[0] == 0 and rp[-1] == len(col) == stats["nnz"]
    lens = np.diff(rp)
    assert np.all(lens >= 0)
    assert np.all((col >= 0) & (col < n1))
    assert np.all(val > 0)
    if len(col) > 1:
        d = np.diff(col.astype(np.int64))
        row_start = np.zeros(len(col), bool)
        row_start[rp[:-1][lens > 0]] = True
        assert np.all((d > 0) | row_start[1:]), "columns not strictly ascending within a row"
    # row sums against the SpMV chain (independent of both sides)
    masks = oracle_mod.query_masks(hin, q)
    sums = np.zeros(n0, dtype=np.int64)
    nz = lens > 0
    sums[nz] = np.add.reduceat(val, rp[:-1][nz])
    assert np.array_equal(sums, spmv_row_sums(hin, q, masks)), q.name
    # the whole result against the oracle
    orp, ocol, oval, st = oracle_mod.eval_full(hin, q, nthreads=host_threads(), masks=masks)
    assert st == oracle_mod.ORC_OK
    assert np.array_equal(rp, orp), f"{q.name}: row pointers"
    assert np.array_equal(col, ocol), f"{q.name}: columns"
    assert np.array_equal(val, oval.astype(np.int64)), f"{q.name}: counts"
    print(f"{name} {q.name}: plan {stats['plan']} nnz {stats['nnz']} n_op {stats['n_op']} "
          f"whole CSR equal to the oracle", flush=True)
