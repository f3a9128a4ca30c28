"""Parity at the full workload sizes (scholarly: 4M authors / 6M papers;
news: 3M articles), in the configuration bench.py times (planner's plan,
one context, default pool).

* sampled rows -- random non-empty rows, the heaviest row, rows that must be
  empty -- are compared element by element with the CPU oracle;
* every row: row sums equal the right-to-left SpMV chain M_1 A_1 ... M_n 1
  (numpy, independent of both sides), the CSR is canonical, and the set of
  non-empty rows is the set with a positive SpMV sum.
"""
import numpy as np
import pytest

from synth import configs

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


@pytest.fixture(scope="module")
def atp():
    import paper_2201_04058_amd as atp
    atp.lib()
    return atp


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


@pytest.mark.parametrize("name", ["scholarly", "news"])
def test_full_size_queries(atp, oracle_mod, name):
    hin, qs = configs.load(name)
    ctx = atp.Context(device=0)
    ctx.load_hin(hin)
    rng = np.random.default_rng(7)
    for q in qs:
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
        # every row: row sums against the SpMV chain
        masks = oracle_mod.query_masks(hin, q)
        sums = np.zeros(n0, dtype=np.int64)
        nz = lens > 0
        sums[nz] = np.add.reduceat(val, rp[:-1][nz])
        ref_sums = spmv_row_sums(hin, q, masks)
        assert np.array_equal(sums, ref_sums), q.name
        # sampled rows element by element
        nonempty = np.nonzero(lens)[0]
        start = [c for c in q.constraints if c.kind == "idset" and c.position == 0][0].ids
        empty_in_start = np.setdiff1d(start, nonempty)
        outside = np.setdiff1d(rng.choice(n0, size=8, replace=False), start)
        pick = list(rng.choice(nonempty, size=min(6, len(nonempty)), replace=False))
        pick.append(int(nonempty[np.argmax(lens[nonempty])]))
        pick += list(empty_in_start[:3]) + list(outside[:3])
        rows = np.unique(np.array(pick, dtype=np.int64))
        rl, ocol, oval, st = oracle_mod.eval_rows(hin, q, rows, nthreads=8)
        assert st == oracle_mod.ORC_OK
        off = np.concatenate([[0], np.cumsum(rl)])
        for z, u in enumerate(rows):
            g_c, g_v = col[rp[u]:rp[u + 1]], val[rp[u]:rp[u + 1]]
            o_c, o_v = ocol[off[z]:off[z + 1]], oval[off[z]:off[z + 1]]
            assert np.array_equal(g_c, o_c), f"{q.name} row {u} columns"
            assert np.array_equal(g_v, o_v.astype(np.int64)), f"{q.name} row {u} counts"
        print(f"{name} {q.name}: plan {stats['plan']} nnz {stats['nnz']} n_op {stats['n_op']} "
              f"rows checked {len(rows)}", flush=True)
    ctx.close()
