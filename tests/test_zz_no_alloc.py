"""The allocation-free entry point atp_eval_noalloc (for callers that cannot
allocate device memory): called through the C-ABI twice in a row, the second
time on a smaller input, its result equals atp_eval's and the oracle's;
output arrays that are too small and queries larger than the static
workspace fail with their documented statuses and leave the context usable."""
import ctypes

import numpy as np
import pytest

from synth import configs
from synth.hin import HIN, Constraint, Query, Relation

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def atp():
    import paper_2201_04058_amd as atp
    atp.lib()
    return atp


class _Hip:
    """The caller's own device arrays, through the HIP runtime (the caller
    may allocate; the entry point under test does not)."""

    def __init__(self):
        self.rt = ctypes.CDLL("libamdhip64.so.7")  # the runtime the library links
        self.rt.hipMalloc.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_size_t]
        self.rt.hipFree.argtypes = [ctypes.c_void_p]
        self.rt.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        self.rt.hipDeviceSynchronize.argtypes = []

    def array(self, host: np.ndarray) -> int:
        p = ctypes.c_void_p()
        assert self.rt.hipMalloc(ctypes.byref(p), max(host.nbytes, 1)) == 0
        assert self.rt.hipMemcpy(p, host.ctypes.data, host.nbytes, 1) == 0  # host to device
        return p.value

    def fetch(self, ptr: int, like: np.ndarray) -> np.ndarray:
        out = np.empty_like(like)
        assert self.rt.hipMemcpy(out.ctypes.data, ptr, out.nbytes, 2) == 0  # device to host
        return out

    def free(self, *ptrs) -> None:
        for p in ptrs:
            assert self.rt.hipFree(ctypes.c_void_p(p)) == 0


@pytest.fixture(scope="module")
def hip(atp):
    return _Hip()


def _noalloc(ctx, hip, q, n_rows, cap, plan=None):
    """One call into caller-owned device arrays pre-filled with -7."""
    h_rp = np.full(n_rows + 1, -7, np.int64)
    h_col = np.full(max(cap, 1), -7, np.int32)
    h_val = np.full(max(cap, 1), -7, np.int64)
    rp, col, val = hip.array(h_rp), hip.array(h_col), hip.array(h_val)
    try:
        nnz = ctx.eval_noalloc(q, rp, col, val, cap, plan=plan)
        return nnz, hip.fetch(rp, h_rp), hip.fetch(col, h_col), hip.fetch(val, h_val)
    finally:
        hip.free(rp, col, val)


def test_noalloc_equals_eval_twice_then_smaller(atp, hip, oracle_mod, tiny_cfg):
    hin, qs = tiny_cfg
    q = qs[0]
    n0 = hin.counts[q.types[0]]
    rng = np.random.default_rng(31)
    small = Query(q.name, q.types, q.constraints +
                  [Constraint(0, "idset", ids=np.sort(rng.choice(n0, 60, replace=False)).astype(np.int32))])
    with atp.Context(device=0) as ctx:
        ctx.load_hin(hin)
        for z, query in enumerate([q, small]):
            ref = ctx.eval_query(query)
            erp, ecol, eval_ = ref.to_host()
            ref.free()
            orp, ocol, oval, st = oracle_mod.eval_full(hin, query)
            assert st == oracle_mod.ORC_OK
            cap = len(ecol) + 17
            nnz, rp, col, val = _noalloc(ctx, hip, query, n0, cap)
            assert nnz == len(ecol) == len(ocol), z
            assert np.array_equal(rp, erp) and np.array_equal(rp, orp), z
            assert np.array_equal(col[:nnz], ecol) and np.array_equal(col[:nnz], ocol), z
            assert np.array_equal(val[:nnz], eval_) and np.array_equal(val[:nnz], oval.astype(np.int64)), z
            assert np.all(col[nnz:] == -7) and np.all(val[nnz:] == -7), "wrote past the result"
        assert len(ocol) < len(ecol) or z == 1


def test_noalloc_every_plan_and_errors(atp, hip, oracle_mod, tiny_cfg):
    hin, qs = tiny_cfg
    q = qs[0]
    n0 = hin.counts[q.types[0]]
    orp, ocol, oval, _ = oracle_mod.eval_full(hin, q)
    with atp.Context(device=0) as ctx:
        ctx.load_hin(hin)
        for plan in ["(((0,1),2),3)", "(0,(1,(2,3)))", "((0,1),(2,3))"]:
            nnz, rp, col, val = _noalloc(ctx, hip, q, n0, len(ocol), plan=plan)
            assert np.array_equal(rp, orp) and np.array_equal(col[:nnz], ocol), plan
            assert np.array_equal(val[:nnz], oval.astype(np.int64)), plan
        # output arrays one entry short: ATP_EINVAL, the size needed is reported
        with pytest.raises(atp.AtpError) as e:
            _noalloc(ctx, hip, q, n0, len(ocol) - 1)
        assert e.value.status == atp.ATP_EINVAL and e.value.nnz == len(ocol)
        nnz, rp, col, val = _noalloc(ctx, hip, q, n0, len(ocol))
        assert np.array_equal(col[:nnz], ocol)


def test_noalloc_rejects_queries_beyond_the_workspace(atp, hip, oracle_mod):
    """A query whose temporaries exceed the static workspace returns
    ATP_EBUDGET; the context keeps working (both entry points)."""
    n = 1_500_000  # the per-row arrays of 750k start rows alone exceed the workspace
    hin = HIN(counts={"U": n, "W": 8})
    rp = np.arange(n + 1, dtype=np.int64)
    col = (np.arange(n) % 8).astype(np.int32)
    hin.relations[("U", "W")] = Relation("U", "W", rp, col)
    wt = np.zeros(8 + 1, np.int64)
    order = np.argsort(col, kind="stable").astype(np.int32)
    np.cumsum(np.bincount(col, minlength=8), out=wt[1:])
    hin.relations[("W", "U")] = Relation("W", "U", wt, order)
    big = Query("U-W-U", ["U", "W", "U"], [Constraint(0, "idset", ids=np.arange(0, n, 2, dtype=np.int32))])
    small = Query("U-W-U", ["U", "W", "U"], [Constraint(0, "idset", ids=np.array([5, 9], np.int32))])
    with atp.Context(device=0) as ctx:
        ctx.load_hin(hin)
        with pytest.raises(atp.AtpError) as e:
            _noalloc(ctx, hip, big, n, 16)
        assert e.value.status == atp.ATP_EBUDGET
        orp, ocol, oval, st = oracle_mod.eval_full(hin, small)
        assert st == oracle_mod.ORC_OK
        nnz, rp2, col2, val2 = _noalloc(ctx, hip, small, n, len(ocol))
        assert np.array_equal(rp2, orp) and np.array_equal(col2[:nnz], ocol)
        assert np.array_equal(val2[:nnz], oval.astype(np.int64))
        r = ctx.eval_query(small)
        grp, gcol, gval = r.to_host()
        r.free()
        assert np.array_equal(gcol, ocol) and np.array_equal(gval, oval.astype(np.int64))
