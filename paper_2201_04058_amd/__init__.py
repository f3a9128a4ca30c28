"""Python binding of libatrapos.so, the MI355X metapath query engine.

Argument marshalling only: every step of a query runs in the HIP library.
Names follow the C-ABI in include/atrapos.h.  Importing this package does not
touch the GPU; loading the library fails loudly if it has not been built.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ATP_LIBRARY names another build of the same library (the sanitizer build of
# build.py --sanitize); there is no fallback implementation
LIB_PATH = os.environ.get("ATP_LIBRARY") or os.path.join(_HERE, "libatrapos.so")

ATP_OK, ATP_EINVAL, ATP_ENOMEM, ATP_EOVERFLOW, ATP_ESCHEMA, ATP_EDEVICE, ATP_EBUDGET, ATP_ESTATE = \
    0, -1, -2, -3, -4, -5, -6, -7
ATP_OPT_PROFILE, ATP_OPT_PLAN_EAC, ATP_OPT_COUNT_BYTES, ATP_OPT_NO_RESTRICT, ATP_OPT_SERIAL_BINS = 1, 2, 4, 8, 16
ATP_REL_DEVICE_PTRS, ATP_REL_ADD_REVERSE = 1, 2
ATP_I16, ATP_I32, ATP_I64 = 1, 2, 3
ATP_C_RANGE, ATP_C_IDSET = 1, 2

EXPORTS = [
    "atp_create", "atp_destroy", "atp_add_node_type", "atp_add_relation", "atp_add_property",
    "atp_eval", "atp_eval_plan", "atp_eval_noalloc", "atp_result_csr", "atp_result_to_host", "atp_result_stats",
    "atp_result_free", "atp_plan_chain", "atp_set_flags", "atp_kernel_times", "atp_kernel_times_reset",
    "atp_set_profile_kernel",
    "atp_device_bytes", "atp_status_str", "atp_cache_configure", "atp_cache_get_stats", "atp_otree_create",
    "atp_otree_destroy", "atp_otree_insert", "atp_otree_frequency", "atp_otree_shape", "atp_cache_simulate",
    "atp_eval_batch", "atp_server_start", "atp_submit", "atp_poll", "atp_server_pending", "atp_server_stop",
    "atp_get_tuning", "atp_set_tuning", "atp_autotune", "atp_cost_fit", "atp_get_cost_model", "atp_set_cost_model",
    "atp_calibrate_cost_model",
]
TUNABLES = ("part_target", "part_hash_cap", "task_ops", "bucket_pct", "split_ops", "bucket_chunk")
ATP_CACHE_OFF, ATP_CACHE_OTREE, ATP_CACHE_PGDS, ATP_CACHE_LRU, ATP_CACHE_CBS1, ATP_CACHE_CBS2 = 0, 1, 2, 3, 4, 5


class AtpError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        super().__init__(f"{where}: {status_str(status)} ({status})")


class atp_options(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int),
                ("hip_stream", ctypes.c_void_p),
                ("alloc", ctypes.c_void_p),
                ("free", ctypes.c_void_p),
                ("alloc_user", ctypes.c_void_p),
                ("mem_budget_bytes", ctypes.c_uint64),
                ("flags", ctypes.c_uint32)]


class atp_constraint(ctypes.Structure):
    _fields_ = [("position", ctypes.c_int32),
                ("kind", ctypes.c_int32),
                ("prop_id", ctypes.c_int32),
                ("lo", ctypes.c_int64),
                ("hi", ctypes.c_int64),
                ("ids", ctypes.c_void_p),
                ("n_ids", ctypes.c_int64)]


class atp_cache_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("queries", "whole_hits", "sub_hits", "insert_attempts", "inserts",
                                              "evictions", "items", "bytes", "otree_nodes", "otree_leaves")]


class atp_query(ctypes.Structure):
    _fields_ = [("types", ctypes.c_void_p),
                ("n_types", ctypes.c_int32),
                ("rel_ids", ctypes.c_void_p),
                ("cons", ctypes.c_void_p),
                ("n_cons", ctypes.c_int32)]


class atp_server_options(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_int32),
                ("max_batch", ctypes.c_int32),
                ("mem_budget_bytes", ctypes.c_uint64)]


class atp_completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64),
                ("status", ctypes.c_int32),
                ("result", ctypes.c_void_p),
                ("t_submit", ctypes.c_double),
                ("t_start", ctypes.c_double),
                ("t_done", ctypes.c_double),
                ("batch_size", ctypes.c_int32),
                ("lane", ctypes.c_int32)]


class atp_tuning(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in TUNABLES]


class atp_eval_stats(ctypes.Structure):
    _fields_ = [("n_products", ctypes.c_int32),
                ("n_op_total", ctypes.c_int64),
                ("nnz_intermediate_total", ctypes.c_int64),
                ("nnz_result", ctypes.c_int64),
                ("slots_total", ctypes.c_int64)]


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library; raises if libatrapos.so was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2201_04058_amd.build` "
                          "or __graft_entry__.build(); there is no fallback implementation")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
    P = ctypes.POINTER
    sig = {
        "atp_create": ([vp, P(vp)], i32),
        "atp_destroy": ([vp], i32),
        "atp_add_node_type": ([vp, ctypes.c_char_p, i64, P(i32)], i32),
        "atp_add_relation": ([vp, i32, i32, vp, vp, i64, u32, P(i32)], i32),
        "atp_add_property": ([vp, i32, ctypes.c_char_p, i32, vp, P(i32)], i32),
        "atp_eval": ([vp, vp, i32, vp, vp, i32, P(vp)], i32),
        "atp_eval_plan": ([vp, vp, i32, vp, vp, i32, ctypes.c_char_p, P(vp)], i32),
        "atp_eval_noalloc": ([vp, vp, i32, vp, vp, i32, ctypes.c_char_p, vp, vp, vp, i64, P(i64)], i32),
        "atp_result_csr": ([vp, P(i64), P(i64), P(i64), P(vp), P(vp), P(vp)], i32),
        "atp_result_to_host": ([vp, vp, vp, vp], i32),
        "atp_result_stats": ([vp, P(atp_eval_stats), ctypes.c_char_p, ctypes.c_size_t], i32),
        "atp_result_free": ([vp], i32),
        "atp_plan_chain": ([i32, vp, vp, ctypes.c_double, ctypes.c_double, ctypes.c_double, i32,
                            ctypes.c_char_p, ctypes.c_size_t, P(ctypes.c_double)], i32),
        "atp_set_flags": ([vp, u32], i32),
        "atp_kernel_times": ([vp, P(ctypes.c_char_p), P(ctypes.c_double), P(i64), P(ctypes.c_double), i32], i32),
        "atp_kernel_times_reset": ([vp], None),
        "atp_set_profile_kernel": ([vp, ctypes.c_char_p], ctypes.c_int32),
        "atp_device_bytes": ([vp], i64),
        "atp_status_str": ([i32], ctypes.c_char_p),
        "atp_cache_configure": ([vp, i32, ctypes.c_uint64], i32),
        "atp_cache_get_stats": ([vp, P(atp_cache_stats)], i32),
        "atp_otree_create": ([P(vp)], i32),
        "atp_otree_destroy": ([vp], i32),
        "atp_otree_insert": ([vp, vp, i32], i32),
        "atp_otree_frequency": ([vp, vp, i32, P(i64)], i32),
        "atp_otree_shape": ([vp, P(i64), P(i64), P(i64), P(i64), P(i64)], i32),
        "atp_cache_simulate": ([i32, ctypes.c_double, i32, vp, vp, vp, i32, vp, vp, vp, vp], i32),
        "atp_eval_batch": ([vp, vp, i32, i32, i32, ctypes.c_uint64, vp, vp], i32),
        "atp_server_start": ([vp, P(atp_server_options)], i32),
        "atp_submit": ([vp, P(atp_query), ctypes.c_uint64], i32),
        "atp_poll": ([vp, vp, i32, i32], i32),
        "atp_server_pending": ([vp], i32),
        "atp_server_stop": ([vp], i32),
        "atp_get_tuning": ([vp, P(atp_tuning)], i32),
        "atp_set_tuning": ([vp, P(atp_tuning)], i32),
        "atp_autotune": ([vp, vp, i32, i32, P(atp_tuning), P(ctypes.c_double), P(ctypes.c_double)], i32),
        "atp_cost_fit": ([i32, vp, vp, vp, vp, vp, P(ctypes.c_double)], i32),
        "atp_get_cost_model": ([vp, vp], i32),
        "atp_set_cost_model": ([vp, vp], i32),
        "atp_calibrate_cost_model": ([vp, vp, i32, vp, P(ctypes.c_double), P(i32)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    return L


def status_str(st: int) -> str:
    return lib().atp_status_str(st).decode()


def _check(st: int, where: str) -> None:
    if st != ATP_OK:
        raise AtpError(st, where)


def plan_chain(dims, nnz=None, alpha=12.0, beta=12.0, gamma=12.0, dense=False) -> tuple:
    """Host-only DP planner (Eq. 1) -> (plan string, cost)."""
    dims = np.ascontiguousarray(dims, dtype=np.int64)
    p = dims.shape[0] - 1
    nz = None if nnz is None else np.ascontiguousarray(nnz, dtype=np.int64)
    buf = ctypes.create_string_buffer(4096)
    cost = ctypes.c_double()
    st = lib().atp_plan_chain(p, dims.ctypes.data, None if nz is None else nz.ctypes.data, alpha, beta, gamma,
                              1 if dense else 0, buf, 4096, ctypes.byref(cost))
    _check(st, "atp_plan_chain")
    return buf.value.decode(), cost.value


class OverlapTree:
    """Standalone Overlap Tree (host only)."""

    def __init__(self):
        h = ctypes.c_void_p()
        _check(lib().atp_otree_create(ctypes.byref(h)), "atp_otree_create")
        self._h = h

    def insert(self, symbols) -> None:
        a = np.ascontiguousarray(symbols, dtype=np.int32)
        _check(lib().atp_otree_insert(self._h, a.ctypes.data, a.shape[0]), "atp_otree_insert")

    def frequency(self, symbols) -> int:
        a = np.ascontiguousarray(symbols, dtype=np.int32)
        f = ctypes.c_int64()
        _check(lib().atp_otree_frequency(self._h, a.ctypes.data if a.size else None, a.shape[0], ctypes.byref(f)),
               "atp_otree_frequency")
        return f.value

    def shape(self) -> dict:
        v = [ctypes.c_int64() for _ in range(5)]
        _check(lib().atp_otree_shape(self._h, *[ctypes.byref(x) for x in v]), "atp_otree_shape")
        return dict(zip(("nodes", "leaves", "lambda", "thin_internal", "leaves_f_not_1"), [x.value for x in v]))

    def __del__(self):
        try:
            lib().atp_otree_destroy(self._h)
        except Exception:
            pass


def cache_simulate(policy: int, budget: float, sizes, costs, parents, requests) -> tuple:
    """Replay requests through a cache policy (host only): (hit, cached_after, final_cached)."""
    sz = np.ascontiguousarray(sizes, dtype=np.float64)
    co = np.ascontiguousarray(costs, dtype=np.float64)
    pa = np.ascontiguousarray(parents, dtype=np.int32)
    rq = np.ascontiguousarray(requests, dtype=np.int32)
    hit = np.zeros(len(rq), np.int32)
    after = np.zeros(len(rq), np.int32)
    fin = np.zeros(len(sz), np.int32)
    _check(lib().atp_cache_simulate(policy, float(budget), len(sz), sz.ctypes.data, co.ctypes.data, pa.ctypes.data,
                                    len(rq), rq.ctypes.data, hit.ctypes.data, after.ctypes.data, fin.ctypes.data),
           "atp_cache_simulate")
    return hit.astype(bool), after.astype(bool), fin.astype(bool)


def cost_fit(nnz_x, n_op, nnz_z, t_ms) -> tuple:
    """Host-only fit of Eq. 2's coefficients -> ((alpha, beta, gamma, delta), r2)."""
    cols = [np.ascontiguousarray(v, dtype=np.float64) for v in (nnz_x, n_op, nnz_z, t_ms)]
    out = (ctypes.c_double * 4)()
    r2 = ctypes.c_double()
    _check(lib().atp_cost_fit(len(cols[3]), *[c.ctypes.data for c in cols], out, ctypes.byref(r2)), "atp_cost_fit")
    return tuple(out), r2.value


def torch_stream_handle(device: int = 0) -> int | None:
    """The HIP stream torch currently issues work on (None = default stream)."""
    import torch
    return torch.cuda.current_stream(device).cuda_stream or None


class Result:
    def __init__(self, ctx: "Context", handle: int):
        self._ctx = ctx
        self._h = ctypes.c_void_p(handle)

    def shape(self) -> tuple:
        r, c, z = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        _check(lib().atp_result_csr(self._h, ctypes.byref(r), ctypes.byref(c), ctypes.byref(z), None, None, None),
               "atp_result_csr")
        return r.value, c.value, z.value

    def device_ptrs(self) -> tuple:
        rp, col, val = ctypes.c_void_p(), ctypes.c_void_p(), ctypes.c_void_p()
        _check(lib().atp_result_csr(self._h, None, None, None, ctypes.byref(rp), ctypes.byref(col),
                                    ctypes.byref(val)), "atp_result_csr")
        return rp.value, col.value, val.value

    def to_host(self) -> tuple:
        n_rows, _, nnz = self.shape()
        rp = np.empty(n_rows + 1, dtype=np.int64)
        col = np.empty(max(nnz, 0), dtype=np.int32)
        val = np.empty(max(nnz, 0), dtype=np.int64)
        _check(lib().atp_result_to_host(self._h, rp.ctypes.data, col.ctypes.data if nnz else None,
                                        val.ctypes.data if nnz else None), "atp_result_to_host")
        return rp, col, val

    def stats(self) -> dict:
        s = atp_eval_stats()
        buf = ctypes.create_string_buffer(4096)
        _check(lib().atp_result_stats(self._h, ctypes.byref(s), buf, 4096), "atp_result_stats")
        return {"plan": buf.value.decode(), "n_products": s.n_products, "n_op": s.n_op_total,
                "nnz_intermediate": s.nnz_intermediate_total, "nnz": s.nnz_result, "slots": s.slots_total}

    def free(self) -> None:
        if self._h and self._h.value:
            lib().atp_result_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            if self._ctx._h.value:
                self.free()
        except Exception:
            pass


class Context:
    """One engine context (device, stream, memory pool, registered network)."""

    def __init__(self, device: int = 0, stream: int | None = None, budget_bytes: int = 0,
                 profile: bool = False, plan_eac: bool = False, no_restrict: bool = False):
        o = atp_options()
        o.device = device
        o.hip_stream = stream
        o.mem_budget_bytes = budget_bytes
        o.flags = (ATP_OPT_PROFILE if profile else 0) | (ATP_OPT_PLAN_EAC if plan_eac else 0) | \
            (ATP_OPT_NO_RESTRICT if no_restrict else 0)
        h = ctypes.c_void_p()
        _check(lib().atp_create(ctypes.byref(o), ctypes.byref(h)), "atp_create")
        self._h = h
        self.type_ids: dict = {}
        self.prop_ids: dict = {}
        self.rel_ids: dict = {}

    def close(self) -> None:
        if self._h.value:
            lib().atp_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- network ---------------------------------------------------------
    def add_node_type(self, name: str, count: int) -> int:
        tid = ctypes.c_int32()
        _check(lib().atp_add_node_type(self._h, name.encode(), int(count), ctypes.byref(tid)), "atp_add_node_type")
        self.type_ids[name] = tid.value
        return tid.value

    def add_relation(self, src: int, dst: int, row_ptr, col, reverse: bool = False) -> int:
        rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
        cl = np.ascontiguousarray(col, dtype=np.int32)
        rid = ctypes.c_int32()
        flags = ATP_REL_ADD_REVERSE if reverse else 0
        _check(lib().atp_add_relation(self._h, src, dst, rp.ctypes.data, cl.ctypes.data if cl.size else None,
                                      cl.shape[0], flags, ctypes.byref(rid)), "atp_add_relation")
        return rid.value

    def add_property(self, type_id: int, name: str, values) -> int:
        v = np.ascontiguousarray(values)
        dt = {np.dtype(np.int16): ATP_I16, np.dtype(np.int32): ATP_I32, np.dtype(np.int64): ATP_I64}[v.dtype]
        pid = ctypes.c_int32()
        _check(lib().atp_add_property(self._h, type_id, name.encode(), dt, v.ctypes.data if v.size else None,
                                      ctypes.byref(pid)), "atp_add_property")
        return pid.value

    def load_hin(self, hin) -> None:
        """Register every node type, relation and property of a network object
        with ``counts``, ``relations`` ((src, dst) -> row_ptr/col) and ``props``."""
        for name, n in hin.counts.items():
            self.add_node_type(name, n)
        for (s, d), r in hin.relations.items():
            self.rel_ids[(s, d)] = self.add_relation(self.type_ids[s], self.type_ids[d], r.row_ptr, r.col)
        for (t, p), v in hin.props.items():
            self.prop_ids[(t, p)] = self.add_property(self.type_ids[t], p, v)

    # --- queries ---------------------------------------------------------
    def _constraints(self, types, constraints):
        arr = (atp_constraint * max(1, len(constraints)))()
        keep = []
        for z, c in enumerate(constraints):
            a = arr[z]
            a.position = c.position
            if c.kind == "range":
                a.kind = ATP_C_RANGE
                a.prop_id = self.prop_ids[(types[c.position], c.prop)]
                a.lo, a.hi = int(c.lo), int(c.hi)
            elif c.kind == "idset":
                ids = np.ascontiguousarray(c.ids, dtype=np.int32)
                keep.append(ids)
                a.kind = ATP_C_IDSET
                a.ids = ids.ctypes.data if ids.size else None
                a.n_ids = ids.shape[0]
            else:
                raise ValueError(c.kind)
        return arr, keep

    def eval(self, types, constraints=(), plan: str | None = None, rel_ids=None) -> Result:
        """Evaluate a constrained metapath given by type names (or ids)."""
        tids = np.array([self.type_ids[t] if isinstance(t, str) else int(t) for t in types], dtype=np.int32)
        names = [t if isinstance(t, str) else None for t in types]
        arr, keep = self._constraints(names, list(constraints))
        rids = None if rel_ids is None else np.ascontiguousarray(rel_ids, dtype=np.int32)
        h = ctypes.c_void_p()
        if plan is None:
            st = lib().atp_eval(self._h, tids.ctypes.data, len(tids), None if rids is None else rids.ctypes.data,
                                arr, len(constraints), ctypes.byref(h))
        else:
            st = lib().atp_eval_plan(self._h, tids.ctypes.data, len(tids),
                                     None if rids is None else rids.ctypes.data, arr, len(constraints),
                                     plan.encode(), ctypes.byref(h))
        del keep
        _check(st, "atp_eval")
        return Result(self, h.value)

    def eval_query(self, query, plan: str | None = None) -> Result:
        return self.eval(query.types, query.constraints, plan=plan)

    def eval_noalloc(self, query, row_ptr: int, col: int, val: int, cap: int, plan: str | None = None) -> int:
        """atp_eval_noalloc: the result into caller-owned device arrays (device
        addresses row_ptr, col, val; col / val hold cap entries).  Returns the
        result's nonzero count; raises AtpError (status and, for a result
        larger than cap, the count needed as .nnz)."""
        tids = np.array([self.type_ids[t] if isinstance(t, str) else int(t) for t in query.types], dtype=np.int32)
        names = [t if isinstance(t, str) else None for t in query.types]
        arr, keep = self._constraints(names, list(query.constraints))
        nnz = ctypes.c_int64(-1)
        st = lib().atp_eval_noalloc(self._h, tids.ctypes.data, len(tids), None, arr, len(query.constraints),
                                    None if plan is None else plan.encode(), row_ptr, col, val, int(cap),
                                    ctypes.byref(nnz))
        del keep
        if st != ATP_OK:
            e = AtpError(st, "atp_eval_noalloc")
            e.nnz = nnz.value
            raise e
        return nnz.value

    def _query(self, query):
        """(atp_query, arrays it points to) for a query object with types / constraints."""
        tids = np.array([self.type_ids[t] if isinstance(t, str) else int(t) for t in query.types], dtype=np.int32)
        names = [t if isinstance(t, str) else None for t in query.types]
        arr, keep = self._constraints(names, list(query.constraints))
        q = atp_query()
        q.types = tids.ctypes.data
        q.n_types = len(tids)
        q.rel_ids = None
        q.cons = ctypes.addressof(arr)
        q.n_cons = len(query.constraints)
        return q, (tids, arr, keep)

    # --- batches and serving ---------------------------------------------
    def eval_batch(self, queries, lanes: int = 4, max_batch: int = 64, mem_budget_bytes: int = 0) -> list:
        """Evaluate a list of queries on `lanes` lanes, fusing queries that differ
        only in their start set.  Returns one Result or AtpError per query."""
        n = len(queries)
        qs = (atp_query * max(1, n))()
        keep = []
        for i, q in enumerate(queries):
            qs[i], k = self._query(q)
            keep.append(k)
        out = (ctypes.c_void_p * max(1, n))()
        st = (ctypes.c_int32 * max(1, n))()
        _check(lib().atp_eval_batch(self._h, qs, n, lanes, max_batch, int(mem_budget_bytes), out, st),
               "atp_eval_batch")
        del keep
        return [Result(self, out[i]) if st[i] == ATP_OK else AtpError(st[i], "atp_eval_batch")
                for i in range(n)]

    def server_start(self, lanes: int = 4, max_batch: int = 64, mem_budget_bytes: int = 0) -> None:
        o = atp_server_options(lanes, max_batch, int(mem_budget_bytes))
        _check(lib().atp_server_start(self._h, ctypes.byref(o)), "atp_server_start")

    def submit(self, query, tag: int) -> None:
        q, keep = self._query(query)
        _check(lib().atp_submit(self._h, ctypes.byref(q), int(tag)), "atp_submit")
        del keep

    def poll(self, max_n: int = 256, wait_ms: int = 0) -> list:
        """Finished requests: dicts with tag, status, result (Result or None),
        t_submit, t_start, t_done (s), batch, lane."""
        buf = (atp_completion * max(1, max_n))()
        k = lib().atp_poll(self._h, buf, max_n, int(wait_ms))
        if k < 0:
            raise AtpError(k, "atp_poll")
        out = []
        for z in range(k):
            c = buf[z]
            out.append({"tag": c.tag, "status": c.status, "result": Result(self, c.result) if c.result else None,
                        "t_submit": c.t_submit, "t_start": c.t_start, "t_done": c.t_done,
                        "batch": c.batch_size, "lane": c.lane})
        return out

    # --- kernel tunables ---------------------------------------------------
    def tuning(self) -> dict:
        t = atp_tuning()
        _check(lib().atp_get_tuning(self._h, ctypes.byref(t)), "atp_get_tuning")
        return {n: getattr(t, n) for n in TUNABLES}

    def set_tuning(self, **kw) -> None:
        cur = self.tuning()
        cur.update(kw)
        t = atp_tuning(*[int(cur[n]) for n in TUNABLES])
        _check(lib().atp_set_tuning(self._h, ctypes.byref(t)), "atp_set_tuning")

    def autotune(self, sample, rounds: int = 1) -> dict:
        """Coordinate-descent search of the tunables on a sample of queries;
        keeps the fastest setting.  Returns it with the sample's ms before/after."""
        n = len(sample)
        qs = (atp_query * max(1, n))()
        keep = []
        for i, q in enumerate(sample):
            qs[i], k = self._query(q)
            keep.append(k)
        t = atp_tuning()
        b, a = ctypes.c_double(), ctypes.c_double()
        _check(lib().atp_autotune(self._h, qs, n, rounds, ctypes.byref(t), ctypes.byref(b), ctypes.byref(a)),
               "atp_autotune")
        del keep
        out = {n_: getattr(t, n_) for n_ in TUNABLES}
        out.update({"ms_before": b.value, "ms_after": a.value})
        return out

    # --- cost model (Eq. 2) ---------------------------------------------------
    def cost_model(self) -> tuple:
        out = (ctypes.c_double * 4)()
        _check(lib().atp_get_cost_model(self._h, out), "atp_get_cost_model")
        return tuple(out)

    def set_cost_model(self, coeffs) -> None:
        c = (ctypes.c_double * 4)(*[float(x) for x in coeffs])
        _check(lib().atp_set_cost_model(self._h, c), "atp_set_cost_model")

    def calibrate_cost_model(self, sample) -> dict:
        """Time every multiplication of the sample, fit Eq. 2 and install the fit."""
        n = len(sample)
        qs = (atp_query * max(1, n))()
        keep = []
        for i, q in enumerate(sample):
            qs[i], k = self._query(q)
            keep.append(k)
        out = (ctypes.c_double * 4)()
        r2 = ctypes.c_double()
        np_ = ctypes.c_int32()
        _check(lib().atp_calibrate_cost_model(self._h, qs, n, out, ctypes.byref(r2), ctypes.byref(np_)),
               "atp_calibrate_cost_model")
        del keep
        return {"coeffs": tuple(out), "r2": r2.value, "products": np_.value}

    def server_pending(self) -> int:
        return int(lib().atp_server_pending(self._h))

    def server_stop(self) -> None:
        _check(lib().atp_server_stop(self._h), "atp_server_stop")

    # --- diagnostics -----------------------------------------------------
    def set_flags(self, profile: bool = False, plan_eac: bool = False, count_bytes: bool = False,
                  no_restrict: bool = False, serial_bins: bool = False) -> None:
        f = (ATP_OPT_PROFILE if profile else 0) | (ATP_OPT_PLAN_EAC if plan_eac else 0) | \
            (ATP_OPT_COUNT_BYTES if count_bytes else 0) | (ATP_OPT_NO_RESTRICT if no_restrict else 0) | \
            (ATP_OPT_SERIAL_BINS if serial_bins else 0)
        _check(lib().atp_set_flags(self._h, f), "atp_set_flags")

    def kernel_times(self) -> dict:
        """kernel name -> (total ms, launches, algorithmic bytes) since the last reset"""
        cap = 64
        names = (ctypes.c_char_p * cap)()
        ms = (ctypes.c_double * cap)()
        n = (ctypes.c_int64 * cap)()
        b = (ctypes.c_double * cap)()
        k = lib().atp_kernel_times(self._h, names, ms, n, b, cap)
        return {names[z].decode(): (ms[z], n[z], b[z]) for z in range(k)}

    def kernel_times_reset(self) -> None:
        lib().atp_kernel_times_reset(self._h)

    def set_profile_kernel(self, name: str | None) -> None:
        """Time only the launches of this kernel (None: every launch) under profile=True."""
        _check(lib().atp_set_profile_kernel(self._h, name.encode() if name else None), "atp_set_profile_kernel")

    def device_bytes(self) -> int:
        return int(lib().atp_device_bytes(self._h))

    # --- workload cache (Overlap Tree + replacement policy) ------------------
    def cache_configure(self, policy: int, budget_bytes: int) -> None:
        _check(lib().atp_cache_configure(self._h, int(policy), int(budget_bytes)), "atp_cache_configure")

    def cache_stats(self) -> dict:
        st = atp_cache_stats()
        _check(lib().atp_cache_get_stats(self._h, ctypes.byref(st)), "atp_cache_get_stats")
        return {n: getattr(st, n) for n, _ in atp_cache_stats._fields_}
