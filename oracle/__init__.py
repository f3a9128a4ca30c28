"""CPU oracle for constrained metapath queries -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the CPU-baseline
leg of ``bench.py`` may import this package.  It shares no code with the GPU
library (``paper_2201_04058_amd``) and neither imports the other.

What it computes (paper Sec. 2: Def. 1-3, Problem 1 and the constrained
adjacency matrices M_c * A defined with it):

    R = M_1 A_{r_1} M_2 A_{r_2} ... A_{r_{n-1}} M_n

R[u, v] = number of instances of the constrained metapath from u to v; the
MQE answer is every (u, v, R[u, v]) with R[u, v] >= 1, returned here as
canonical CSR (int64 row pointers, int32 columns ascending within each row,
no stored zeros, int64 counts).

Readings of the paper used here (the paper leaves them open):
  * every position may carry a constraint, the last one included; a
    constraint at position i is the 0/1 diagonal M_i on the nodes of o_i;
    several constraints at one position are ANDed;
  * a "range" constraint keeps lo <= v.prop <= hi (inclusive); an "idset"
    constraint keeps the listed node ids;
  * counts are exact integers; a final count >= 2^63 does not fit int64 and
    is reported as overflow (values are then saturated at 2^63).

Pins (tests/test_oracle_*.py): brute-force DFS enumeration of instances on
small random networks, scipy.sparse products, closed forms and invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
# ATP_ORACLE_LIBRARY names another build of oracle.c (the sanitizer build)
_LIB = os.environ.get("ATP_ORACLE_LIBRARY") or os.path.join(_HERE, "_liboracle.so")

ORC_OK, ORC_OVERFLOW, ORC_RANGE, ORC_NOMEM = 0, 1, 2, 3
SAT63 = 1 << 63


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (plain C, OpenMP for the row loop)."""
    if os.environ.get("ATP_ORACLE_LIBRARY"):
        return _LIB  # a build made elsewhere (build_sanitized)
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fopenmp", "-shared", "-fPIC",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


def build_sanitized(out: str, clang: str = "/opt/rocm/llvm/bin/clang") -> str:
    """oracle.c with AddressSanitizer and UndefinedBehaviorSanitizer (clang,
    the runtime of the library's sanitizer build; no OpenMP: one thread)."""
    tmp = out + f".tmp{os.getpid()}"
    subprocess.check_call([clang, "-O1", "-g", "-std=c11", "-shared", "-fPIC", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", _SRC, "-o", tmp])
    os.replace(tmp, out)
    return out


class _Result(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64),
                ("row_len", ctypes.POINTER(ctypes.c_int64)),
                ("nnz", ctypes.c_int64),
                ("col", ctypes.POINTER(ctypes.c_int32)),
                ("val", ctypes.POINTER(ctypes.c_uint64)),
                ("status", ctypes.c_int32)]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        lib.orc_chain_rows.restype = ctypes.c_int
        lib.orc_chain_rows.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_int64, ctypes.c_int, ctypes.POINTER(_Result)]
        lib.orc_spgemm.restype = ctypes.c_int
        lib.orc_spgemm.argtypes = [ctypes.c_int64, ctypes.c_int64] + [ctypes.c_void_p] * 6 + \
                                  [ctypes.POINTER(_Result)]
        lib.orc_free.argtypes = [ctypes.POINTER(_Result)]
        lib.orc_max_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _take(res: _Result) -> tuple:
    n = res.n_rows
    nnz = res.nnz
    row_len = np.ctypeslib.as_array(res.row_len, shape=(n,)).copy() if n else np.zeros(0, np.int64)
    col = np.ctypeslib.as_array(res.col, shape=(nnz,)).copy() if nnz else np.zeros(0, np.int32)
    val = np.ctypeslib.as_array(res.val, shape=(nnz,)).copy() if nnz else np.zeros(0, np.uint64)
    return row_len, col, val


# ---------------------------------------------------------------------------
# constraints -> diagonal masks (Def. 3 and the M_c matrices of Sec. 2)

def constraint_mask(hin, node_type: str, c) -> np.ndarray:
    """0/1 byte per node of ``node_type``: the diagonal of M_c."""
    n = hin.counts[node_type]
    if c.kind == "range":
        p = np.asarray(hin.props[(node_type, c.prop)]).astype(np.int64)
        return ((p >= c.lo) & (p <= c.hi)).astype(np.uint8)
    if c.kind == "idset":
        m = np.zeros(n, dtype=np.uint8)
        m[np.asarray(c.ids, dtype=np.int64)] = 1
        return m
    raise ValueError(c.kind)


def query_masks(hin, query) -> list:
    """One mask per position (None = unconstrained); constraints at the same
    position are ANDed."""
    masks = [None] * len(query.types)
    for c in query.constraints:
        m = constraint_mask(hin, query.types[c.position], c)
        masks[c.position] = m if masks[c.position] is None else (masks[c.position] & m)
    return masks


def _chain_arrays(hin, query, rel_list=None):
    types = query.types
    rels = rel_list if rel_list is not None else \
        [hin.rel(types[i], types[i + 1]) for i in range(len(types) - 1)]
    dims = np.array([hin.counts[t] for t in types], dtype=np.int64)
    rps = [np.ascontiguousarray(r.row_ptr, dtype=np.int64) for r in rels]
    cols = [np.ascontiguousarray(r.col, dtype=np.int32) for r in rels]
    return dims, rps, cols


def eval_rows(hin, query, rows, nthreads: int = 1, masks=None) -> tuple:
    """Rows ``rows`` of R as (row_len int64[len(rows)], col int32, val uint64,
    status).  ``status`` is ORC_OK or ORC_OVERFLOW."""
    lib = _load()
    dims, rps, cols = _chain_arrays(hin, query)
    masks = query_masks(hin, query) if masks is None else masks
    n = len(query.types)
    rp_arr = (ctypes.c_void_p * (n - 1))(*[_ptr(a) for a in rps])
    col_arr = (ctypes.c_void_p * (n - 1))(*[_ptr(a) for a in cols])
    mk = [None if m is None else np.ascontiguousarray(m, dtype=np.uint8) for m in masks]
    mk_arr = (ctypes.c_void_p * n)(*[None if m is None else _ptr(m) for m in mk])
    rows = np.ascontiguousarray(rows, dtype=np.int64)
    res = _Result()
    st = lib.orc_chain_rows(n, _ptr(dims), ctypes.addressof(rp_arr), ctypes.addressof(col_arr),
                            ctypes.addressof(mk_arr), _ptr(rows), rows.shape[0], int(nthreads),
                            ctypes.byref(res))
    try:
        if st not in (ORC_OK, ORC_OVERFLOW):
            raise RuntimeError(f"oracle failed with status {st}")
        row_len, col, val = _take(res)
    finally:
        lib.orc_free(ctypes.byref(res))
    return row_len, col, val, st


def eval_full(hin, query, nthreads: int = 1, masks=None) -> tuple:
    """The whole |o_1| x |o_n| result: (row_ptr int64, col int32, val uint64,
    status)."""
    n0 = hin.counts[query.types[0]]
    row_len, col, val, st = eval_rows(hin, query, np.arange(n0, dtype=np.int64), nthreads, masks)
    row_ptr = np.zeros(n0 + 1, dtype=np.int64)
    np.cumsum(row_len, out=row_ptr[1:])
    return row_ptr, col, val, st


def spgemm(m: int, n: int, xrp, xcol, xval, yrp, ycol, yval) -> tuple:
    """Z = X * Y for CSR operands with optional int64 values (None = all 1).
    Returns (row_ptr, col, val uint64, status)."""
    lib = _load()
    xrp = np.ascontiguousarray(xrp, dtype=np.int64)
    xcol = np.ascontiguousarray(xcol, dtype=np.int32)
    yrp = np.ascontiguousarray(yrp, dtype=np.int64)
    ycol = np.ascontiguousarray(ycol, dtype=np.int32)
    xv = None if xval is None else np.ascontiguousarray(xval, dtype=np.int64)
    yv = None if yval is None else np.ascontiguousarray(yval, dtype=np.int64)
    res = _Result()
    st = lib.orc_spgemm(m, n, _ptr(xrp), _ptr(xcol), None if xv is None else _ptr(xv),
                        _ptr(yrp), _ptr(ycol), None if yv is None else _ptr(yv), ctypes.byref(res))
    try:
        if st not in (ORC_OK, ORC_OVERFLOW):
            raise RuntimeError(f"oracle failed with status {st}")
        row_len, col, val = _take(res)
    finally:
        lib.orc_free(ctypes.byref(res))
    rp = np.zeros(m + 1, dtype=np.int64)
    np.cumsum(row_len, out=rp[1:])
    return rp, col, val, st


def max_threads() -> int:
    return int(_load().orc_max_threads())
