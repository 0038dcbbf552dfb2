"""Seeded synthetic inputs shared by the tests, the benchmark and the serving
driver.  Holds no eigensolver arithmetic: only matrix generators, value
rounding to a storage precision and small closed-form graphs.

Workload recipes (stand-ins for the paper's Table I graphs, which are not
shipped here):

* ``er(n, d, seed)``: Erdos-Renyi over the strict upper triangle with
  p = d/(n-1), mirrored; off-diagonal uniform(-1,1), diagonal uniform(0,1).
  With d = 9 the matrix has about 10 non-zeros per row including the diagonal.
* ``rmat(scale, edge_factor, ...)``: R-MAT with (a, b, c, d) =
  (0.57, 0.19, 0.19, 0.05), edge_factor * 2^scale directed draws, self loops
  dropped, undirected and deduplicated, uniform(0,1) weights per pair, vertex
  ids relabelled by a seeded permutation.
* ``normalize_sym``: D^{-1/2} A D^{-1/2} (symmetric, same spectrum as the
  row-normalised D^{-1} A).
* ``round_values``: round values once to the lowest storage precision of a
  comparison so that every run sees the same matrix.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.cpp")
_LIB = os.path.join(_HERE, "libsynth.so")
_lib = None


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P, i64, u64, f64, i32 = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64,
                                 ctypes.c_double, ctypes.c_int)
        lib.syn_er.restype = P
        lib.syn_er.argtypes = [i64, f64, u64]
        lib.syn_rmat.restype = P
        lib.syn_rmat.argtypes = [i64, i32, i64, f64, f64, f64, u64, i32]
        lib.syn_n.restype = i64
        lib.syn_n.argtypes = [P]
        lib.syn_nnz.restype = i64
        lib.syn_nnz.argtypes = [P]
        lib.syn_copy.restype = None
        lib.syn_copy.argtypes = [P, P, P, P]
        lib.syn_free.restype = None
        lib.syn_free.argtypes = [P]
        lib.syn_normalize_sym.restype = None
        lib.syn_normalize_sym.argtypes = [i64, P, P, P]
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _take(h):
    lib = _load()
    if not h:
        raise ValueError("generator rejected its arguments")
    try:
        n, nnz = lib.syn_n(h), lib.syn_nnz(h)
        rowptr = np.empty(n + 1, np.int64)
        col = np.empty(nnz, np.int32)
        val = np.empty(nnz, np.float64)
        lib.syn_copy(h, _p(rowptr), _p(col), _p(val))
    finally:
        lib.syn_free(h)
    return rowptr, col, val


def er(n: int, offdiag_per_row: float = 9.0, seed: int = 0):
    """Symmetric Erdos-Renyi matrix with a full diagonal (CSR, float64)."""
    return _take(_load().syn_er(int(n), float(offdiag_per_row), seed & (2 ** 64 - 1)))


def rmat(scale: int, edge_factor: float, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 0, n: int | None = None, permute: bool = True):
    """Symmetrised, deduplicated R-MAT graph with uniform(0,1) weights (CSR)."""
    nv = (1 << scale) if n is None else int(n)
    draws = int(round(edge_factor * nv))
    return _take(_load().syn_rmat(nv, int(scale), draws, a, b, c, seed & (2 ** 64 - 1),
                                  1 if permute else 0))


def rmat_n(n: int, avg_degree: float, seed: int = 0, **kw):
    """R-MAT on n vertices (any n >= 2) with about avg_degree non-zeros per row."""
    scale = max(1, math.ceil(math.log2(n)))
    return rmat(scale, avg_degree / 2.0, seed=seed, n=n, **kw)


def normalize_sym(rowptr, col, val):
    """D^{-1/2} A D^{-1/2} in float64 (returns a new value array)."""
    val = np.array(val, dtype=np.float64, copy=True)
    _load().syn_normalize_sym(rowptr.size - 1, _p(np.ascontiguousarray(rowptr, np.int64)),
                              _p(np.ascontiguousarray(col, np.int32)), _p(val))
    return val


# ---------------------------------------------------------------- precisions
PRECISIONS = ("fp64", "fp32", "bf16")


def f32_to_bf16_bits(x32: np.ndarray) -> np.ndarray:
    """Round-to-nearest-even of float32 values to bfloat16, as uint16 bits."""
    u = np.ascontiguousarray(x32, dtype=np.float32).view(np.uint32).astype(np.uint64)
    nan = np.isnan(np.asarray(x32, dtype=np.float32))
    r = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    r = np.where(nan, (u >> 16) | 0x40, r)
    return r.astype(np.uint16)


def bf16_bits_to_f64(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


def round_values(val, precision: str) -> np.ndarray:
    """Values rounded to what `precision` can store, returned as float64."""
    val = np.asarray(val, dtype=np.float64)
    if precision == "fp64":
        return val.copy()
    if precision == "fp32":
        return val.astype(np.float32).astype(np.float64)
    if precision == "bf16":
        return bf16_bits_to_f64(f32_to_bf16_bits(val.astype(np.float32)))
    raise ValueError(precision)


def to_storage(val, precision: str) -> np.ndarray:
    """Values in the storage type of `precision` (bf16 as uint16 bits)."""
    val = np.asarray(val, dtype=np.float64)
    if precision == "fp64":
        return val.copy()
    if precision == "fp32":
        return val.astype(np.float32)
    if precision == "bf16":
        return f32_to_bf16_bits(val.astype(np.float32))
    raise ValueError(precision)


# ------------------------------------------------------ closed-form graphs
def from_edges(n: int, edges, weights=None, diag=None):
    """Symmetric CSR from an undirected edge list (each pair once)."""
    rows, cols, vals = [], [], []
    for e, (u, v) in enumerate(edges):
        w = 1.0 if weights is None else float(weights[e])
        rows += [u, v]
        cols += [v, u]
        vals += [w, w]
    if diag is not None:
        for i in range(n):
            if diag[i] != 0.0:
                rows.append(i)
                cols.append(i)
                vals.append(float(diag[i]))
    rows = np.asarray(rows, np.int64)
    cols = np.asarray(cols, np.int64)
    vals = np.asarray(vals, np.float64)
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, cols.astype(np.int32), vals


def path(n):
    return from_edges(n, [(i, i + 1) for i in range(n - 1)])


def cycle(n):
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def complete(n):
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)])


def star(s):
    return from_edges(s + 1, [(0, j) for j in range(1, s + 1)])


def complete_bipartite(a, b):
    return from_edges(a + b, [(i, a + j) for i in range(a) for j in range(b)])


def hypercube(d):
    n = 1 << d
    return from_edges(n, [(i, i ^ (1 << k)) for i in range(n) for k in range(d) if i < i ^ (1 << k)])


def diagonal(d):
    d = np.asarray(d, np.float64)
    return from_edges(d.size, [], diag=d)


def dense_to_csr(A):
    """CSR of the non-zero pattern of a dense matrix (tests only)."""
    A = np.asarray(A, np.float64)
    n = A.shape[0]
    rowptr = np.zeros(n + 1, np.int64)
    cols, vals = [], []
    for i in range(n):
        nz = np.nonzero(A[i])[0]
        cols.extend(nz.tolist())
        vals.extend(A[i, nz].tolist())
        rowptr[i + 1] = rowptr[i] + nz.size
    return rowptr, np.asarray(cols, np.int32), np.asarray(vals, np.float64)
