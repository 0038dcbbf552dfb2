"""FP64 CPU oracle for the Lanczos + Jacobi Top-K eigensolver.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  The product library
(``paper_2201_07498_amd``) never imports it and shares no code with it.

The arithmetic lives in ``lanczos_oracle.c`` (plain sequential C, binary64);
this module only marshals numpy arrays through ctypes and composes the
steps in the order of Sec. III of the paper:

  1. Lanczos with full reorthogonalisation (Algorithm 1) -> alpha, beta, V
  2. Jacobi on the tridiagonal T (Sec. III, second phase) -> theta, S
  3. Top-K by modulus (Sec. I)
  4. Ritz vectors V S (Sec. III)
  5. Accuracy report (Sec. IV-D): residuals, orthogonality, mean angle

Matrix values are taken as float64 (values stored in a lower precision are
upcast exactly before the call).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lanczos_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

UNIT_ROUNDOFF = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16": 2.0 ** -8}


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-ffp-contract=off", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i64, i32, u64, f64 = ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, ctypes.c_double
        lib.orc_splitmix64.restype = u64
        lib.orc_splitmix64.argtypes = [u64, u64]
        lib.orc_u01.restype = f64
        lib.orc_u01.argtypes = [u64, u64]
        lib.orc_spmv.restype = None
        lib.orc_spmv.argtypes = [i64, P, P, P, P, P]
        lib.orc_lanczos.restype = i32
        lib.orc_lanczos.argtypes = [i64, P, P, P, i32, u64, i32, f64, P, P, P]
        lib.orc_jacobi.restype = i32
        lib.orc_jacobi.argtypes = [i32, P, P, i32]
        lib.orc_select_topk.restype = None
        lib.orc_select_topk.argtypes = [i32, P, i32, P]
        lib.orc_ritz.restype = None
        lib.orc_ritz.argtypes = [i64, i32, P, P, i32, P, P]
        lib.orc_residuals.restype = None
        lib.orc_residuals.argtypes = [i64, P, P, P, i32, P, P, P, P]
        lib.orc_ortho_loss.restype = f64
        lib.orc_ortho_loss.argtypes = [i64, i32, P]
        lib.orc_mean_angle_deg.restype = f64
        lib.orc_mean_angle_deg.argtypes = [i64, i32, P]
        lib.orc_round_bits.restype = f64
        lib.orc_round_bits.argtypes = [f64, i32]
        lib.orc_spmv_emul.restype = None
        lib.orc_spmv_emul.argtypes = [i64, P, P, P, P, P, i32]
        lib.orc_lanczos_emul.restype = i32
        lib.orc_lanczos_emul.argtypes = [i64, P, P, P, i32, u64, i32, f64, i32, i32, i32, P, P, P]
        lib.orc_start_vector.restype = None
        lib.orc_start_vector.argtypes = [i64, u64, P]
        lib.orc_set_progress.restype = None
        lib.orc_set_progress.argtypes = [i32]
        _lib = lib
    return _lib


def set_progress(on: bool) -> None:
    """Print one line per Lanczos step on stderr (long runs); results are
    unaffected."""
    _load().orc_set_progress(1 if on else 0)


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _csr(rowptr, col, val):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int64)
    col = np.ascontiguousarray(col, dtype=np.int32)
    val = np.ascontiguousarray(val, dtype=np.float64)
    return rowptr, col, val


def splitmix64(seed: int, r: int) -> int:
    """Output number r (0-based) of the SplitMix64 stream started at seed."""
    return int(_load().orc_splitmix64(seed & (2 ** 64 - 1), r))


def u01(seed: int, r: int) -> float:
    return float(_load().orc_u01(seed & (2 ** 64 - 1), r))


def start_vector(n: int, seed: int = 0) -> np.ndarray:
    """v_1 = u/||u|| with u_r = U01(SplitMix64(seed, r)), as lanczos() uses it."""
    v = np.empty(n, dtype=np.float64)
    _load().orc_start_vector(n, seed & (2 ** 64 - 1), _p(v))
    return v


def spmv(rowptr, col, val, x) -> np.ndarray:
    rowptr, col, val = _csr(rowptr, col, val)
    n = rowptr.size - 1
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    _load().orc_spmv(n, _p(rowptr), _p(col), _p(val), _p(x), _p(y))
    return y


def lanczos(rowptr, col, val, m: int, seed: int = 0, passes: int = 2,
            unit_roundoff: float = 2.0 ** -53):
    """Algorithm 1 for m steps.  Returns (alpha[m], beta[m+1], V[n, m+1], restarts).

    beta[0] is beta_1 = 0; beta[i] couples v_i and v_{i+1} (1-based);
    beta[m] is the norm of the residual vector after the last step.
    """
    rowptr, col, val = _csr(rowptr, col, val)
    n = rowptr.size - 1
    alpha = np.zeros(m, dtype=np.float64)
    beta = np.zeros(m + 1, dtype=np.float64)
    V = np.zeros((m + 1, n), dtype=np.float64)   # row k = v_{k+1}
    rc = _load().orc_lanczos(n, _p(rowptr), _p(col), _p(val), m, seed & (2 ** 64 - 1),
                             passes, unit_roundoff, _p(alpha), _p(beta), _p(V))
    if rc < 0:
        raise ValueError(f"oracle lanczos failed with code {rc}")
    return alpha, beta, V.T, rc


# Significant bits of the emulated formats: (stored vectors, SpMV
# accumulation, working vector).  "fp32" and "bf16" are the storage modes of
# Sec. III-A with a binary32 accumulator; "fp64" rounds nothing.
EMULATION = {"fp64": (53, 53, 53), "fp32": (24, 24, 24), "bf16": (8, 24, 24)}


def round_bits(x: float, bits: int) -> float:
    """x rounded to `bits` significant bits, ties to even (24: binary32,
    8: bfloat16, in their normal ranges)."""
    return float(_load().orc_round_bits(float(x), int(bits)))


def spmv_emul(rowptr, col, val, x, acc_bits: int) -> np.ndarray:
    """y = M x with products and partial sums rounded to acc_bits."""
    rowptr, col, val = _csr(rowptr, col, val)
    n = rowptr.size - 1
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.empty(n, dtype=np.float64)
    _load().orc_spmv_emul(n, _p(rowptr), _p(col), _p(val), _p(x), _p(y), int(acc_bits))
    return y


def lanczos_emul(rowptr, col, val, m: int, emulate: str, seed: int = 0, passes: int = 2,
                 unit_roundoff: float = 2.0 ** -53):
    """Algorithm 1 with the roundings of a reduced-precision storage mode
    (EMULATION[emulate]); same outputs as lanczos()."""
    store, acc, work = EMULATION[emulate]
    rowptr, col, val = _csr(rowptr, col, val)
    n = rowptr.size - 1
    alpha = np.zeros(m, dtype=np.float64)
    beta = np.zeros(m + 1, dtype=np.float64)
    V = np.zeros((m + 1, n), dtype=np.float64)
    rc = _load().orc_lanczos_emul(n, _p(rowptr), _p(col), _p(val), m, seed & (2 ** 64 - 1), passes,
                                  unit_roundoff, store, acc, work, _p(alpha), _p(beta), _p(V))
    if rc < 0:
        raise ValueError(f"oracle lanczos_emul failed with code {rc}")
    return alpha, beta, V.T, rc


def tridiag(alpha, beta) -> np.ndarray:
    """T = tridiag(beta_2..beta_m; alpha_1..alpha_m; beta_2..beta_m)."""
    m = alpha.size
    T = np.diag(np.asarray(alpha, dtype=np.float64))
    for i in range(m - 1):
        T[i, i + 1] = T[i + 1, i] = beta[i + 1]
    return T


def jacobi(A, max_sweeps: int = 60):
    """Cyclic Jacobi on a dense symmetric matrix.  Returns (theta, S, sweeps)."""
    A = np.array(A, dtype=np.float64, order="C", copy=True)
    m = A.shape[0]
    S = np.zeros((m, m), dtype=np.float64)
    sweeps = _load().orc_jacobi(m, _p(A), _p(S), max_sweeps)
    if sweeps < 0:
        raise RuntimeError("oracle Jacobi did not converge")
    return np.diag(A).copy(), S, sweeps


def select_topk(theta, K: int) -> np.ndarray:
    theta = np.ascontiguousarray(theta, dtype=np.float64)
    idx = np.zeros(K, dtype=np.int32)
    _load().orc_select_topk(theta.size, _p(theta), K, _p(idx))
    return idx


def ritz(V, S, idx) -> np.ndarray:
    """Y = V[:, :m] S[:, idx], unit columns, sign rule.  V is (n, >=m)."""
    n = V.shape[0]
    m = S.shape[0]
    Vc = np.ascontiguousarray(np.asarray(V)[:, :m].T, dtype=np.float64)   # column-major
    S = np.ascontiguousarray(S, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    K = idx.size
    Y = np.zeros((K, n), dtype=np.float64)
    _load().orc_ritz(n, m, _p(Vc), _p(S), K, _p(idx), _p(Y))
    return Y.T


def residuals(rowptr, col, val, vals, Y):
    rowptr, col, val = _csr(rowptr, col, val)
    n = rowptr.size - 1
    vals = np.ascontiguousarray(vals, dtype=np.float64)
    Yc = np.ascontiguousarray(np.asarray(Y).T, dtype=np.float64)
    K = vals.size
    ab = np.zeros(K)
    rel = np.zeros(K)
    _load().orc_residuals(n, _p(rowptr), _p(col), _p(val), K, _p(vals), _p(Yc), _p(ab), _p(rel))
    return ab, rel


def ortho_loss(X) -> float:
    Xc = np.ascontiguousarray(np.asarray(X).T, dtype=np.float64)
    return float(_load().orc_ortho_loss(Xc.shape[1], Xc.shape[0], _p(Xc)))


def mean_angle_deg(Y) -> float:
    Yc = np.ascontiguousarray(np.asarray(Y).T, dtype=np.float64)
    return float(_load().orc_mean_angle_deg(Yc.shape[1], Yc.shape[0], _p(Yc)))


def topk(rowptr, col, val, K: int, m: int, seed: int = 0, passes: int = 2,
         unit_roundoff: float = 2.0 ** -53, report: bool = True, emulate: str | None = None) -> dict:
    """The whole solve: Lanczos, Jacobi on T, Top-K, Ritz vectors, report.
    With `emulate` ("fp32", "bf16") the Lanczos phase rounds its stored
    vectors and SpMV as that storage mode does (lanczos_emul); the rest is
    binary64 either way."""
    if not (1 <= K <= m <= rowptr.size - 1):
        raise ValueError("need 1 <= K <= m <= n")
    if emulate is None:
        alpha, beta, V, restarts = lanczos(rowptr, col, val, m, seed, passes, unit_roundoff)
    else:
        alpha, beta, V, restarts = lanczos_emul(rowptr, col, val, m, emulate, seed, passes, unit_roundoff)
    T = tridiag(alpha, beta)
    theta, S, sweeps = jacobi(T)
    idx = select_topk(theta, K)
    vals = theta[idx]
    Y = ritz(V, S, idx)
    out = dict(vals=vals, vecs=Y, alpha=alpha, beta=beta, theta=theta, S=S, idx=idx,
               restarts=restarts, sweeps=sweeps, V=V)
    if report:
        ab, rel = residuals(rowptr, col, val, vals, Y)
        out.update(abs_resid=ab, rel_resid=rel, ortho_loss=ortho_loss(V[:, :m]),
                   ritz_ortho_loss=ortho_loss(Y), mean_angle_deg=mean_angle_deg(Y),
                   resid_estimate=np.abs(beta[m] * S[m - 1, idx]))
    return out
