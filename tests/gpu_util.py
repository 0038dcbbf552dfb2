"""Helpers for the GPU tests: move CSR inputs to the device in a storage
precision, and compare eigenpairs with tie- and sign-aware rules."""
import numpy as np

import oracle
import synth


def device_csr(rowptr, col, val, precision, dev="cuda:0"):
    import torch
    rp = torch.from_numpy(np.ascontiguousarray(rowptr, np.int64)).to(dev)
    c = torch.from_numpy(np.ascontiguousarray(col, np.int32)).to(dev)
    v = device_values(val, precision, dev)
    return rp, c, v


def device_values(val, precision, dev="cuda:0"):
    import torch
    s = synth.to_storage(val, precision)
    if precision == "bf16":
        return torch.from_numpy(s.view(np.int16)).to(dev).view(torch.bfloat16)
    return torch.from_numpy(s).to(dev)


def eig_rel_err(got, want):
    """max_k |got_k - want_k| / |want_k| after pairing by the Top-K order
    (denominator floored at 1e-12 * max|want|)."""
    got, want = np.asarray(got), np.asarray(want)
    den = np.maximum(np.abs(want), 1e-12 * np.max(np.abs(want)))
    return float(np.max(np.abs(got - want) / den))


def multiset_rel_err(got, want):
    """Like eig_rel_err but pairing sorted values (for ties in |lambda|)."""
    return eig_rel_err(np.sort(got), np.sort(want))


def subspace_cos(Y, Z, vals, tol):
    """For every Ritz vector y_k: the norm of its projection onto the span of
    the reference vectors whose eigenvalues lie within tol of vals[k]."""
    out = []
    for k in range(Y.shape[1]):
        near = np.nonzero(np.abs(vals - vals[k]) <= tol * max(1.0, abs(vals[k])))[0]
        Q, _ = np.linalg.qr(Z[:, near])
        out.append(np.linalg.norm(Q.T @ Y[:, k]))
    return np.array(out)


def topk_pair_err(got, want, tol, theta_ref=None):
    """Per-position relative eigenvalue errors in Top-K order (R17) with the
    tie rule of R8: reference positions whose moduli agree within `tol`
    (relative) form a group, and a group is compared as sorted values, so
    either member of a tie may come first.  If the last group also ties with
    Ritz values outside the reference's Top-K (all of them in theta_ref),
    each of its values is matched to the nearest of those candidates."""
    got, want = np.asarray(got, np.float64), np.asarray(want, np.float64)
    K = want.size
    den_floor = 1e-12 * np.max(np.abs(want))
    err = np.zeros(K)
    k = 0
    while k < K:
        e = k + 1
        while e < K and abs(want[e - 1]) - abs(want[e]) <= tol * abs(want[e - 1]):
            e += 1
        g = np.sort(got[k:e])
        w = np.sort(want[k:e])
        boundary = e == K and theta_ref is not None
        if boundary:
            th = np.asarray(theta_ref, np.float64)
            cand = th[np.abs(th) >= abs(want[e - 1]) * (1 - tol)]
            for i, x in enumerate(g):
                j = np.argmin(np.abs(cand - x))
                err[k + i] = abs(x - cand[j]) / max(abs(cand[j]), den_floor)
        else:
            err[k:e] = np.abs(g - w) / np.maximum(np.abs(w), den_floor)
        k = e
    return err


def ritz_gaps(vals, theta_all):
    """Distance from each selected Ritz value to the nearest other Ritz value
    of the same solve (all m of them)."""
    th = np.sort(np.asarray(theta_all, np.float64))
    out = []
    for x in np.asarray(vals, np.float64):
        i = int(np.argmin(np.abs(th - x)))
        rest = np.delete(th, i)
        out.append(np.min(np.abs(rest - x)) if rest.size else np.inf)
    return np.array(out)


def ritz_entry_tol(vals, theta_all, dalpha, dbeta, tnorm, m, u):
    """Entry-wise bound on the difference of two computations of the same Ritz
    vectors whose tridiagonal matrices differ by at most
    dT = max|d alpha| + 2 max|d beta| (the 2-norm of a symmetric tridiagonal
    perturbation).  A Ritz vector is y = V s with s the eigenvector of T:
      * by the Davis-Kahan sin-theta bound, ||ds|| <= sqrt(2) dT / gap, gap
        the distance to the nearest other Ritz value;
      * the bases differ by about the same relative amount as T does, so
        ||dV s|| is taken as sqrt(m) dT / ||T||;
    plus a rounding floor of 64 u.  Entries are bounded by the 2-norm.  Safety
    factor 4."""
    gaps = ritz_gaps(vals, theta_all)
    dT = float(np.max(np.abs(dalpha))) + 2.0 * float(np.max(np.abs(dbeta)))
    return 4.0 * (np.sqrt(2.0) * dT / gaps + np.sqrt(m) * dT / tnorm) + 64.0 * u, gaps


def top2_margin(Y):
    """Per column: largest |entry| minus the second largest (full vectors)."""
    A = np.abs(np.asarray(Y))
    part = -np.partition(-A, 1, axis=0)[:2]
    return part[0] - part[1]


def check_ritz_entries(Yg, Yr, tol, margin, what="", extra=None):
    """Yg, Yr: rows x K entries of the GPU and reference Ritz vectors at the
    same rows; tol: per-vector entry bound; margin: the GPU vector's largest
    |entry| minus its second largest; extra: optional (g, r) pairs of length
    K, one more entry per vector (e.g. at the reference's largest entry).
    Where margin > 2 tol both vectors have their largest entry in the same
    row, so the sign rule (R9) fixes the sign and entries are compared as they
    are; otherwise up to sign.  The bound is asserted for every vector; a
    vector counts as informative when some compared reference entry exceeds
    10 tol (a wrong vector would then show).  Returns (max abs differences,
    informative mask, signed mask)."""
    Yg, Yr = np.asarray(Yg, np.float64), np.asarray(Yr, np.float64)
    if extra is not None:
        Yg = np.vstack([Yg, np.asarray(extra[0], np.float64)[None, :]])
        Yr = np.vstack([Yr, np.asarray(extra[1], np.float64)[None, :]])
    signed = np.asarray(margin) > 2.0 * tol
    d_plus = np.max(np.abs(Yg - Yr), axis=0)
    d_minus = np.max(np.abs(Yg + Yr), axis=0)
    diff = np.where(signed, d_plus, np.minimum(d_plus, d_minus))
    informative = np.max(np.abs(Yr), axis=0) > 10.0 * tol
    bad = diff > tol
    assert not np.any(bad), f"{what}: entry diffs {diff[bad]} over bounds {tol[bad]} (vectors {np.nonzero(bad)[0]})"
    return diff, informative, signed

U_STORE = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16": 2.0 ** -8}
U_WORK = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16": 2.0 ** -24}


def first_step_bounds(rowptr, col, val, precision, seed=0):
    """Bounds on |d alpha_1| and |d beta_2| between the GPU solve and the
    oracle: both depend only on v_1 and one SpMV.  Row r of A v_1 is a sum of
    L_r products; two summation orders in a working precision with unit
    roundoff u_w each stay within L_r u_w sum_k |a_rk v_k|, the stored v_1
    adds u_s, and the working vector's rounding u_w, so
      |d (A v_1)_r| <= e_r = (2 L_r u_w + u_s + u_w) (|A| |v_1|)_r,
      |d alpha_1| <= v_1 . e,   |d beta_2| <= ||e|| + |d alpha_1|
    (the orthogonalisation against v_1 moves beta_2 by rounding only).
    Returned with a safety factor of 2."""
    n = rowptr.size - 1
    v1 = oracle.start_vector(n, seed)
    mag = oracle.spmv(rowptr, col, np.abs(np.asarray(val, np.float64)), v1)
    L = np.diff(rowptr).astype(np.float64)
    e = (2.0 * L * U_WORK[precision] + U_STORE[precision] + U_WORK[precision]) * mag
    ba = float(v1 @ e)
    return 2.0 * ba, 2.0 * (float(np.linalg.norm(e)) + ba)


BF16_TOL = 1e-3


def bf16_bounds(ref, emul_vals, gpu_abs_resid):
    """Per-pair bound of a BF16-storage solve against the FP64 oracle: 1e-3
    on the pairs the FP64 oracle has converged (relative residual <= 1e-6);
    elsewhere the larger of four times the largest error of the oracle's
    emulation of the BF16 mode and the two runs' residuals (each Ritz value
    lies within its residual of an eigenvalue of the matrix), at least 1e-3.
    Which unconverged pairs move, and how far, depends on the rounding of the
    whole Krylov sequence (Sec. III-A found 16-bit storage unstable).
    Returns (bounds, converged mask, emulated errors)."""
    vals = np.asarray(ref["vals"])
    emul_err = topk_pair_err(emul_vals, vals, 1e-3, np.asarray(ref["theta"]))
    conv = np.asarray(ref["rel_resid"]) <= 1e-6
    band = np.maximum(max(BF16_TOL, 4.0 * float(np.max(emul_err))),
                      (np.asarray(ref["abs_resid"]) + np.asarray(gpu_abs_resid)) / np.abs(vals))
    return np.where(conv, BF16_TOL, band), conv, emul_err
