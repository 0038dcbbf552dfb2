"""Helpers for the GPU tests: move CSR inputs to the device in a storage
precision, and compare eigenpairs with tie- and sign-aware rules."""
import numpy as np

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
