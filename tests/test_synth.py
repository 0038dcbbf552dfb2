"""Input generators: structure, symmetry, sizes and determinism."""
import numpy as np
import scipy.sparse as sp

import synth


def _sym_ok(rp, c, v):
    n = rp.size - 1
    A = sp.csr_matrix((v, c, rp), shape=(n, n))
    assert (abs(A - A.T)).max() == 0.0
    for r in range(0, n, max(1, n // 97)):
        row = c[rp[r]:rp[r + 1]]
        assert np.all(np.diff(row) > 0)             # sorted, no duplicates
    return A


def test_er_shape_values_and_determinism():
    rp, c, v = synth.er(10000, 9.0, seed=0)
    n = 10000
    assert rp.size == n + 1 and rp[0] == 0 and np.all(np.diff(rp) >= 1)
    nnz = rp[-1]
    assert 97000 < nnz < 103000                    # ~10 per row with the diagonal
    A = _sym_ok(rp, c, v)
    d = A.diagonal()
    assert np.all((d >= 0) & (d < 1))
    off = A - sp.diags(d)
    assert off.data.min() >= -1 and off.data.max() < 1
    rp2, c2, v2 = synth.er(10000, 9.0, seed=0)
    assert np.array_equal(rp, rp2) and np.array_equal(c, c2) and np.array_equal(v, v2)
    rp3, _, _ = synth.er(10000, 9.0, seed=1)
    assert not np.array_equal(rp, rp3)


def test_rmat_structure_and_skew():
    rp, c, v = synth.rmat(14, 8, seed=0)
    n = 1 << 14
    A = _sym_ok(rp, c, v)
    assert A.diagonal().max() == 0.0                # self loops dropped
    assert np.all((v > 0) & (v < 1))
    deg = np.diff(rp)
    assert deg.max() > 20 * deg.mean()              # power-law hubs
    assert 0.6 * 16 * n < rp[-1] <= 16 * n          # at most 2 per draw, duplicates merged
    rp2, c2, v2 = synth.rmat(14, 8, seed=0)
    assert np.array_equal(c, c2) and np.array_equal(v, v2)


def test_rmat_truncated_n_and_normalisation():
    rp, c, v = synth.rmat_n(3000, 12.0, seed=3)
    assert rp.size == 3001 and c.max() < 3000
    _sym_ok(rp, c, v)
    w = synth.normalize_sym(rp, c, v)
    n = 3000
    A = sp.csr_matrix((w, c, rp), shape=(n, n))
    # D^{-1/2} A D^{-1/2} has spectral radius 1 with the sqrt-degree vector as eigenvector.
    d = np.asarray(sp.csr_matrix((v, c, rp), shape=(n, n)).sum(axis=1)).ravel()
    x = np.sqrt(d)
    np.testing.assert_allclose(A @ x, x, rtol=1e-12, atol=1e-12)


def test_rounding_to_storage_precisions():
    x = np.array([1.0, 1.0 / 3.0, 1e-3, 0.7, -2.5, 3.0e38])
    np.testing.assert_array_equal(synth.round_values(x, "fp64"), x)
    np.testing.assert_array_equal(synth.round_values(x, "fp32"), x.astype(np.float32).astype(np.float64))
    b = synth.to_storage(x, "bf16")
    assert b.dtype == np.uint16
    back = synth.bf16_bits_to_f64(b)
    assert np.all(np.abs(back - x) <= np.abs(x) * 2.0 ** -8)
    # Round-to-nearest-even on an exact tie: 1 + 2^-8 lies between 1 and 1 + 2^-7.
    tie = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8], dtype=np.float64)
    np.testing.assert_array_equal(synth.round_values(tie, "bf16"), [1.0, 1.0 + 2.0 ** -6])
