"""CPU checks of the comparison rules the GPU parity tests use (tie-aware
Top-K pairing, the Ritz-vector entry bound and the sign rule), so that a
plausible mistake on the GPU side cannot pass them."""
import numpy as np
import pytest

from gpu_util import check_ritz_entries, ritz_entry_tol, top2_margin, topk_pair_err


def test_pairing_allows_ties_in_modulus_only():
    want = np.array([1.0, -1.0, 0.5, 0.25])
    # The +-1 tie may come in either order.
    assert np.all(topk_pair_err([-1.0, 1.0, 0.5, 0.25], want, 1e-6) == 0.0)
    # Values that do not tie must come in Top-K order: 0.5 and 0.25 swapped fail.
    err = topk_pair_err([1.0, -1.0, 0.25, 0.5], want, 1e-6)
    assert err[2] == pytest.approx(0.5) and err[3] == pytest.approx(1.0)
    # A sign error on a non-tied value is caught.
    assert topk_pair_err([1.0, -1.0, -0.5, 0.25], want, 1e-6)[2] == pytest.approx(2.0)


def test_pairing_at_the_topk_boundary_uses_all_ritz_values():
    # The reference kept 0.5, but -0.5 (outside its Top-2) ties in modulus.
    want = np.array([2.0, 0.5])
    theta = np.array([2.0, 0.5, -0.5, 0.1])
    assert np.all(topk_pair_err([2.0, -0.5], want, 1e-6, theta) == 0.0)
    assert topk_pair_err([2.0, 0.1], want, 1e-6, theta)[1] > 0.5


def test_entry_bound_grows_as_the_gap_shrinks():
    vals = np.array([1.0, 0.9])
    theta = np.array([1.0, 0.9, 0.899, 0.1])
    tol, gaps = ritz_entry_tol(vals, theta, np.array([1e-12]), np.array([1e-12]), 1.0, 4, 2.0 ** -53)
    assert gaps[0] == pytest.approx(0.1) and gaps[1] == pytest.approx(0.001)
    assert tol[1] > 50 * tol[0] > 0


def test_entry_check_catches_sign_and_column_mistakes():
    rng = np.random.default_rng(0)
    n, K = 400, 3
    Q, _ = np.linalg.qr(rng.standard_normal((n, K)))
    Q[7, :] = 0.5            # a clear largest entry in every column
    Q /= np.linalg.norm(Q, axis=0)
    tol = np.full(K, 1e-9)
    margin = top2_margin(Q)
    check_ritz_entries(Q + 1e-12, Q, tol, margin)
    # A flipped sign with an unambiguous largest entry breaks the sign rule.
    F = Q.copy()
    F[:, 1] *= -1
    with pytest.raises(AssertionError):
        check_ritz_entries(F, Q, tol, top2_margin(F))
    # An ambiguous largest entry leaves the sign free.
    A = Q.copy()
    A[8, :] = -A[7, :]
    A[:, 1] *= -1
    check_ritz_entries(A, A * np.array([1, -1, 1]), tol, top2_margin(A))
    # Columns in the wrong order fail.
    with pytest.raises(AssertionError):
        check_ritz_entries(Q[:, ::-1], Q, tol, margin)


@pytest.mark.parametrize("mode", ["fp32", "bf16"])
def test_first_step_bounds_hold_for_the_emulated_storage_modes(mode):
    # The oracle's emulation of a storage mode differs from the FP64 oracle in
    # alpha_1 and beta_2 by less than the bound; an SpMV that drops the last
    # entry of every row (a tile-boundary mistake) does not.
    import oracle
    import synth
    from gpu_util import first_step_bounds
    rp, c, v = synth.rmat(12, 8, seed=2)
    v = synth.round_values(v, mode)
    a64, b64, _, _ = oracle.lanczos(rp, c, v, 2, seed=0)
    ae, be, _, _ = oracle.lanczos_emul(rp, c, v, 2, mode, seed=0)
    ba, bb = first_step_bounds(rp, c, v, mode)
    assert abs(ae[0] - a64[0]) <= ba and abs(be[1] - b64[1]) <= bb
    v2 = v.copy()
    v2[rp[1:][np.diff(rp) > 0] - 1] = 0.0
    aw, bw, _, _ = oracle.lanczos(rp, c, v2, 2, seed=0)
    assert abs(aw[0] - a64[0]) > ba or abs(bw[1] - b64[1]) > bb
