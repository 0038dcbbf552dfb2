"""Pins for the FP64 CPU oracle, against facts that do not come from the
oracle itself: published generator outputs, dense LAPACK eigensolves,
closed-form graph spectra, extended-precision Krylov projections, ARPACK and
the algebraic invariants of the Lanczos relation (Sec. III, Algorithm 1).

The paper prints no eigenvalues or worked example, so every pin here is
mathematical or from an independent library routine.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth

EPS = 2.0 ** -52
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def dense(rowptr, col, val):
    n = rowptr.size - 1
    return sp.csr_matrix((val, col, rowptr), shape=(n, n)).toarray()


def csr_matrix(rowptr, col, val):
    n = rowptr.size - 1
    return sp.csr_matrix((val, col, rowptr), shape=(n, n))


def random_sym(n, seed, density=1.0, distinct=True):
    rng = np.random.default_rng(seed)
    A = rng.uniform(-1, 1, (n, n))
    if density < 1.0:
        A *= rng.random((n, n)) < density
    A = np.triu(A)
    A = A + np.triu(A, 1).T
    return A


def multiset_close(got, want, tol):
    got = np.sort(np.asarray(got))
    want = np.sort(np.asarray(want))
    assert got.shape == want.shape
    assert np.max(np.abs(got - want)) <= tol, (got, want)


# ----------------------------------------------------------------- RNG
def test_splitmix64_published_vectors():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "splitmix64.txt")) if l.strip() and l[0] != "#"]
    assert len(rows) == 6
    for seed, idx, hx in rows:
        assert oracle.splitmix64(int(seed), int(idx)) == int(hx, 16)


def test_u01_is_top_53_bits():
    for r in range(5):
        assert oracle.u01(0, r) == (oracle.splitmix64(0, r) >> 11) / 2.0 ** 53
    u = np.array([oracle.u01(7, r) for r in range(20000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.01 and abs(u.var() - 1 / 12) < 0.005


def test_start_vector_is_normalised_u01_and_the_lanczos_v1():
    n = 1000
    u = np.array([(oracle.splitmix64(3, r) >> 11) / 2.0 ** 53 for r in range(n)])
    v = oracle.start_vector(n, seed=3)
    assert np.allclose(v, u / np.linalg.norm(u), rtol=1e-15, atol=0)
    rp, c, val = synth.er(n, 6.0, seed=1)
    _, _, V, _ = oracle.lanczos(rp, c, val, 3, seed=3)
    assert np.array_equal(V[:, 0], v)


# -------------------------------------------------------------- SpMV
def test_spmv_matches_dense_product():
    A = random_sym(40, 1, density=0.3)
    rp, c, v = synth.dense_to_csr(A)
    x = np.random.default_rng(2).standard_normal(40)
    np.testing.assert_allclose(oracle.spmv(rp, c, v, x), A @ x, rtol=1e-14, atol=1e-14)


# ------------------------------------------------------------ Jacobi
@pytest.mark.parametrize("m,seed", [(2, 0), (5, 1), (24, 2), (48, 3), (64, 4)])
def test_jacobi_random_dense_vs_lapack(m, seed):
    A = random_sym(m, seed)
    theta, S, sweeps = oracle.jacobi(A)
    lam = np.linalg.eigvalsh(A)
    nrm = np.linalg.norm(A, 2)
    multiset_close(theta, lam, 20 * m * EPS * nrm)
    assert np.max(np.abs(S.T @ S - np.eye(m))) < 50 * m * EPS
    assert np.max(np.abs(A @ S - S * theta)) < 50 * m * EPS * nrm
    assert abs(theta.sum() - np.trace(A)) < 50 * m * EPS * nrm
    assert abs((theta ** 2).sum() - (A ** 2).sum()) < 50 * m * EPS * nrm ** 2
    assert sweeps <= 20


def sturm_count(a, b, x):
    """Number of eigenvalues of tridiag(b; a; b) below x (Sylvester inertia)."""
    cnt, d = 0, 1.0
    for i in range(a.size):
        d = a[i] - x - (b[i - 1] ** 2 / d if i > 0 else 0.0)
        if d == 0.0:
            d = -1e-300
        cnt += d < 0
    return cnt


@pytest.mark.parametrize("m,seed", [(8, 0), (32, 1), (64, 2)])
def test_jacobi_tridiagonal_sturm_counts(m, seed):
    rng = np.random.default_rng(seed)
    a, b = rng.uniform(-2, 2, m), rng.uniform(0.1, 1, m - 1)
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    theta, _, _ = oracle.jacobi(T)
    th = np.sort(theta)
    # Between consecutive computed eigenvalues the Sturm count must step by one.
    for k in range(m):
        assert sturm_count(a, b, th[k] - 1e-9) == k
        assert sturm_count(a, b, th[k] + 1e-9) == k + 1


def test_jacobi_diagonal_and_2x2_closed_form():
    theta, S, sweeps = oracle.jacobi(np.diag([3.0, -1.0, 2.0]))
    assert list(theta) == [3.0, -1.0, 2.0] and sweeps == 1
    assert np.array_equal(S, np.eye(3))
    a, b, c = 1.5, 0.7, -0.4
    theta, S, _ = oracle.jacobi(np.array([[a, b], [b, c]]))
    mid, rad = (a + c) / 2, math.hypot((a - c) / 2, b)
    multiset_close(theta, [mid - rad, mid + rad], 4 * EPS * 2)


# ---------------------------------------------------------- selection
def test_select_orders_by_modulus_then_value_then_index():
    th = np.array([0.5, -2.0, 2.0, 1.0, -1.0, 2.0, 0.0])
    idx = oracle.select_topk(th, 7)
    assert list(idx) == [2, 5, 1, 3, 4, 0, 6]
    assert list(oracle.select_topk(th, 3)) == [2, 5, 1]


# ------------------------------------------- whole oracle, m = n (exact)
@pytest.mark.parametrize("n,seed", [(30, 0), (80, 1), (150, 2)])
def test_full_krylov_recovers_dense_spectrum(n, seed):
    A = random_sym(n, seed, density=0.2) + np.diag(np.random.default_rng(seed).uniform(0, 1, n))
    rp, c, v = synth.dense_to_csr(A)
    out = oracle.topk(rp, c, v, K=n, m=n, seed=seed)
    lam = np.linalg.eigvalsh(A)
    nrm = np.linalg.norm(A, 2)
    multiset_close(out["theta"], lam, 1e-12 * nrm)
    # Top-K by modulus.
    top = lam[np.argsort(-np.abs(lam), kind="stable")][:5]
    multiset_close(out["vals"][:5], top, 1e-12 * nrm)
    assert out["ortho_loss"] < 1e-13
    assert np.max(out["abs_resid"]) < 1e-10 * nrm


def closed_form_cases():
    cases = []
    n = 25
    cases.append(("path25", synth.path(n), [2 * math.cos(math.pi * k / (n + 1)) for k in range(1, n + 1)]))
    n = 20
    cases.append(("cycle20", synth.cycle(n), [2 * math.cos(2 * math.pi * k / n) for k in range(n)]))
    n = 12
    cases.append(("complete12", synth.complete(n), [n - 1.0] + [-1.0] * (n - 1)))
    s = 9
    cases.append(("star9", synth.star(s), [3.0, -3.0] + [0.0] * (s - 1)))
    a, b = 3, 5
    cases.append(("k35", synth.complete_bipartite(a, b), [math.sqrt(15), -math.sqrt(15)] + [0.0] * (a + b - 2)))
    d = 4
    ev = []
    for k in range(d + 1):
        ev += [float(d - 2 * k)] * math.comb(d, k)
    cases.append(("hypercube4", synth.hypercube(d), ev))
    dg = [5.0, -4.0, 3.0, 3.0, 1.0, -0.5, 2.0, 0.25]
    cases.append(("diag8", synth.diagonal(dg), dg))
    return cases


@pytest.mark.parametrize("name,csr,lam", closed_form_cases(), ids=[c[0] for c in closed_form_cases()])
def test_closed_form_spectra_with_restarts(name, csr, lam):
    rp, c, v = csr
    n = rp.size - 1
    out = oracle.topk(rp, c, v, K=n, m=n, seed=3)
    multiset_close(out["theta"], lam, 1e-11 * max(1.0, max(abs(x) for x in lam)))
    lam = np.asarray(lam)
    top = lam[np.argsort(-np.abs(lam), kind="stable")][:4]
    np.testing.assert_allclose(np.sort(np.abs(out["vals"][:4])), np.sort(np.abs(top)), atol=1e-11)
    assert out["ortho_loss"] < 1e-12
    if name in ("complete12", "star9", "k35", "hypercube4", "diag8", "cycle20"):
        assert out["restarts"] > 0        # repeated eigenvalues force breakdowns
    if name == "path25":
        assert out["restarts"] == 0


# ------------------------------ extended-precision Krylov projection (m < n)
def _mp_ritz_values(A, v, m, dps=50):
    import mpmath as mp
    mp.mp.dps = dps
    n = A.shape[0]
    Am = mp.matrix(A.tolist())
    x = mp.matrix([mp.mpf(t) for t in v])
    basis = []
    for k in range(m):
        w = x if k == 0 else Am * basis[-1]
        for _ in range(2):
            for q in basis:
                w = w - q * (q.T * w)[0]
        w = w / mp.norm(w)
        basis.append(w)
    Q = mp.matrix(n, m)
    for k in range(m):
        for r in range(n):
            Q[r, k] = basis[k][r]
    H = Q.T * Am * Q
    H = (H + H.T) / 2
    E = mp.eigsy(H, eigvals_only=True)
    return np.array(sorted(float(e) for e in E))


@pytest.mark.parametrize("n,m,seed", [(12, 4, 0), (18, 6, 1), (20, 8, 2)])
def test_lanczos_ritz_values_equal_extended_precision_krylov_projection(n, m, seed):
    A = random_sym(n, seed, density=0.5) + np.diag(np.random.default_rng(seed + 9).uniform(0, 1, n))
    rp, c, v = synth.dense_to_csr(A)
    out = oracle.topk(rp, c, v, K=m, m=m, seed=seed)
    u = np.array([oracle.u01(seed, r) for r in range(n)])
    want = _mp_ritz_values(A, u / np.linalg.norm(u), m)
    got = np.sort(out["theta"])
    assert np.max(np.abs(got - want) / np.maximum(np.abs(want), 1e-3)) < 1e-13


# -------------------------------------------------------------- invariants
def test_lanczos_relation_and_orthogonality_on_er():
    rp, c, v = synth.er(1500, 9.0, seed=4)
    m = 40
    alpha, beta, V, restarts = oracle.lanczos(rp, c, v, m, seed=4)
    A = csr_matrix(rp, c, v)
    Vm = V[:, :m]
    T = oracle.tridiag(alpha, beta)
    nrm = spla.norm(A, 1)
    assert restarts == 0
    assert np.max(np.abs(Vm.T @ Vm - np.eye(m))) < 10 * m * EPS
    assert np.max(np.abs(Vm.T @ (A @ Vm) - T)) < 100 * EPS * nrm
    R = A @ Vm - Vm @ T
    R[:, m - 1] -= beta[m] * V[:, m]
    assert np.max(np.abs(R)) < 100 * EPS * nrm
    # Residual identity ||A y - theta y|| = beta_{m+1} |S_{m,k}|.
    out = oracle.topk(rp, c, v, K=8, m=m, seed=4)
    np.testing.assert_allclose(out["abs_resid"], out["resid_estimate"], rtol=1e-6, atol=1e-11)


def test_cauchy_interlacing():
    A = random_sym(300, 5, density=0.05)
    rp, c, v = synth.dense_to_csr(A)
    m = 20
    out = oracle.topk(rp, c, v, K=m, m=m, seed=5)
    lam = np.sort(np.linalg.eigvalsh(A))[::-1]
    th = np.sort(out["theta"])[::-1]
    for k in range(m):                      # k-th largest Ritz <= k-th largest eigenvalue
        assert th[k] <= lam[k] + 1e-12
        assert th[::-1][k] >= lam[::-1][k] - 1e-12
    assert th.max() <= lam.max() + 1e-12 and th.min() >= lam.min() - 1e-12


def test_reorthogonalisation_improves_orthogonality():
    # Sec. IV-D: full reorthogonalisation gives better orthogonality than none.
    rp, c, v = synth.er(2000, 9.0, seed=6)
    m = 150
    lo, ang = {}, {}
    for passes in (0, 1, 2):
        out = oracle.topk(rp, c, v, K=8, m=m, seed=6, passes=passes)
        lo[passes], ang[passes] = out["ortho_loss"], out["mean_angle_deg"]
    assert lo[2] < 1e-13 and lo[1] < 1e-13
    assert lo[0] > 1e-3                     # converged Ritz values: orthogonality lost
    assert ang[2] > 89.999 and ang[0] < ang[2] - 0.5


@pytest.mark.slow
def test_converged_pairs_agree_with_arpack():
    # ARPACK (scipy eigsh) is the paper's CPU baseline library (Sec. IV-A).
    rp, c, v = synth.er(10000, 9.0, seed=0)
    A = csr_matrix(rp, c, v)
    lam = spla.eigsh(A, k=8, which="LM", tol=1e-13, v0=np.ones(A.shape[0]))[0]
    out = oracle.topk(rp, c, v, K=8, m=400, seed=0)
    conv = out["abs_resid"] < 1e-8
    assert conv.sum() == 8
    want = lam[np.argsort(-np.abs(lam))]
    for k in np.nonzero(conv)[0]:
        assert np.min(np.abs(want - out["vals"][k])) <= out["abs_resid"][k] + 1e-12


def test_ritz_vectors_unit_orthogonal_and_signed():
    rp, c, v = synth.er(800, 9.0, seed=8)
    out = oracle.topk(rp, c, v, K=6, m=30, seed=8)
    Y = out["vecs"]
    assert np.max(np.abs(Y.T @ Y - np.eye(6))) < 1e-12
    for k in range(6):
        assert Y[np.argmax(np.abs(Y[:, k])), k] > 0
    assert 89.99 < out["mean_angle_deg"] <= 90.0


def test_restart_keeps_basis_orthonormal_and_t_block_diagonal():
    # Two disjoint triangles plus an isolated path: several invariant subspaces.
    edges = [(0, 1), (1, 2), (0, 2), (3, 4), (4, 5), (3, 5), (6, 7), (7, 8)]
    rp, c, v = synth.from_edges(9, edges)
    alpha, beta, V, restarts = oracle.lanczos(rp, c, v, 9, seed=1)
    assert restarts >= 1
    zero_beta = np.nonzero(beta[1:9] == 0.0)[0]
    assert zero_beta.size == restarts
    assert np.max(np.abs(V[:, :9].T @ V[:, :9] - np.eye(9))) < 1e-13


# ------------------------------------------------------ accuracy metrics
@pytest.mark.parametrize("phi_deg", [90.0, 60.0, 30.0, 1.0, 120.0])
def test_ortho_loss_and_mean_angle_of_two_vectors_at_a_known_angle(phi_deg):
    # Sec. IV-D metrics on constructed vectors: two unit vectors at angle phi
    # have X^T X - I = [[0, cos phi], [cos phi, 0]], so the loss is |cos phi|,
    # and the angle between the lines they span is min(phi, 180 - phi).
    phi = math.radians(phi_deg)
    n = 7
    X = np.zeros((n, 2))
    X[2, 0] = 1.0
    X[2, 1], X[5, 1] = math.cos(phi), math.sin(phi)
    assert abs(oracle.ortho_loss(X) - abs(math.cos(phi))) <= 4 * EPS
    assert abs(oracle.mean_angle_deg(X) - min(phi_deg, 180.0 - phi_deg)) <= 1e-9


def test_mean_angle_averages_pairs_and_ortho_loss_sees_norms():
    # e1, e2 and (e1 + e2)/sqrt(2): pair angles 90, 45, 45 -> mean 60.
    X = np.zeros((4, 3))
    X[0, 0] = 1.0
    X[1, 1] = 1.0
    X[0, 2] = X[1, 2] = 1.0 / math.sqrt(2.0)
    assert abs(oracle.mean_angle_deg(X) - 60.0) <= 1e-9
    assert abs(oracle.ortho_loss(X) - 1.0 / math.sqrt(2.0)) <= 4 * EPS
    # A column of norm 2 has |x.x - 1| = 3; orthogonal columns lose nothing.
    Y = np.zeros((5, 2))
    Y[1, 0] = 2.0
    Y[3, 1] = 1.0
    assert oracle.ortho_loss(Y) == 3.0
    assert oracle.mean_angle_deg(Y) == 90.0
    assert oracle.mean_angle_deg(Y[:, :1]) == 90.0     # a single vector has no pairs


def test_relative_residual_of_a_zero_ritz_value_is_the_absolute_one():
    # Sec. IV-D residuals: relative to |theta|, and equal to the absolute
    # residual when theta is exactly zero (no division by zero).
    rp, c, v = synth.path(5)
    y = np.array([1.0, 0.0, 0.0, 0.0, 0.0])[:, None]
    ab, rel = oracle.residuals(rp, c, v, np.array([0.0]), y)
    # A e_0 = e_1, so ||A y - 0 y|| = 1.
    assert ab[0] == 1.0 and rel[0] == 1.0
    ab2, rel2 = oracle.residuals(rp, c, v, np.array([2.0]), y)
    assert ab2[0] == math.sqrt(5.0) and rel2[0] == math.sqrt(5.0) / 2.0


# ------------------------------------------------------ precision emulation
def test_round_bits_24_is_the_binary32_conversion():
    rng = np.random.default_rng(11)
    x = rng.standard_normal(2000) * 10.0 ** rng.integers(-20, 20, 2000)
    want = x.astype(np.float32).astype(np.float64)
    got = np.array([oracle.round_bits(t, 24) for t in x])
    assert np.array_equal(got, want)
    assert oracle.round_bits(0.1, 53) == 0.1


def test_round_bits_8_is_bfloat16_nearest_even():
    one = 1.0
    ulp = 2.0 ** -7                         # bfloat16 spacing in [1, 2)
    cases = [(one + ulp / 2, one),                       # tie -> even (1.0)
             (one + 1.5 * ulp, one + 2 * ulp),           # tie -> even (odd neighbour below)
             (one + ulp / 2 + 2.0 ** -30, one + ulp),    # just above the tie
             (-(one + ulp / 2 + 2.0 ** -30), -(one + ulp)),
             (3.0 * 2.0 ** -40, 3.0 * 2.0 ** -40),       # exactly representable
             (255.5, 256.0)]                             # 8 significant bits: 255.5 is a tie, 256 even
    for x, want in cases:
        assert oracle.round_bits(x, 8) == want, x
    # Against the input module's binary32 -> bfloat16 bit conversion, on
    # values that are binary32 numbers (no double rounding involved).
    rng = np.random.default_rng(12)
    x32 = (rng.standard_normal(3000) * 10.0 ** rng.integers(-8, 8, 3000)).astype(np.float32)
    want = synth.bf16_bits_to_f64(synth.f32_to_bf16_bits(x32))
    got = np.array([oracle.round_bits(float(t), 8) for t in x32])
    assert np.array_equal(got, want)


def test_spmv_emul_accumulates_in_the_given_precision():
    # Row 0: 1 + 2^-30 - 1.  In binary64 the sum is 2^-30; a binary32
    # accumulator absorbs 2^-30 into 1 and returns 0.  Row 1 checks that the
    # products are rounded too: (1 + 2^-30) * 1 -> 1 in binary32.
    rowptr = np.array([0, 3, 4], np.int64)
    col = np.array([0, 1, 0, 1], np.int32)
    val = np.array([1.0, 2.0 ** -30, -1.0, 1.0 + 2.0 ** -30])
    x = np.array([1.0, 1.0])
    y53 = oracle.spmv_emul(rowptr, col, val, x, 53)
    y24 = oracle.spmv_emul(rowptr, col, val, x, 24)
    assert np.array_equal(y53, oracle.spmv(rowptr, col, val, x))
    assert y53[0] == 2.0 ** -30 and y24[0] == 0.0
    assert y53[1] == 1.0 + 2.0 ** -30 and y24[1] == 1.0


@pytest.mark.parametrize("gen", ["er", "rmat", "cycle"])
def test_lanczos_emul_without_rounding_is_the_oracle(gen):
    if gen == "er":
        rp, c, v = synth.er(700, 9.0, seed=4)
    elif gen == "rmat":
        rp, c, v = synth.rmat(10, 8, seed=4)
    else:
        rp, c, v = synth.cycle(40)            # double eigenvalues: restarts
    m = 30
    a1, b1, V1, r1 = oracle.lanczos(rp, c, v, m, seed=4)
    a2, b2, V2, r2 = oracle.lanczos_emul(rp, c, v, m, "fp64", seed=4)
    assert r1 == r2
    assert np.array_equal(a1, a2) and np.array_equal(b1, b2) and np.array_equal(V1, V2)


@pytest.mark.parametrize("mode,bits", [("bf16", 8), ("fp32", 24)])
def test_lanczos_emul_stores_rounded_vectors(mode, bits):
    # Every accepted Lanczos vector is a stored (rounded) vector scaled to
    # unit length: V[:, i] * beta_{i+1} lies on the format's grid (up to the
    # binary64 rounding of the division and product), and the rounding moves
    # the coefficients by about the format's unit roundoff.
    rp, c, v = synth.er(600, 9.0, seed=5)
    m = 20
    a, b, V, r = oracle.lanczos_emul(rp, c, v, m, mode, seed=5)
    assert r == 0
    for i in range(1, m):
        w = V[:, i] * b[i]
        g = np.array([oracle.round_bits(t, bits) for t in w])
        assert np.all(np.abs(g - w) <= 8 * EPS * np.abs(w)), i
    a64, b64, V64, _ = oracle.lanczos(rp, c, v, m, seed=5)
    d = np.max(np.abs(a - a64)) / np.max(np.abs(a64))
    u = 2.0 ** -bits
    assert u / 100 < d < 100 * u, d
