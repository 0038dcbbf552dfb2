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
