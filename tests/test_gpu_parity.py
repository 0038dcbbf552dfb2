"""GPU parity: the HIP library, called through its C ABI, against the FP64 CPU
oracle on the same seeded inputs.

Tolerances:
  * SpMV: per row |y - y_ref| <= c * len * u_acc * sum_k |a_k x_k| (rounding
    of a length-len dot product in the accumulation precision).
  * Eigenvalues: relative error <= 1e-10 (FP64), 1e-6 (FP32 storage),
    1e-3 (BF16 storage), the bounds the solver is specified to meet.
  * Jacobi alone: eigenvalues within 1e-13 ||T||.
"""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import device_csr, device_values, eig_rel_err, multiset_rel_err, subspace_cos, topk_pair_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2201_07498_amd as lz  # noqa: E402

U_ACC = {"fp64": 2.0 ** -53, "fp32": 2.0 ** -24, "bf16": 2.0 ** -24}
EIG_TOL = {"fp64": 1e-10, "fp32": 1e-6, "bf16": 1e-3}


def spmv_cases():
    cases = {}
    cases["er5000"] = synth.er(5000, 9.0, seed=11)
    cases["rmat14"] = synth.rmat(14, 8, seed=12)
    # One hub row with 10 000 non-zeros (three chunks) plus a sparse tail.
    rp, c, v = synth.star(10000)
    cases["star10000"] = (rp, c, np.random.default_rng(3).uniform(0, 1, c.size))
    cases["path3"] = synth.path(3)
    cases["single"] = synth.diagonal([2.5])
    # Rows of every length class, with empty rows between them.
    rng = np.random.default_rng(5)
    n = 6000
    edges = set()
    for hub, deg in ((17, 1500), (2048, 5000), (4095, 900), (5999, 4097)):
        for t in rng.choice(n, deg, replace=False):
            if t != hub:
                edges.add((min(hub, t), max(hub, t)))
    for i in range(0, n, 7):
        edges.add((i, (i * 31 + 5) % n) if i != (i * 31 + 5) % n else (i, (i + 1) % n))
    edges = sorted(e for e in edges if e[0] != e[1])
    cases["mixed6000"] = synth.from_edges(n, edges, weights=rng.uniform(-1, 1, len(edges)))
    # Hub-first relabelling: the longest rows lead and every empty row
    # (isolated vertex) sits at the end.
    cases["rmat14_hubfirst"] = hub_first(*synth.rmat(14, 8, seed=13))
    # Long runs of empty rows before, between and after a few short rows.
    cases["empty_runs"] = rows_with_lengths([0] * 3000 + [3, 1, 2] + [0] * 2500 + [5] + [0] * 4000, seed=6)
    # Row lengths around the 1024-item tile: a row of length L and its end
    # marker take L + 1 items.
    cases["tile_edges"] = rows_with_lengths([1023, 1023, 1, 1022, 1024, 2047, 0, 2048, 3071, 7, 1023], seed=7)
    return cases


def hub_first(rp, c, v):
    """Symmetric relabelling by non-increasing row length (stable)."""
    n = rp.size - 1
    deg = np.diff(rp)
    order = np.argsort(-deg, kind="stable")
    new = np.empty(n, np.int64)
    new[order] = np.arange(n)
    nd = deg[order]
    nrp = np.concatenate([[0], np.cumsum(nd)]).astype(np.int64)
    idx = np.repeat(rp[order] - nrp[:-1], nd) + np.arange(nrp[-1])
    return nrp, new[c[idx]].astype(np.int32), v[idx]


def rows_with_lengths(lens, seed):
    """Square CSR with the given row lengths, random columns and values
    (not symmetric: the SpMV does not need it)."""
    rng = np.random.default_rng(seed)
    n = len(lens)
    rp = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    c = rng.integers(0, n, int(rp[-1])).astype(np.int32)
    return rp, c, rng.uniform(-1, 1, c.size)


SPMV = spmv_cases()


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("name", sorted(SPMV))
def test_spmv_matches_oracle(name, precision):
    rp, c, v = SPMV[name]
    n = rp.size - 1
    print(f"spmv {name} n={n} nnz={rp[-1]} {precision}", flush=True)
    vr = synth.round_values(v, precision)
    x = synth.round_values(np.random.default_rng(1).uniform(-1, 1, n), precision)
    drp, dc, dv = device_csr(rp, c, vr, precision)
    dx = device_values(x, precision)
    y = lz.spmv(drp, dc, dv, dx, precision).double().cpu().numpy()
    want = oracle.spmv(rp, c, vr, x)
    mag = oracle.spmv(rp, c, np.abs(vr), np.abs(x))
    lens = np.diff(rp)
    bound = 2.0 * (lens + 2) * U_ACC[precision] * mag + 1e-300
    assert np.all(np.abs(y - want) <= bound), np.max(np.abs(y - want) / bound)


@pytest.mark.parametrize("m,seed", [(1, 0), (2, 1), (7, 2), (24, 3), (48, 4), (64, 5)])
def test_tridiagonal_jacobi_matches_oracle(m, seed):
    rng = np.random.default_rng(seed)
    a, b = rng.uniform(-2, 2, m), rng.uniform(0.05, 1, max(m - 1, 0))
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    theta, S, sweeps = lz.tridiag_eig(a, b)
    ref, _, _ = oracle.jacobi(T)
    nrm = max(1.0, np.linalg.norm(T, 2))
    assert np.max(np.abs(np.sort(theta) - np.sort(ref))) <= 1e-13 * nrm
    assert np.max(np.abs(S.T @ S - np.eye(m))) <= 1e-13
    assert np.max(np.abs(T @ S - S * theta)) <= 1e-13 * nrm
    assert 1 <= sweeps <= 20


def run_gpu(rp, c, v, K, m, precision="fp64", seed=0, reorth="twice", **kw):
    drp, dc, dv = device_csr(rp, c, v, precision)
    vals, vecs, rep = lz.topk(drp, dc, dv, K, m, precision, seed=seed, reorth=reorth, **kw)
    torch.cuda.synchronize()
    return vals.cpu().numpy(), vecs.cpu().numpy(), rep


def test_fp64_er10000_k8_m24_matches_oracle():
    # Erdos-Renyi n=10 000, ~10 nnz/row, K=8, m=24, seed 0, FP64 everywhere.
    rp, c, v = synth.er(10000, 9.0, seed=0)
    K, m = 8, 24
    vals, Y, rep = run_gpu(rp, c, v, K, m, "fp64", seed=0)
    ref = oracle.topk(rp, c, v, K, m, seed=0)
    err = eig_rel_err(vals, ref["vals"])
    print(f"fp64 er10000 eig rel err {err:.3e} resid {rep['resid'].max():.3e} ortho {rep['ortho_loss']:.2e}")
    assert err <= 1e-10
    np.testing.assert_allclose(rep["alpha"], ref["alpha"], rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(rep["beta"], ref["beta"], rtol=1e-12, atol=1e-13)
    cos = np.abs(np.sum(Y * ref["vecs"], axis=0))
    assert np.all(cos >= 1 - 1e-9), cos
    np.testing.assert_allclose(rep["abs_resid"], ref["abs_resid"], rtol=1e-7)
    assert rep["restarts"] == 0 and rep["m_eff"] == m


@pytest.mark.parametrize("name", ["rmat14_hubfirst", "mixed6000"])
def test_fp64_solve_on_skewed_rows_matches_oracle(name):
    # Hub rows spanning many SpMV tiles and runs of empty rows, through the
    # whole solve: the Lanczos coefficients follow the oracle's.
    rp, c, v = SPMV[name]
    K, m = 4, 16
    vals, Y, rep = run_gpu(rp, c, v, K, m, "fp64", seed=3)
    ref = oracle.topk(rp, c, v, K, m, seed=3)
    print(f"{name}: eig rel err {eig_rel_err(vals, ref['vals']):.3e} restarts {rep['restarts']}")
    assert rep["restarts"] == ref["restarts"]
    assert eig_rel_err(vals, ref["vals"]) <= 1e-10
    np.testing.assert_allclose(rep["alpha"][:m], ref["alpha"], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(rep["beta"][1:m], ref["beta"][1:m], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("reorder", ["off", "hubs"])
@pytest.mark.parametrize("name", ["rmat14", "rmat14_hubfirst", "mixed6000", "empty_runs_sym"])
def test_hub_first_relabelling_matches_oracle(name, reorder):
    # The solve on P A P^T: same Lanczos coefficients (start vector drawn by
    # original index), eigenvalues, and Ritz vectors back in original order.
    if name == "empty_runs_sym":
        rp, c, v = synth.rmat_n(20000, 6.0, seed=21)
        # isolated vertices between the others: every third row emptied
        keep = np.arange(rp.size - 1) % 3 != 0
        rp, c, v = restrict_rows_cols(rp, c, v, keep)
    else:
        rp, c, v = SPMV[name]
    K, m = 6, 20
    drp, dc, dv = device_csr(rp, c, v, "fp64")
    vals, vecs, rep = lz.topk(drp, dc, dv, K, m, "fp64", seed=5, reorder=reorder)
    torch.cuda.synchronize()
    Y = vecs.cpu().numpy()
    ref = oracle.topk(rp, c, v, K, m, seed=5)
    assert rep["reordered"] == (reorder == "hubs")
    assert rep["restarts"] == ref["restarts"]
    assert eig_rel_err(vals.cpu().numpy(), ref["vals"]) <= 1e-10
    np.testing.assert_allclose(rep["alpha"], ref["alpha"], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(rep["beta"][1:m], ref["beta"][1:m], rtol=1e-10, atol=1e-12)
    # Converged pairs: same vector, same sign (largest entry positive).
    conv = ref["rel_resid"] < 1e-8
    dots = np.sum(Y * ref["vecs"], axis=0)
    assert np.all(dots[conv] >= 1 - 1e-8), dots
    np.testing.assert_allclose(rep["abs_resid"], ref["abs_resid"], rtol=1e-6, atol=1e-12)


def restrict_rows_cols(rp, c, v, keep):
    """Zeroes the rows and columns not in `keep` (the matrix keeps its size)."""
    n = rp.size - 1
    rows = np.repeat(np.arange(n), np.diff(rp))
    ok = keep[rows] & keep[c]
    cnt = np.bincount(rows[ok], minlength=n)
    nrp = np.concatenate([[0], np.cumsum(cnt)]).astype(np.int64)
    return nrp, c[ok].astype(np.int32), v[ok]


@pytest.mark.parametrize("kind", ["rmat", "er"])
def test_auto_relabelling_decision(kind):
    # n = 2^17: R-MAT rows are skewed enough to relabel, Erdos-Renyi rows not.
    n = 1 << 17
    if kind == "rmat":
        rp, c, v = synth.rmat(17, 8, seed=4)
    else:
        rp, c, v = synth.er(n, 9.0, seed=4)
    K, m = 4, 16
    drp, dc, dv = device_csr(rp, c, v, "fp64")
    vals, vecs, rep = lz.topk(drp, dc, dv, K, m, "fp64", seed=1)
    torch.cuda.synchronize()
    assert rep["reordered"] == (kind == "rmat")
    ref = oracle.topk(rp, c, v, K, m, seed=1)
    assert eig_rel_err(vals.cpu().numpy(), ref["vals"]) <= 1e-10
    np.testing.assert_allclose(rep["alpha"], ref["alpha"], rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("n", [1, 2, 5, 37, 2047, 2049, 4097])
def test_ragged_sizes(n):
    rp, c, v = synth.er(n, min(9.0, max(n - 1, 0)), seed=n)
    m = min(n, 10)
    K = min(m, 3)
    vals, Y, rep = run_gpu(rp, c, v, K, m, "fp64", seed=2)
    ref = oracle.topk(rp, c, v, K, m, seed=2)
    assert multiset_rel_err(vals, ref["vals"]) <= 1e-10
    assert rep["m_eff"] == m


CLOSED = {
    "complete12": (synth.complete(12), [11.0] + [-1.0] * 11),
    "star9": (synth.star(9), [3.0, -3.0] + [0.0] * 8),
    "cycle20": (synth.cycle(20), [2 * np.cos(2 * np.pi * k / 20) for k in range(20)]),
    "hypercube4": (synth.hypercube(4), [4.0] + [2.0] * 4 + [0.0] * 6 + [-2.0] * 4 + [-4.0]),
    "path25": (synth.path(25), [2 * np.cos(np.pi * k / 26) for k in range(1, 26)]),
}


@pytest.mark.parametrize("name", sorted(CLOSED))
def test_closed_form_spectra_with_restarts(name):
    (rp, c, v), lam = CLOSED[name]
    n = rp.size - 1
    vals, Y, rep = run_gpu(rp, c, v, n, n, "fp64", seed=3)
    ref = oracle.topk(rp, c, v, n, n, seed=3)
    assert np.max(np.abs(np.sort(rep["theta"]) - np.sort(lam))) <= 1e-10 * max(1, np.max(np.abs(lam)))
    assert rep["restarts"] == ref["restarts"]
    assert np.max(np.abs(np.abs(vals) - np.abs(ref["vals"]))) <= 1e-10


@pytest.mark.parametrize("name", sorted(CLOSED))
def test_closed_form_spectra_in_sweep_blocks(name):
    # The same graphs relabelled and forced into sweep blocks: one block
    # (the star's hub row first), restarts drawn by the sweep kernel.
    (rp, c, v), lam = CLOSED[name]
    n = rp.size - 1
    vals, Y, rep = run_gpu(rp, c, v, n, n, "fp64", seed=3, reorder="hubs", sweep="on")
    assert rep["spmv_layout"] == 4
    ref = oracle.topk(rp, c, v, n, n, seed=3)
    assert np.max(np.abs(np.sort(rep["theta"]) - np.sort(lam))) <= 1e-10 * max(1, np.max(np.abs(lam)))
    assert rep["restarts"] == ref["restarts"]
    assert np.max(np.abs(np.abs(vals) - np.abs(ref["vals"]))) <= 1e-10


@pytest.mark.parametrize("n", [2, 5, 37, 2049, 70000])
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ragged_sizes_in_sweep_blocks(n, precision):
    # Forced sweep blocks at sizes from two rows to many blocks (70 000 rows
    # of about 10 entries: 20 blocks in FP64, 40 in FP32, rows cut at every
    # block edge); the oracle solves the same rounded matrix.
    rp, c, v = synth.er(n, min(9.0, max(n - 1, 0)), seed=n)
    v = synth.round_values(v, precision)
    m = min(n, 12)
    K = min(m, 3)
    vals, Y, rep = run_gpu(rp, c, v, K, m, precision, seed=2, reorder="hubs", sweep="on")
    assert rep["spmv_layout"] == 4 and rep["m_eff"] == m
    ref = oracle.topk(rp, c, v, K, m, seed=2)
    assert multiset_rel_err(vals, ref["vals"]) <= EIG_TOL[precision]


def test_deterministic_bitwise():
    rp, c, v = synth.rmat(13, 8, seed=4)
    a = run_gpu(rp, c, v, 6, 20, "fp64", seed=9)
    b = run_gpu(rp, c, v, 6, 20, "fp64", seed=9)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert np.array_equal(a[2]["alpha"], b[2]["alpha"])


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_mixed_precision_er_accuracy(precision):
    rp, c, v = synth.er(10000, 9.0, seed=0)
    v = synth.round_values(v, precision)
    K, m = 8, 24
    vals, Y, rep = run_gpu(rp, c, v, K, m, precision, seed=0)
    ref = oracle.topk(rp, c, v, K, m, seed=0)
    err = eig_rel_err(vals, ref["vals"])
    print(f"{precision} er10000 eig rel err {err:.3e} ortho {rep['ortho_loss']:.2e} resid {rep['resid'].max():.2e}")
    assert err <= EIG_TOL[precision]


@pytest.mark.parametrize("reorth", ["none", "once", "selective"])
def test_reorth_modes_run(reorth):
    rp, c, v = synth.er(4000, 9.0, seed=7)
    K, m = 4, 20
    vals, Y, rep = run_gpu(rp, c, v, K, m, "fp64", seed=7, reorth=reorth)
    passes = {"none": 0, "once": 1, "selective": 2}[reorth]
    ref = oracle.topk(rp, c, v, K, m, seed=7, passes=passes)
    assert eig_rel_err(vals, ref["vals"]) <= 1e-9


def test_profiled_solve_matches_unprofiled_and_fills_timings():
    # Events only observe the stream: results are bitwise those of a solve
    # without them, and the phase times are positive and consistent.
    rp, c, v = synth.rmat(13, 8, seed=4)
    K, m = 6, 20
    drp, dc, dv = device_csr(rp, c, v, "fp32")
    a = lz.topk(drp, dc, dv, K, m, "fp32", seed=9)
    b = lz.topk(drp, dc, dv, K, m, "fp32", seed=9, profile=True)
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    r = b[2]
    for key in ("t_setup_ms", "t_lanczos_ms", "t_spmv_ms", "t_finish_ms"):
        assert r[key] > 0.0, key
    assert r["t_orth_ms"] >= 0.0
    assert m * r["t_spmv_ms"] <= r["t_lanczos_ms"] * 1.05
    assert a[2]["t_lanczos_ms"] == 0.0


def test_reorthogonalisation_keeps_basis_and_ritz_vectors_orthogonal():
    # Sec. IV-D: without reorthogonalisation the basis loses orthogonality
    # once Ritz values converge (ghost copies appear); two passes keep it at
    # rounding level, and the Ritz vectors' mean pairwise angle nearer 90.
    rp, c, v = synth.rmat(14, 8, seed=2)
    K, m = 8, 60
    _, _, r2 = run_gpu(rp, c, v, K, m, "fp64", seed=3, reorth="twice")
    _, _, r0 = run_gpu(rp, c, v, K, m, "fp64", seed=3, reorth="none")
    print(f"ortho twice {r2['ortho_loss']:.2e} none {r0['ortho_loss']:.2e}; "
          f"angle twice {r2['mean_angle_deg']:.4f} none {r0['mean_angle_deg']:.4f}")
    assert r2["ortho_loss"] <= 1e-12
    assert r0["ortho_loss"] >= 1e-6
    assert abs(90.0 - r2["mean_angle_deg"]) <= abs(90.0 - r0["mean_angle_deg"])
    assert r2["ritz_ortho_loss"] <= 1e-10


# All-FP32 arithmetic (dots, norms, reorthogonalisation, SpMV epilogue in
# FP32; FP32 storage).  Sec. IV-D orders the configurations' errors
# all-double < float-storage/double-arithmetic < all-float.  Tolerance of the
# all-float eigenvalues: FP32 sums of n terms carry relative errors of order
# sqrt(n) u_32 (about 1e-5 at n = 1e4 with u_32 = 6e-8), passed on to the
# Lanczos coefficients and the Ritz values.
FFF_TOL = 1e-5


@pytest.mark.parametrize("name", ["er10k", "rmat13"])
def test_all_fp32_arithmetic_accuracy_and_ordering(name):
    rp, c, v = synth.er(10000, 9.0, seed=0) if name == "er10k" else synth.rmat(13, 8, seed=4)
    v = synth.round_values(v, "fp32")
    K, m = 8, 24
    ref = oracle.topk(rp, c, v, K, m, seed=0)
    res = {}
    for label, prec, arith in (("DDD", "fp64", "mixed"), ("FDF", "fp32", "mixed"), ("FFF", "fp32", "fp32")):
        drp, dc, dv = device_csr(rp, c, v, prec)
        vals, _, rep = lz.topk(drp, dc, dv, K, m, prec, seed=0, arith=arith)
        torch.cuda.synchronize()
        res[label] = (eig_rel_err(vals.cpu().numpy(), ref["vals"]), rep["ortho_loss"])
        print(f"{name} {label}: eig err {res[label][0]:.2e} ortho {res[label][1]:.1e}")
    assert res["FFF"][0] <= FFF_TOL
    assert res["DDD"][0] < res["FDF"][0] < res["FFF"][0]
    assert res["DDD"][1] < res["FDF"][1] < res["FFF"][1]


@pytest.mark.parametrize("reorth", ["twice", "selective", "once"])
def test_all_fp32_arithmetic_reorth_modes_and_determinism(reorth):
    rp, c, v = synth.er(6000, 9.0, seed=3)
    v = synth.round_values(v, "fp32")
    K, m = 6, 20
    passes = {"twice": 2, "selective": 2, "once": 1}[reorth]
    ref = oracle.topk(rp, c, v, K, m, seed=5, passes=passes)
    drp, dc, dv = device_csr(rp, c, v, "fp32")
    a = lz.topk(drp, dc, dv, K, m, "fp32", seed=5, reorth=reorth, arith="fp32")
    b = lz.topk(drp, dc, dv, K, m, "fp32", seed=5, reorth=reorth, arith="fp32")
    torch.cuda.synchronize()
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    assert eig_rel_err(a[0].cpu().numpy(), ref["vals"]) <= FFF_TOL


def test_all_fp32_arithmetic_needs_fp32_storage():
    rp, c, v = synth.er(500, 6.0, seed=1)
    for prec in ("fp64", "bf16"):
        drp, dc, dv = device_csr(rp, c, v, prec)
        with pytest.raises(lz.LanczosError):
            lz.topk(drp, dc, dv, 2, 8, prec, arith="fp32")


def test_plain_entry_point_matches_ex():
    rp, c, v = synth.er(3000, 9.0, seed=0)
    drp, dc, dv = device_csr(rp, c, v, "fp64")
    vals, vecs = lz.topk_plain(drp, dc, dv, 4, 12, "fp64")
    vals2, vecs2, _ = lz.topk(drp, dc, dv, 4, 12, "fp64")
    torch.cuda.synchronize()
    assert torch.equal(vals, vals2) and torch.equal(vecs, vecs2)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("n,c", [(1, 1), (300, 5), (1000, 16), (999, 17), (4133, 48), (2048, 64)])
def test_gram_orthogonality_loss_matches_numpy(n, c, precision):
    # MFMA f64 Gram kernel of the report: max |X^T X - I| for a perturbed
    # orthonormal X with a known, non-trivial loss pattern.
    rng = np.random.default_rng(n + c)
    Q, _ = np.linalg.qr(rng.standard_normal((n, c))) if n >= c else (np.ones((1, 1)), None)
    X = Q @ (np.eye(c) + 1e-2 * np.triu(rng.standard_normal((c, c))))
    X = synth.round_values(X, precision).reshape(n, c)
    want = np.max(np.abs(X.T @ X - np.eye(c)))
    dX = device_values(X.T.copy().ravel(), precision).view(c, n).T    # column-major n x c
    got = lz.ortho_loss(dX, precision)
    assert abs(got - want) <= 1e-12 * max(1.0, want), (got, want)


def test_report_metrics_match_oracle_definitions():
    rp, c, v = synth.er(6000, 9.0, seed=5)
    K, m = 6, 30
    vals, Y, rep = run_gpu(rp, c, v, K, m, "fp64", seed=5)
    ref = oracle.topk(rp, c, v, K, m, seed=5)
    assert rep["ortho_loss"] < 1e-13 and ref["ortho_loss"] < 1e-13
    assert abs(rep["ritz_ortho_loss"] - oracle.ortho_loss(Y)) < 1e-13
    assert abs(rep["mean_angle_deg"] - oracle.mean_angle_deg(Y)) < 1e-9
    ab, rel = oracle.residuals(rp, c, v, vals, Y)
    np.testing.assert_allclose(rep["abs_resid"], ab, rtol=1e-9, atol=1e-14)
    np.testing.assert_allclose(rep["resid"], rel, rtol=1e-9, atol=1e-14)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_relabelled_between_2e20_and_2e22_rows_matches_caller_order(precision):
    # 2^20 < n < 2^22: the relabelled copy stores each tile column-sorted
    # (smaller matrices use groups of four tiles).  The solve on P A P^T
    # follows the caller-order solve up to rounding.
    rp, c, v = synth.rmat(21, 4, seed=5)
    n = rp.size - 1
    assert (1 << 20) < n < (1 << 22)
    K, m = 4, 16
    drp, dc, dv = device_csr(rp, c, v, precision)
    a = lz.topk(drp, dc, dv, K, m, precision, seed=2, reorder="hubs")
    b = lz.topk(drp, dc, dv, K, m, precision, seed=2, reorder="off")
    torch.cuda.synchronize()
    assert a[2]["reordered"] and not b[2]["reordered"]
    err = eig_rel_err(a[0].cpu().numpy(), b[0].cpu().numpy())
    print(f"rmat21 {precision}: hub-first vs caller order eig rel err {err:.2e}")
    assert err <= (1e-9 if precision == "fp64" else 1e-5)


def test_two_pass_remeasures_under_strong_cancellation():
    # Six eigenvalue clusters of width ~1e-10: after six steps beta falls to
    # ~1e-9 of ||A v||, far above the breakdown threshold.  Second
    # coefficients taken as c - G c would leave the rounding of c (u ||A v||)
    # in the new vector, an orthogonality loss of about u ||A v|| / beta
    # (~1e-7 here); the two-pass mode re-measures them in that case and keeps
    # the basis orthogonal to rounding level, like the oracle's MGS twice.
    rng = np.random.default_rng(0)
    n = 60
    lam = np.repeat([5.0, 3.0, 1.0, -1.0, -2.5, -4.0], 10) + 1e-10 * rng.standard_normal(n)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    A = (Q * lam) @ Q.T
    A = (A + A.T) / 2
    rp, c, v = synth.dense_to_csr(A)
    K, m = 4, 20
    ref = oracle.topk(rp, c, v, K, m, seed=5)
    vals, Y, rep = run_gpu(rp, c, v, K, m, "fp64", seed=5)
    print(f"clusters: ortho loss gpu {rep['ortho_loss']:.2e} oracle {ref['ortho_loss']:.2e}, "
          f"min beta {np.min(ref['beta'][1:m]):.2e}, restarts {rep['restarts']}")
    assert rep["restarts"] == ref["restarts"] == 0
    assert np.min(ref["beta"][1:m]) < 1e-6 * np.max(np.abs(lam))
    assert rep["ortho_loss"] <= 1e-13 and ref["ortho_loss"] <= 1e-13
    # Past the near-breakdown the Krylov sequence amplifies rounding by about
    # ||A v|| / beta, so only the converged Ritz values are comparable (G21).
    conv = ref["rel_resid"] <= 1e-8
    errs = topk_pair_err(vals, ref["vals"], 1e-9, ref["theta"])
    print(f"clusters: converged {conv}, eig rel err {errs}")
    assert conv.sum() >= 2 and np.all(errs[conv] <= 1e-10)
