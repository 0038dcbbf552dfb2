"""The stream-ordered entry point lanczos_topk_async: results bit for bit those
of the blocking lanczos_topk_ex, breakdowns absorbed by the enqueued restart
budget, the report written to device memory, and the call captured in a
hipGraph and replayed."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import device_csr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2201_07498_amd as lz  # noqa: E402

KEYS = ("status", "m_eff", "restarts", "jacobi_sweeps", "beta_last", "resid", "abs_resid", "ortho_loss",
        "ritz_ortho_loss", "mean_angle_deg", "alpha", "beta", "theta", "reordered", "spmv_layout")


def same_report(a, b):
    for k in KEYS:
        x, y = a[k], b[k]
        if isinstance(x, np.ndarray):
            assert np.array_equal(x, y), k
        else:
            assert x == y, (k, x, y)


CASES = {
    "er_fp64": (lambda: synth.er(5000, 9.0, seed=2), "fp64", 6, 20),
    "rmat14_fp32": (lambda: synth.rmat(14, 8, seed=3), "fp32", 8, 24),
    # n = 2^20 in BF16: the SpMV variant with the head of x in LDS applies to
    # the relabelled matrix only, so both variants are enqueued and the
    # device's row-order decision picks one (R-MAT: relabelled; ER: not).
    "rmat20_bf16": (lambda: synth.rmat(20, 2, seed=4), "bf16", 4, 12),
    "er20_bf16": (lambda: synth.er(1 << 20, 5.0, seed=4), "bf16", 4, 12),
    # Sweep blocks (opted in; 20 blocks in FP64, 40 in FP32 and BF16, rows
    # split at their edges):
    # the row sums are LDS atomics in one wavefront's fixed order, so two
    # solves agree bit for bit.
    "rmat16_fp32_sweep": (lambda: synth.rmat(16, 8, seed=3), "fp32", 8, 24, dict(sweep="on", reorder="hubs")),
    "rmat16_fp64_sweep": (lambda: synth.rmat(16, 8, seed=3), "fp64", 8, 24, dict(sweep="on", reorder="hubs")),
    "rmat16_bf16_sweep": (lambda: synth.rmat(16, 8, seed=3), "bf16", 8, 24, dict(sweep="on", reorder="hubs")),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_async_matches_blocking_bitwise(name):
    gen, prec, K, m = CASES[name][:4]
    kw = CASES[name][4] if len(CASES[name]) > 4 else {}
    rp, c, v = gen()
    print(f"async {name} n={rp.size - 1} nnz={c.size}", flush=True)
    drp, dc, dv = device_csr(rp, c, v, prec)
    a_vals, a_vecs, a_rep = lz.topk(drp, dc, dv, K, m, prec, seed=7, **kw)
    b_vals, b_vecs, d_rep = lz.topk_async(drp, dc, dv, K, m, prec, seed=7, **kw)
    torch.cuda.synchronize()
    b_rep = lz.report_from_device(d_rep, K, m)
    assert torch.equal(a_vals, b_vals) and torch.equal(a_vecs, b_vecs)
    same_report(a_rep, b_rep)
    assert b_rep["status"] == 0 and b_rep["m_eff"] == m
    if name == "rmat20_bf16":
        assert b_rep["spmv_layout"] == 3 | 16          # group-sorted, x head in LDS
    if name == "er20_bf16":
        assert b_rep["spmv_layout"] == 0
    if name.endswith("_sweep"):
        assert b_rep["spmv_layout"] == 4
        # A second blocking solve repeats the first exactly.
        c_vals, c_vecs, _ = lz.topk(drp, dc, dv, K, m, prec, seed=7, **kw)
        assert torch.equal(a_vals, c_vals) and torch.equal(a_vecs, c_vecs)


@pytest.mark.parametrize("sweep", [None, "on"])
def test_async_restart_budget(sweep):
    # K_12 (eigenvalues 11 and -1 x 11): the Krylov space of the start vector
    # has dimension 2, so m = 12 steps take 10 restarts.  With sweep blocks
    # (relabelled, one block) the restart draws come from that SpMV kernel.
    rp, c, v = synth.complete(12)
    K = m = 12
    kw = {} if sweep is None else dict(sweep=sweep, reorder="hubs")
    ref = oracle.topk(rp, c, v, K, m, seed=3)
    drp, dc, dv = device_csr(rp, c, v, "fp64")
    a_vals, a_vecs, a_rep = lz.topk(drp, dc, dv, K, m, "fp64", seed=3, **kw)
    b_vals, b_vecs, d_rep = lz.topk_async(drp, dc, dv, K, m, "fp64", seed=3, **kw)
    torch.cuda.synchronize()
    b_rep = lz.report_from_device(d_rep, K, m)
    assert a_rep["restarts"] == b_rep["restarts"] == ref["restarts"] >= 8
    assert torch.equal(a_vals, b_vals) and torch.equal(a_vecs, b_vecs)
    same_report(a_rep, b_rep)
    # A budget below the restarts needed: the report says so and the solve
    # stops before the finish.
    if sweep:
        assert b_rep["spmv_layout"] == 4
    _, _, d2 = lz.topk_async(drp, dc, dv, K, m, "fp64", seed=3, max_restarts=ref["restarts"] - 1, **kw)
    torch.cuda.synchronize()
    r2 = lz.report_from_device(d2, K, m)
    assert r2["status"] == -9 and r2["m_eff"] < m


def test_async_reports_invalid_columns_in_device_report():
    rp, c, v = synth.er(2000, 6.0, seed=1)
    c = c.copy()
    c[17] = 2000                                        # outside [0, n)
    drp, dc, dv = device_csr(rp, c, v, "fp64")
    _, _, d_rep = lz.topk_async(drp, dc, dv, 2, 8, "fp64")
    torch.cuda.synchronize()
    assert lz.report_from_device(d_rep, 2, 8)["status"] == -1


@pytest.mark.parametrize("sweep", [None, "on"])
def test_async_in_hip_graph_replays_bitwise(sweep):
    # The whole solve captured in one graph on a torch stream; replays, with
    # other eager solves and synchronisations between them, reproduce the
    # eager result exactly.  With sweep blocks the capture holds the
    # segmented sort of the setup too.
    rp, c, v = synth.rmat(13, 8, seed=5)
    rp2, c2, v2 = synth.er(3000, 9.0, seed=6)
    K, m = 6, 20
    n = rp.size - 1
    kw = {} if sweep is None else dict(sweep=sweep, reorder="hubs")
    drp, dc, dv = device_csr(rp, c, v, "fp32")
    ws = torch.empty(lz.workspace_size(n, c.size, K, m, "fp32", **kw), dtype=torch.uint8, device="cuda:0")
    out = (torch.empty(K, dtype=torch.float64, device="cuda:0"),
           torch.empty(K, n, dtype=torch.float64, device="cuda:0"))
    d_rep = torch.empty(lz.REPORT_BYTES, dtype=torch.uint8, device="cuda:0")
    e_vals, e_vecs, e_rep = lz.topk(drp, dc, dv, K, m, "fp32", seed=11, workspace=ws, **kw)
    if sweep:
        assert e_rep["spmv_layout"] == 4
    e_vals, e_vecs = e_vals.clone(), e_vecs.clone()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            lz.topk_async(drp, dc, dv, K, m, "fp32", seed=11, workspace=ws, out=out, d_report=d_rep,
                          stream=side, **kw)
    torch.cuda.current_stream().wait_stream(side)
    other = device_csr(rp2, c2, v2, "fp64")
    for rep_i in range(3):
        out[0].zero_()
        out[1].zero_()
        d_rep.zero_()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out[0], e_vals), rep_i
        assert torch.equal(out[1].T, e_vecs), rep_i
        same_report(e_rep, lz.report_from_device(d_rep, K, m))
        lz.topk(*other, 4, 12, "fp64", seed=rep_i)       # eager work between replays
        torch.cuda.synchronize()
