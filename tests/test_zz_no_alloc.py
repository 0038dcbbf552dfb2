"""lanczos_topk_noalloc, the entry point that allocates nothing (its
workspace is the library's fixed device scratch array), against
lanczos_topk_async with a caller workspace: bit for bit, on two calls in a
row, the second on a smaller input."""
import ctypes

import numpy as np
import pytest

import synth
from gpu_util import device_csr

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2201_07498_amd as lz  # noqa: E402


def _solve_both(rp, c, v, K, m, prec, seed, **kw):
    drp, dc, dv = device_csr(rp, c, v, prec)
    n = rp.size - 1
    ws = torch.empty(lz.workspace_size(n, c.size, K, m, prec, **kw), dtype=torch.uint8, device="cuda:0")
    assert ws.numel() <= lz.noalloc_max_bytes()
    a = lz.topk_async(drp, dc, dv, K, m, prec, seed=seed, workspace=ws, **kw)
    b = lz.topk_noalloc(drp, dc, dv, K, m, prec, seed=seed, **kw)
    torch.cuda.synchronize()
    return a, b


def test_noalloc_matches_async_on_two_calls_second_smaller():
    first = synth.rmat(15, 8, seed=1)
    second = synth.er(3000, 9.0, seed=2)
    for (rp, c, v), K, m, prec in ((first, 8, 24, "fp32"), (second, 4, 12, "fp64")):
        print(f"noalloc n={rp.size - 1} nnz={c.size} K={K} m={m} {prec}", flush=True)
        a, b = _solve_both(rp, c, v, K, m, prec, seed=5)
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
        ra, rb = lz.report_from_device(a[2], K, m), lz.report_from_device(b[2], K, m)
        assert ra["status"] == rb["status"] == 0
        for key in ("alpha", "beta", "theta", "resid", "abs_resid"):
            assert np.array_equal(ra[key], rb[key]), key
        for key in ("restarts", "m_eff", "ortho_loss", "ritz_ortho_loss", "mean_angle_deg", "spmv_layout"):
            assert ra[key] == rb[key], key


def test_noalloc_matches_async_with_sweep_blocks():
    # The sweep-block layout (opted in) puts the segmented sort's scratch in
    # the array too; two calls, the second smaller.
    for (rp, c, v), prec in ((synth.rmat(14, 8, seed=3), "fp32"), (synth.rmat(12, 8, seed=4), "bf16")):
        print(f"noalloc sweep n={rp.size - 1} nnz={c.size} {prec}", flush=True)
        a, b = _solve_both(rp, c, v, 6, 20, prec, seed=2, sweep="on", reorder="hubs")
        assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
        ra, rb = lz.report_from_device(a[2], 6, 20), lz.report_from_device(b[2], 6, 20)
        assert ra["status"] == rb["status"] == 0 and ra["spmv_layout"] == rb["spmv_layout"] == 4
        for key in ("alpha", "beta", "theta", "resid", "abs_resid"):
            assert np.array_equal(ra[key], rb[key]), key


def test_noalloc_rejects_sizes_beyond_the_scratch_array():
    L = lz.lib()
    n, nnz, K, m = 1 << 22, 40 << 20, 8, 24
    assert lz.workspace_size(n, nnz, K, m, "fp64") > lz.noalloc_max_bytes()
    d = ctypes.c_void_p(16)
    assert L.lanczos_topk_noalloc(d, d, d, n, nnz, K, m, 0, None, d, d, None, None) == -5   # LZ_ERR_TOO_LARGE
    opt = lz.Options()
    L.lz_options_init(ctypes.byref(opt))
    opt.workspace = d
    opt.workspace_bytes = 1 << 30
    assert L.lanczos_topk_noalloc(d, d, d, 1000, 5000, 2, 4, 0, None, d, d, ctypes.byref(opt), None) == -1
