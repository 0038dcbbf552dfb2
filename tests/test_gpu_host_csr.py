"""Host-resident matrices (lanczos_topk_host): the column indices and values
stay in pinned host memory and stream to the device in slabs of whole SpMV
tiles, the leading slabs optionally resident.

  * Against the device-resident solve in the caller's row order: bit for bit
    (eigenvalues, Ritz vectors, Lanczos coefficients, residuals) in the modes
    whose alpha comes from the orthogonalisation, for every slab size and
    resident share, in the three storage precisions, with rows longer than a
    slab, runs of empty rows and restarts.
  * Against the FP64 oracle: eigenvalues 1e-10 and the coefficients, also in
    the one-pass modes (alpha summed slab by slab).
  * The bytes streamed: the resident slabs once, the others once per pass.
  * A bad column index in a late slab is reported before any kernel gathers
    through it.
"""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from gpu_util import device_csr, eig_rel_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2201_07498_amd as lz  # noqa: E402

VB = {"fp64": 8, "fp32": 4, "bf16": 2}


def host_csr(rp, c, v, precision):
    """CPU row pointers; column indices and storage values in new pinned tensors."""
    rpt = torch.from_numpy(np.ascontiguousarray(rp, np.int64))
    ct = torch.from_numpy(np.ascontiguousarray(c, np.int32)).pin_memory()
    s = synth.to_storage(v, precision)
    if precision == "bf16":
        vt = torch.from_numpy(s.view(np.int16)).view(torch.bfloat16).pin_memory()
    else:
        vt = torch.from_numpy(np.ascontiguousarray(s)).pin_memory()
    assert ct.is_pinned() and vt.is_pinned()
    return rpt, ct, vt


def mixed_rows(n=6000, seed=5):
    """Rows of every length class (hubs of 900 to 5000 entries, longer than
    the smallest slab) with runs of empty rows; symmetric."""
    rng = np.random.default_rng(seed)
    edges = set()
    for hub, deg in ((17, 1500), (2048, 5000), (4095, 900), (5999, 4097)):
        for t in rng.choice(n, deg, replace=False):
            if t != hub:
                edges.add((min(hub, t), max(hub, t)))
    for i in range(0, n, 7):
        j = (i * 31 + 5) % n
        edges.add((min(i, j), max(i, j)) if i != j else (i, (i + 1) % n))
    edges = sorted(e for e in edges if e[0] != e[1])
    return synth.from_edges(n, edges, weights=rng.uniform(-1, 1, len(edges)))


CASES = {
    "mixed6000": mixed_rows(),
    "rmat13": synth.rmat(13, 8, seed=21),
    "er5000": synth.er(5000, 9.0, seed=22),
}


def device_solve(rp, c, v, K, m, precision, **kw):
    drp, dc, dv = device_csr(rp, c, v, precision)
    vals, vecs, rep = lz.topk(drp, dc, dv, K, m, precision, reorder="off", **kw)
    torch.cuda.synchronize()
    return vals.cpu(), vecs.cpu(), rep


def host_solve(rp, c, v, K, m, precision, slab, resident, **kw):
    hrp, hc, hv = host_csr(rp, c, v, precision)
    vals, vecs, rep = lz.topk_host(hrp, hc, hv, K, m, precision, slab_nnz=slab, resident_nnz=resident, **kw)
    torch.cuda.synchronize()
    return vals.cpu(), vecs.cpu(), rep


@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("slab,resident", [(2048, 0), (9000, 0), (9000, 20000), (0, 0), (4096, 1 << 40)])
def test_host_resident_equals_device_resident_bitwise(name, precision, slab, resident):
    rp, c, v = CASES[name]
    K, m = 6, 24
    print(f"host-resident {name} {precision} slab={slab} resident={resident}", flush=True)
    a = device_solve(rp, c, v, K, m, precision, seed=4)
    b = host_solve(rp, c, v, K, m, precision, slab, resident, seed=4)
    assert torch.equal(a[0], b[0])
    assert torch.equal(a[1], b[1])
    for key in ("alpha", "beta", "theta", "abs_resid", "resid"):
        assert np.array_equal(a[2][key], b[2][key]), key
    assert a[2]["ortho_loss"] == b[2]["ortho_loss"]
    assert b[2]["restarts"] == a[2]["restarts"] and b[2]["m_eff"] == m
    nnz = int(rp[-1])
    assert b[2]["bytes_streamed"] >= nnz * (4 + VB[precision])
    if resident >= nnz:
        assert b[2]["bytes_streamed"] == nnz * (4 + VB[precision])
    elif resident == 0 and b[2]["restarts"] == 0:
        # m Lanczos steps and the residual product, every entry each time.
        assert b[2]["bytes_streamed"] == (m + 1) * nnz * (4 + VB[precision])


def test_host_resident_share_cuts_the_streamed_bytes():
    rp, c, v = CASES["rmat13"]
    K, m = 6, 24
    nnz = int(rp[-1])
    r0 = host_solve(rp, c, v, K, m, "fp32", 4096, 0, seed=1)[2]
    rh = host_solve(rp, c, v, K, m, "fp32", 4096, nnz // 2, seed=1)[2]
    ra = host_solve(rp, c, v, K, m, "fp32", 4096, nnz, seed=1)[2]
    assert r0["restarts"] == 0
    assert r0["bytes_streamed"] == (m + 1) * nnz * 8
    assert ra["bytes_streamed"] == nnz * 8
    # Whole slabs of at most 4096 entries stay: between nnz/2 - 4096 and nnz/2.
    e_res = (rh["bytes_streamed"] - (m + 1) * nnz * 8) / (-m * 8)
    assert nnz // 2 - 4096 <= e_res <= nnz // 2, e_res


def test_host_resident_fp64_matches_oracle():
    rp, c, v = CASES["mixed6000"]
    K, m = 4, 16
    vals, Y, rep = host_solve(rp, c, v, K, m, "fp64", 2048, 0, seed=3)
    ref = oracle.topk(rp, c, v, K, m, seed=3)
    print(f"host-resident mixed6000 eig rel err {eig_rel_err(vals.numpy(), ref['vals']):.3e}")
    assert rep["restarts"] == ref["restarts"]
    assert eig_rel_err(vals.numpy(), ref["vals"]) <= 1e-10
    np.testing.assert_allclose(rep["alpha"][:m], ref["alpha"], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(rep["beta"][1:m], ref["beta"][1:m], rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(rep["abs_resid"], ref["abs_resid"], rtol=1e-6, atol=1e-12)


@pytest.mark.parametrize("reorth", ["none", "once", "selective"])
def test_host_resident_reorth_modes_match_oracle(reorth):
    # In the one-pass modes alpha is summed from per-workgroup partials of
    # every slab, in slab order.
    rp, c, v = synth.er(4000, 9.0, seed=7)
    K, m = 4, 20
    vals, _, rep = host_solve(rp, c, v, K, m, "fp64", 4096, 8192, seed=7, reorth=reorth)
    passes = {"none": 0, "once": 1, "selective": 2}[reorth]
    ref = oracle.topk(rp, c, v, K, m, seed=7, passes=passes)
    assert eig_rel_err(vals.numpy(), ref["vals"]) <= 1e-9
    np.testing.assert_allclose(rep["alpha"][:m], ref["alpha"], rtol=1e-9, atol=1e-12)


def test_host_resident_restarts_equal_device_resident():
    # Four distinct eigenvalues: the Krylov space is exhausted after four
    # steps and every later step draws a restart vector (slab 0's launch
    # draws it; the other slabs' launches return).
    d = np.repeat([3.0, -2.0, 1.0, 0.5], 1500)
    rp, c, v = synth.diagonal(d)
    K, m = 4, 12
    a = device_solve(rp, c, v, K, m, "fp64", seed=2)
    b = host_solve(rp, c, v, K, m, "fp64", 2048, 0, seed=2)
    assert a[2]["restarts"] > 0
    assert b[2]["restarts"] == a[2]["restarts"]
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


@pytest.mark.parametrize("n", [1, 37, 2049])
def test_host_resident_small_and_ragged(n):
    rp, c, v = synth.path(n) if n > 1 else synth.diagonal([2.5])
    K = 1 if n == 1 else 2
    m = min(n, 8)
    a = device_solve(rp, c, v, K, m, "fp32", seed=5)
    b = host_solve(rp, c, v, K, m, "fp32", 2048, 0, seed=5)
    assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])


def test_host_resident_bad_column_in_a_late_slab_is_reported():
    rp, c, v = CASES["er5000"]
    c = c.copy()
    c[c.size - 10] = rp.size + 5          # out of range, in the last slab
    hrp, hc, hv = host_csr(rp, c, v, "fp64")
    with pytest.raises(lz.LanczosError) as e:
        lz.topk_host(hrp, hc, hv, 4, 12, "fp64", slab_nnz=2048)
    torch.cuda.synchronize()
    assert e.value.code == -1
    # The library stays usable.
    good = host_solve(*CASES["er5000"], 4, 12, "fp64", 2048, 0, seed=0)
    assert good[2]["status"] == 0


def test_host_resident_rejects_device_memory_and_hub_relabelling():
    rp, c, v = CASES["er5000"]
    hrp, hc, hv = host_csr(rp, c, v, "fp64")
    L = lz.lib()
    out = torch.empty(4 + 4 * (rp.size - 1), dtype=torch.float64, device="cuda:0")
    dc = hc.to("cuda:0")
    rc = L.lanczos_topk_host(hrp.data_ptr(), dc.data_ptr(), hv.data_ptr(), rp.size - 1, 4, 12, 0, 0, 0, None,
                             out.data_ptr(), out.data_ptr() + 32, None, None)
    assert rc == -1
    opt = lz.Options()
    L.lz_options_init(ctypes.byref(opt))
    opt.reorder = lz.REORDER["hubs"]
    rc = L.lanczos_topk_host(hrp.data_ptr(), hc.data_ptr(), hv.data_ptr(), rp.size - 1, 4, 12, 0, 0, 0, None,
                             out.data_ptr(), out.data_ptr() + 32, ctypes.byref(opt), None)
    assert rc == -1
