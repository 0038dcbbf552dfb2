"""The C ABI library loads and exports every entry point its header declares;
argument errors are reported before any GPU work (runs without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_2201_07498_amd as lz

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lanczos_topk.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([a-z_][a-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "while")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ("lanczos_topk", "lanczos_topk_ex", "lanczos_topk_workspace_size", "lz_options_init",
                 "lz_status_string", "lz_spmv", "lz_tridiag_eig"):
        assert want in names


def test_library_exports_every_declared_symbol():
    L = lz.lib()
    for name in declared_functions():
        assert hasattr(L, name), name


def test_status_strings_and_defaults():
    L = lz.lib()
    assert L.lz_status_string(0) == b"ok"
    assert L.lz_status_string(-1) == b"invalid argument"
    opt = lz.Options()
    L.lz_options_init(ctypes.byref(opt))
    assert opt.reorth == 2 and opt.report == 1 and opt.seed == 0 and not opt.workspace
    assert opt.reorder == lz.REORDER["auto"]
    assert opt.arith == lz.ARITH["mixed"]
    assert opt.sweep == -1


# The solve below is FP64, so the all-FP32 arithmetic (FP32 storage only) is
# rejected as well as out-of-range values.
@pytest.mark.parametrize("field,value", [("reorder", 3), ("reorder", -1), ("reorth", 4), ("arith", 2),
                                         ("arith", -1), ("arith", 1), ("sweep", 2), ("sweep", -2)])
def test_invalid_options_rejected_without_gpu(field, value):
    L = lz.lib()
    d = ctypes.c_void_p(16)
    opt = lz.Options()
    L.lz_options_init(ctypes.byref(opt))
    setattr(opt, field, value)
    assert L.lanczos_topk_ex(d, d, d, 100, 500, 2, 4, 0, None, d, d, ctypes.byref(opt), None) == -1


@pytest.mark.parametrize("n,K,m,prec", [(0, 1, 1, 0), (10, 0, 1, 0), (10, 3, 2, 0), (10, 1, 65, 0),
                                         (10, 4, 11, 0), (10, 1, 2, 3), (10, 1, 2, -1)])
def test_invalid_arguments_rejected_without_gpu(n, K, m, prec):
    L = lz.lib()
    dummy = ctypes.c_void_p(16)
    rc = L.lanczos_topk(dummy, dummy, dummy, n, K, m, prec, None, dummy, dummy)
    assert rc == -1
    rc = L.lanczos_topk_ex(dummy, dummy, dummy, n, 100, K, m, prec, None, dummy, dummy, None, None)
    assert rc == -1


def test_null_pointers_rejected():
    L = lz.lib()
    d = ctypes.c_void_p(16)
    assert L.lanczos_topk(None, d, d, 10, 1, 2, 0, None, d, d) == -1
    assert L.lanczos_topk_ex(d, d, d, 10, 5, 1, 2, 0, None, None, d, None, None) == -1
    assert L.lz_spmv(d, None, d, 10, 5, 0, d, d, None) == -1
    assert L.lz_tridiag_eig(None, None, 3, None, None, None) == -1


def test_workspace_size_grows_with_shape():
    a = lz.workspace_size(10000, 100000, 8, 24, "fp64")
    b = lz.workspace_size(10000, 100000, 8, 24, "fp32")
    c = lz.workspace_size(20000, 200000, 8, 24, "fp64")
    assert a > 10000 * 25 * 8 and b < a and c > a
    assert lz.workspace_size(0, 1, 1, 1, "fp64") == 0


def test_workspace_size_of_the_sweep_blocks():
    # Opted in below the automatic size: columns, rows within the block,
    # values and the sort positions per entry (10 + 4 bytes in FP32), the
    # sort's scratch and the block table on top of the default.
    n, nnz = 100000, 1000000
    base = lz.workspace_size(n, nnz, 8, 24, "fp32")
    assert lz.workspace_size(n, nnz, 8, 24, "fp32", sweep="auto") == base
    assert lz.workspace_size(n, nnz, 8, 24, "fp32", sweep="off") == base
    on = lz.workspace_size(n, nnz, 8, 24, "fp32", sweep="on")
    assert on >= base + nnz * (10 + 4 + 8)
    # No relabelling, no sweep blocks.
    assert lz.workspace_size(n, nnz, 8, 24, "fp32", sweep="on", reorder="off") == base
    # FP64 values take 4 more bytes per entry (its blocks are twice as long,
    # so its block table is shorter).
    on64 = lz.workspace_size(n, nnz, 8, 24, "fp64", sweep="on")
    assert on64 - lz.workspace_size(n, nnz, 8, 24, "fp64") >= on - base + 4 * nnz - 4096
    # Invalid options: size 0.
    opt = lz.Options()
    lz.lib().lz_options_init(ctypes.byref(opt))
    opt.sweep = 3
    assert lz.lib().lanczos_topk_workspace_size_opt(n, nnz, 8, 24, 1, ctypes.byref(opt)) == 0
    # The automatic choice: x of at least 64 MiB (FP32: n >= 2^24).
    big = 1 << 24
    assert (lz.workspace_size(big, 16 * big, 8, 32, "fp32")
            >= lz.workspace_size(big, 16 * big, 8, 32, "fp32", sweep="off") + 16 * big * 14)
    assert (lz.workspace_size(big // 2, 16 * big, 8, 32, "fp32")
            == lz.workspace_size(big // 2, 16 * big, 8, 32, "fp32", sweep="off"))


def _host_rowptr(n, nnz):
    import numpy as np
    rp = np.linspace(0, nnz, n + 1).astype(np.int64)
    rp[-1] = nnz
    return rp


@pytest.mark.parametrize("case", ["K0", "m_gt_n", "slab_small", "resident_neg", "too_many_slabs", "rowptr0",
                                  "hubs", "null_out"])
def test_host_resident_arguments_rejected_before_gpu_work(case):
    import numpy as np
    L = lz.lib()
    d = ctypes.c_void_p(16)
    n, nnz, K, m, slab, res = 100, 1000, 2, 4, 4096, 0
    rp = _host_rowptr(n, nnz)
    opt = lz.Options()
    L.lz_options_init(ctypes.byref(opt))
    out = d
    if case == "K0":
        K = 0
    elif case == "m_gt_n":
        n, m = 3, 4
        rp = _host_rowptr(n, nnz)
    elif case == "slab_small":
        slab = 2047
    elif case == "resident_neg":
        res = -1
    elif case == "too_many_slabs":
        rp = _host_rowptr(n, 1 << 26)          # 2^26 entries in slabs of 2048: more than 16384 slabs
        slab = 2048
    elif case == "rowptr0":
        rp = rp.copy()
        rp[0] = 1
    elif case == "hubs":
        opt.reorder = lz.REORDER["hubs"]
    elif case == "null_out":
        out = None
    rc = L.lanczos_topk_host(rp.ctypes.data, d, d, n, K, m, 0, slab, res, None, out, d, ctypes.byref(opt), None)
    assert rc == -1, case


def test_host_resident_rejects_pageable_entries():
    """Column indices and values in ordinary (pageable) host memory are
    refused: the streamed copies need page-locked memory."""
    import numpy as np
    L = lz.lib()
    n, nnz = 100, 1000
    rp = _host_rowptr(n, nnz)
    col = np.zeros(nnz, dtype=np.int32)
    val = np.zeros(nnz, dtype=np.float64)
    d = ctypes.c_void_p(16)
    rc = L.lanczos_topk_host(rp.ctypes.data, col.ctypes.data, val.ctypes.data, n, 2, 4, 0, 0, 0, None, d, d,
                             None, None)
    assert rc == -1


def test_caller_workspace_checked_against_the_sweep_plan():
    # A workspace sized for the default options is too small once sweep
    # blocks are asked for; the size from workspace_size(..., sweep="on") is
    # accepted up to the point where the call would touch the GPU.  Both
    # checks happen before any device work (dummy device pointers).
    L = lz.lib()
    d = ctypes.c_void_p(16)
    n, nnz, K, m = 100000, 1000000, 4, 12
    opt = lz.Options()
    L.lz_options_init(ctypes.byref(opt))
    opt.sweep = 1
    opt.reorder = lz.REORDER["hubs"]
    need = lz.workspace_size(n, nnz, K, m, "fp32", sweep="on", reorder="hubs")
    assert need > lz.workspace_size(n, nnz, K, m, "fp32")
    opt.workspace = d
    opt.workspace_bytes = lz.workspace_size(n, nnz, K, m, "fp32")
    for entry in ("lanczos_topk_ex", "lanczos_topk_async"):
        last = None if entry == "lanczos_topk_ex" else ctypes.c_void_p(0)
        rc = getattr(L, entry)(d, d, d, n, nnz, K, m, 1, None, d, d, ctypes.byref(opt), last)
        assert rc == -4, (entry, rc)                       # LZ_ERR_WORKSPACE_TOO_SMALL
    opt.workspace_bytes = need - 1
    assert L.lanczos_topk_async(d, d, d, n, nnz, K, m, 1, None, d, d, ctypes.byref(opt), None) == -4


def test_host_workspace_excludes_the_relabelled_copy():
    n, nnz = 100000, 2000000
    for prec, vb in (("fp64", 8), ("fp32", 4), ("bf16", 2)):
        dev = lz.workspace_size(n, nnz, 8, 24, prec)
        host = lz.host_workspace_size(n, nnz, 8, 24, prec)
        assert 0 < host < dev
        assert dev - host >= nnz * (4 + vb) + 2 * n * 4 - 4 * 256
    assert lz.host_workspace_size(0, 1, 1, 1, "fp64") == 0


def test_async_entry_point_rejects_bad_arguments_before_gpu_work():
    L = lz.lib()
    d = ctypes.c_void_p(16)
    opt = lz.Options()
    L.lz_options_init(ctypes.byref(opt))
    assert opt.max_restarts == -1
    assert L.lanczos_topk_async(d, d, d, 100, 500, 3, 2, 0, None, d, d, ctypes.byref(opt), None) == -1
    assert L.lanczos_topk_async(d, d, d, 100, 500, 2, 4, 0, None, None, d, ctypes.byref(opt), None) == -1
    opt.profile = 1                       # timings need host-side events
    assert L.lanczos_topk_async(d, d, d, 100, 500, 2, 4, 0, None, d, d, ctypes.byref(opt), None) == -1
    opt.profile = 0
    opt.max_restarts = 129                # above LZ_MAX_RESTART_BUDGET
    assert L.lanczos_topk_async(d, d, d, 100, 500, 2, 4, 0, None, d, d, ctypes.byref(opt), None) == -1
    opt.max_restarts = 0
    opt.workspace = d
    opt.workspace_bytes = 1024            # far too small
    assert L.lanczos_topk_async(d, d, d, 100, 500, 2, 4, 0, None, d, d, ctypes.byref(opt), None) == -4
    assert L.lz_status_string(-9).startswith(b"more breakdowns")


def test_report_struct_matches_the_header_layout():
    # lz_report: 4 ints, beta_last, 2 x 64 residuals, 3 metrics, alpha[64],
    # beta[65], theta[64], 5 timings, 2 ints, bytes_streamed.
    assert lz.REPORT_BYTES == 4 * 4 + 8 + 2 * 64 * 8 + 3 * 8 + 64 * 8 + 65 * 8 + 64 * 8 + 5 * 8 + 2 * 4 + 8


def test_check_symmetric():
    import numpy as np
    import synth
    rp, c, v = synth.rmat(10, 8, seed=3)
    for prec in ("fp64", "fp32", "bf16"):
        assert lz.check_symmetric(rp, c, synth.to_storage(v, prec), prec) == (True, -1)
    # One value changed: its row (or its mirror's) is reported.
    w = v.copy()
    w[rp[5]] += 0.25
    ok, bad = lz.check_symmetric(rp, c, w, "fp64")
    assert not ok and bad in (5, int(c[rp[5]]))
    assert lz.check_symmetric(rp, c, w, "fp64", rtol=1.0)[0]
    # Duplicates are summed: split one entry of an off-diagonal pair in two.
    r = 7
    e = int(rp[r])
    rp2 = rp.copy()
    rp2[r + 1:] += 1
    c2 = np.insert(c, e + 1, c[e])
    v2 = np.insert(v, e + 1, 0.5 * v[e])
    v2[e] = 0.5 * v[e]
    assert lz.check_symmetric(rp2, c2, v2, "fp64", rtol=1e-15)[0]
    # A one-sided entry is caught; a column index outside [0, n) is an error.
    p = synth.from_edges(4, [(0, 1)])
    c3 = p[1].copy()
    c3[0] = 2
    assert not lz.check_symmetric(p[0], c3, p[2], "fp64")[0]
    c3[0] = 9
    with pytest.raises(lz.LanczosError):
        lz.check_symmetric(p[0], c3, p[2], "fp64")


def test_ctypes_structs_match_the_c_header(tmp_path):
    # The binding's Options and Report mirror lz_options and lz_report: same
    # size and field offsets as a C compiler lays them out from the header.
    import subprocess
    src = tmp_path / "layout.c"
    fields = {"lz_report": [f for f, _ in lz.Report._fields_], "lz_options": [f for f, _ in lz.Options._fields_]}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for st, fs in fields.items():
        lines.append(f'printf("{st} %zu\\n", sizeof({st}));')
        for f in fs:
            lines.append(f'printf("{st}.{f} %zu\\n", offsetof({st}, {f}));')
    lines += ["return 0;", "}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-o", str(exe), str(src)])
    got = dict(line.split() for line in subprocess.check_output([str(exe)]).decode().splitlines())
    for st, cls in (("lz_report", lz.Report), ("lz_options", lz.Options)):
        assert int(got[st]) == ctypes.sizeof(cls), st
        for f in fields[st]:
            assert int(got[f"{st}.{f}"]) == getattr(cls, f).offset, (st, f)
