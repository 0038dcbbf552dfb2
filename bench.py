"""Benchmark of the Top-K Lanczos eigensolver on one MI355X.

A step is one whole Top-K solve (start vector, m Lanczos iterations with
SpMV + two-pass reorthogonalisation, Jacobi, selection, Ritz vectors,
residual/orthogonality report) on a matrix already resident in HBM.

Default workload: symmetrised R-MAT scale 26 (n = 2^26, edge factor 16,
a/b/c/d = 0.57/0.19/0.19/0.05, duplicates merged, 2.1 billion non-zeros, int64
row pointers), uniform(0,1) weights rounded once to FP32 so the FP32 and FP64
runs see the same matrix; K = 8, m = 32.  The headline is the FP32 storage mode
(FP32 values/basis/SpMV accumulation, FP64 dots, reorth, Jacobi); the FP64
mode runs on the same input for comparison.  Eigenvalue errors are taken
against the FP64 oracle's solve of the same matrix stored in
tests/golden/rmat26.json (written by tests/golden/make_golden.py).  A short
saturation leg of the serving stream (FP32 and FP64 forced) follows unless
--no-serving.

Other workloads (--workload): rmat20 (scale 20, edge factor 8, D^-1/2 A D^-1/2,
K = 16, m = 48, FP32 against FP64), er10k (Erdos-Renyi n = 10 000, K = 8,
m = 24, FP64), rmat23 (scale 23, edge factor 16, BF16 mode against an FP64
run, K = 24, m = 64), serving (a stream of requests through the
continuous-batching server: saturation throughput per precision and Poisson
arrivals at fractions of the FP64 capacity).

Prints one JSON line.  Usage: python bench.py [--steps K] [--warmup W]
[--workload NAME]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SpMV HBM GB/s + Top-K solves/sec, p50/p99 latency at eigval rel err ≤1e-6"
HBM_PEAK_GBPS = 8000.0
BYTES = {"fp64": (8, 8), "fp32": (4, 4), "bf16": (2, 4),   # (stored value/vector bytes, working-vector bytes)
         "fp32-fff": (4, 4)}


def mode_of(p: str):
    """Bench mode -> (storage precision, arithmetic).  "fp32-fff" is FP32
    storage with all-FP32 arithmetic (dots, norms, reorthogonalisation)."""
    return ("fp32", "fp32") if p == "fp32-fff" else (p, "mixed")


def workload(name: str, cache: str | None = None):
    """The workload's matrix; with `cache`, the generated arrays are kept
    there as .npy files and reloaded by later runs."""
    if cache:
        files = [os.path.join(cache, f"{name}.{k}.npy") for k in ("rp", "col", "val")]
        if all(os.path.exists(f) for f in files):
            W = workload_spec(name)
            W.update(rp=np.load(files[0]), col=np.load(files[1]), val=np.load(files[2]).astype(np.float64))
            return W
    W = workload_spec(name)
    W.update(zip(("rp", "col", "val"), generate(name)))
    if cache:
        os.makedirs(cache, exist_ok=True)
        np.save(files[0], W["rp"])
        np.save(files[1], W["col"])
        np.save(files[2], W["val"].astype(np.float32) if name != "er10k" else W["val"])
    return W


def workload_spec(name: str) -> dict:
    if name == "rmat20":
        return dict(K=16, m=48, precisions=("fp32", "fp64", "fp32-fff"),
                    desc="R-MAT scale 20, edge factor 8, (0.57,0.19,0.19,0.05), symmetrised, "
                         "D^-1/2 A D^-1/2, FP32-rounded values")
    if name == "er10k":
        return dict(K=8, m=24, precisions=("fp64",),
                    desc="Erdos-Renyi n=10000, ~10 nnz/row, offdiag U(-1,1), diag U(0,1)")
    if name == "rmat23":
        return dict(K=24, m=64, precisions=("bf16", "fp64"),
                    desc="R-MAT scale 23, edge factor 16, U(0,1) weights rounded to BF16")
    if name == "rmat26":
        return dict(K=8, m=32, precisions=("fp32", "fp64"),
                    desc="R-MAT scale 26, edge factor 16, (0.57,0.19,0.19,0.05), symmetrised, U(0,1) weights "
                         "rounded to FP32")
    raise SystemExit(f"unknown workload {name}")


def generate(name: str):
    import synth
    if name == "rmat20":
        rp, c, v = synth.rmat(20, 8, seed=0)
        v = synth.normalize_sym(rp, c, synth.round_values(v, "fp32"))
        return rp, c, synth.round_values(v, "fp32")
    if name == "er10k":
        return synth.er(10000, 9.0, seed=0)
    if name == "rmat23":
        rp, c, v = synth.rmat(23, 16, seed=0)
        return rp, c, synth.round_values(v, "bf16")
    if name == "rmat26":
        rp, c, v = synth.rmat(26, 16, seed=0)
        return rp, c, synth.round_values(v, "fp32")
    raise SystemExit(f"unknown workload {name}")


def golden(name: str):
    """The FP64 oracle's stored solve of the workload (tests/golden), if any."""
    path = os.path.join(ROOT, "tests", "golden", f"{name}.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        return json.load(fh)


LAYOUTS = {0: "caller's rows", 1: "hub-first rows", 2: "hub-first rows, tiles in column order",
           3: "hub-first rows, tile groups in column order", 4: "hub-first rows, sweep blocks in column order"}


def layout_name(code: int) -> str:
    name = LAYOUTS.get(code & 15, str(code))
    return name + (", x head in LDS" if code & 16 else "")


def spmv_bytes(n: int, nnz: int, precision: str) -> int:
    """Algorithmic HBM bytes of one SpMV step: col + val per non-zero, the
    int64 row pointer, one read of x and of v_{j-1}, one write of w."""
    vb, wb = BYTES[precision]
    return nnz * (4 + vb) + (n + 1) * 8 + n * (2 * vb + wb)


def kernel_source_hash(sweep: bool) -> str:
    """SHA-256 of the sources of the Lanczos-step SpMV kernel, with the
    source that builds the sweep-block layout when the solve used it."""
    import hashlib
    h = hashlib.sha256()
    files = ("lz_spmv.h", "lz_step_spmv.hip", "lz_device.h", "lz_internal.h") + (("lz_sweep.hip",) if sweep else ())
    for f in files:
        with open(os.path.join(ROOT, "paper_2201_07498_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(workload: str, precision: str, sweep: bool):
    """HBM bytes per SpMV launch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE, each scaled by the copy-kernel calibration), or
    None when no summary matches this workload or the kernel sources changed
    since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"k_spmv_step-{workload}-{precision}-traffic.md")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for ln in fh:
            if ln.startswith("- ") and ": " in ln:
                k, v = ln[2:].split(": ", 1)
                vals[k.strip()] = v.strip().strip("`")
    if vals.get("source_sha256") != kernel_source_hash(sweep):
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def run_mode(lz, dev_csr, K, m, mode, steps, warmup, ws):
    import torch
    rp, col, val = dev_csr
    precision, arith = mode_of(mode)
    n = rp.numel() - 1
    out = (torch.empty(K, dtype=torch.float64, device=rp.device),
           torch.empty(K, n, dtype=torch.float64, device=rp.device))
    for _ in range(warmup):
        lz.topk(rp, col, val, K, m, precision, seed=0, workspace=ws, out=out, profile=True, arith=arith)
    torch.cuda.synchronize()
    lat, reps = [], []
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        vals, vecs, rep = lz.topk(rp, col, val, K, m, precision, seed=0, workspace=ws, out=out, profile=True,
                                  arith=arith)
        lat.append(time.perf_counter() - ts)
        reps.append(rep)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return dict(elapsed=elapsed, lat=np.array(lat), reps=reps, vals=out[0].cpu().numpy(),
                vecs=out[1].T.cpu().numpy())


# ------------------------------------------------------------ host-resident
PCIE_PEAK_GBPS = 64.0      # PCIe 5.0 x16, one direction


def host_main(args, W, lz, torch, eig_rel_err):
    """The workload's head storage precision with the column indices and
    values in pinned host memory (lanczos_topk_host), streamed in slabs at
    every SpMV, for several shares of the entries kept on the device."""
    import synth
    rp, col, val, K, m = W["rp"], W["col"], W["val"], W["K"], W["m"]
    n, nnz = rp.size - 1, int(rp[-1])
    prec = mode_of(W["precisions"][0])[0]
    vb = BYTES[prec][0]
    dev = torch.device("cuda:0")
    hrp = torch.from_numpy(np.ascontiguousarray(rp, np.int64))
    hc = torch.from_numpy(np.ascontiguousarray(col, np.int32)).pin_memory()
    st = synth.to_storage(val, prec)
    hv = (torch.from_numpy(st.view(np.int16)).view(torch.bfloat16) if prec == "bf16"
          else torch.from_numpy(np.ascontiguousarray(st))).pin_memory()
    # What the host link delivers: pinned -> device copies of 256 MiB.
    src = torch.empty(1 << 28, dtype=torch.uint8).pin_memory()
    dst = torch.empty(1 << 28, dtype=torch.uint8, device=dev)
    for _ in range(2):
        dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(5):
        dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    link = 5 * (1 << 28) / (time.perf_counter() - t) / 1e9
    del src, dst
    print(f"[host] pinned->device copy {link:.1f} GB/s", file=sys.stderr, flush=True)
    ws = torch.empty(lz.host_workspace_size(n, nnz, K, m, prec), dtype=torch.uint8, device=dev)
    out = (torch.empty(K, dtype=torch.float64, device=dev), torch.empty(K, n, dtype=torch.float64, device=dev))
    # The headline: every entry streamed, library slab size.  Then the
    # resident sweep on slabs of nnz/8 entries (residency is by whole slabs).
    sweep_slab = args.slab_nnz or max(2048, -(-nnz // 8))
    cases = [(0.0, args.slab_nnz)] + [(float(x), sweep_slab) for x in args.resident.split(",") if x]
    runs = []
    for f, slab in cases:
        res = nnz if f >= 1.0 else int(f * nnz)
        kw = dict(slab_nnz=slab, resident_nnz=res, seed=0, workspace=ws, out=out, profile=True)
        for _ in range(args.warmup):
            lz.topk_host(hrp, hc, hv, K, m, prec, **kw)
        torch.cuda.synchronize()
        reps = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            reps.append(lz.topk_host(hrp, hc, hv, K, m, prec, **kw)[2])
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        r = reps[-1]
        passes = m + 1 + r["restarts"]
        # Entries kept on the device: the streamed bytes are
        # e_res (4+vb) + passes (nnz - e_res) (4+vb).
        e_res = (passes * nnz * (4 + vb) - r["bytes_streamed"]) / ((passes - 1) * (4 + vb))
        t_spmv = float(np.mean([x["t_spmv_ms"] for x in reps]))
        per_pass = (nnz - e_res) * (4 + vb)
        runs.append(dict(resident_frac=f, slab_nnz=slab or (1 << 24), resident_entries=int(round(e_res)),
                         solves_per_s=args.steps / el,
                         ms_per_solve=el / args.steps * 1e3, spmv_ms=t_spmv,
                         h2d_bytes_per_spmv=int(round(per_pass)),
                         h2d_gbps=per_pass / (t_spmv * 1e-3) / 1e9 if per_pass > 0 else None,
                         bytes_streamed_per_solve=r["bytes_streamed"],
                         finish_ms=float(np.mean([x["t_finish_ms"] for x in reps])),
                         vals=out[0].cpu().numpy()))
        x = runs[-1]
        gb = f"{x['h2d_gbps']:.1f} GB/s" if x["h2d_gbps"] else "no streaming"
        print(f"[host] slab {x['slab_nnz']} resident {f:.2f}: {x['solves_per_s']:.2f} solves/s, "
              f"spmv {t_spmv:.3f} ms ({gb})", file=sys.stderr, flush=True)
    head = runs[0]
    line = {
        "metric": METRIC,
        "value": head["solves_per_s"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_solve"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16"}[prec],
        "data": "synthetic",
        "config": {"workload": f"{args.workload}-host", "description": W["desc"] + "; column indices and values "
                   "in pinned host memory, streamed to the device at every SpMV", "n": n, "nnz": nnz, "K": K,
                   "m": m, "precision": prec, "reorth": "twice", "slab_nnz": head["slab_nnz"],
                   "resident_frac": 0.0, "parallelism": "single-gpu"},
        "roofline": {"bound": "pcie", "kernel": "host-to-device slab copies of the Lanczos-step SpMV",
                     "achieved": head["h2d_gbps"], "peak": PCIE_PEAK_GBPS, "unit": "GB/s",
                     "frac": head["h2d_gbps"] / PCIE_PEAK_GBPS if head["h2d_gbps"] else None,
                     "traffic": None, "bytes_per_launch": head["h2d_bytes_per_spmv"]},
        "link_copy_gbps": link,
        "resident_sweep": [{k: v for k, v in x.items() if k != "vals"} for x in runs[1:]],
        # Every slab size and resident share gives the same solve, bit for bit.
        "identical_across_runs": all(np.array_equal(x["vals"], head["vals"]) for x in runs[1:]),
    }
    if not args.no_cpu and nnz <= 64_000_000:
        import oracle
        t = time.perf_counter()
        ref = oracle.topk(rp, col, val, K, m, seed=0, report=False)
        dt = time.perf_counter() - t
        line["cpu_baseline"] = {"value": 1.0 / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
                                "sample": f"one whole FP64 oracle solve of the same workload ({dt:.1f} s)"}
        line["eig_rel_err"] = eig_rel_err(head["vals"], ref["vals"])
    print(json.dumps(line), flush=True)


# ------------------------------------------------------------------ serving
def serving_pool(n_pool: int, seed: int = 0):
    """Distinct matrices of the request stream: n log-uniform in [1e4, 2e6],
    average degree U[4, 32], R-MAT or ER, weights U(0,1)."""
    import synth
    rng = np.random.default_rng(seed)
    pool = []
    for i in range(n_pool):
        n = int(10 ** rng.uniform(4.0, np.log10(2e6)))
        d = float(rng.uniform(4, 32))
        if rng.random() < 0.5:
            rp, c, v = synth.rmat_n(n, d, seed=seed * 1000 + i)
            kind = "rmat"
        else:
            rp, c, v = synth.er(n, d - 1.0, seed=seed * 1000 + i)
            v = np.abs(v)
            kind = "er"
        v = synth.round_values(v, "fp32")      # FP32 and FP64 requests see one matrix
        pool.append(dict(rp=rp, col=c, val=v, n=n, nnz=int(rp[-1]), kind=kind))
    return pool


def pinned(a):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return t.pin_memory()


def serving_requests(pool, n_req: int, seed: int = 1):
    rng = np.random.default_rng(seed)
    reqs = []
    for i in range(n_req):
        K = int(rng.choice([4, 8, 16]))
        reqs.append(dict(pool=int(rng.integers(len(pool))), K=K, m=3 * K,
                         prec=str(rng.choice(["fp64", "fp32", "bf16"])), seed=i))
    return reqs


CONVERGED_RESID = 1e-6


def fp32_vs_fp64_err(r32, r64) -> dict:
    """Relative difference of the FP32 Ritz values from the FP64 ones, pair by
    pair in Top-K order: the median and maximum over requests of each
    request's largest difference, and the maximum over the pairs the FP64
    solve has converged (relative residual <= CONVERGED_RESID).  Unconverged
    Ritz values of clustered spectra move with the rounding of the Krylov
    sequence in any precision, so the eigenvalue bound is read on the
    converged ones."""
    per_req, conv = [], []
    pairs = 0
    for (v32, _), (v64, res) in zip(r32, r64):
        den = np.maximum(np.abs(v64), 1e-12 * np.max(np.abs(v64)))
        e = np.abs(v32 - v64) / den
        per_req.append(float(np.max(e)))
        ok = np.asarray(res["resid"]) <= CONVERGED_RESID
        pairs += e.size
        conv.extend(e[ok].tolist())
    return {"max": float(np.max(per_req)), "median": float(np.median(per_req)), "pairs": pairs,
            "converged_pairs": len(conv), "max_converged": float(np.max(conv)) if conv else None}


def warm_up_serving(lz, pool_dev, reqs, precisions, budget, args, count: int = 32):
    """Untimed: the first `count` requests in each precision through a server
    of the timed runs' shape, so that no timed run pays first-use costs (code
    loading, first touches of pinned and device memory)."""
    head = reqs[:count]
    for p in precisions:
        run_stream(lz, pool_dev, head, np.zeros(len(head)), p, budget, args.slots, not args.no_graphs)


def run_stream(lz, pool_dev, reqs, arrivals, force_prec, budget, slots, graphs=True):
    """Submits requests at their arrival times (seconds from start) and waits
    for all.  Returns (elapsed_s, latencies_ms, results by index)."""
    srv = lz.Server(budget, max_slots=slots, use_graphs=graphs)
    try:
        t0 = time.perf_counter()
        tickets = []
        for q, ta in zip(reqs, arrivals):
            now = time.perf_counter() - t0
            if ta > now:
                time.sleep(ta - now)
            p = force_prec or q["prec"]
            src = pool_dev[q["pool"]]
            tickets.append(srv.submit(src["rp"], src["col"], src[p], q["K"], q["m"], p, seed=q["seed"]))
        out = []
        for t in tickets:
            vals, _, res = srv.wait(t)
            out.append((vals.copy(), res))
            srv.release(t)
        elapsed = time.perf_counter() - t0
        stats = srv.stats()
    finally:
        srv.close()
    lat = np.array([r["t_done_ms"] - r["t_submit_ms"] for _, r in out])
    return elapsed, lat, out, stats


def serving_saturation(args) -> dict:
    """A short saturation run of the serving stream (every request queued at
    once), FP32 and FP64 forced, on a smaller pool: solves/s, latency and the
    FP32 Ritz values against the FP64 ones."""
    import synth
    import paper_2201_07498_amd as lz
    pool = serving_pool(max(4, args.pool // 2))
    pool_dev = []
    for m_ in pool:
        d = dict(rp=pinned(m_["rp"]), col=pinned(m_["col"]))
        for p in ("fp64", "fp32"):
            d[p] = pinned(synth.to_storage(m_["val"], p))
        pool_dev.append(d)
    reqs = serving_requests(pool, args.serving_requests)
    burst = np.zeros(len(reqs))
    budget = int(args.budget_gb * (1 << 30))
    warm_up_serving(lz, pool_dev, reqs, ("fp32", "fp64"), budget, args)
    out = {}
    vals = {}
    for p in ("fp32", "fp64"):
        el, lat, res, st = run_stream(lz, pool_dev, reqs, burst, p, budget, args.slots, not args.no_graphs)
        out[p] = {"solves_per_s": len(reqs) / el, "latency_ms": {"p50": float(np.percentile(lat, 50)),
                                                                 "p99": float(np.percentile(lat, 99))}}
        vals[p] = res
        print(f"[bench] serving saturation {p}: {len(reqs) / el:.1f} solves/s", file=sys.stderr, flush=True)
    out.update(requests=len(reqs), pool=len(pool), slots=args.slots,
               speedup_fp32_vs_fp64=out["fp32"]["solves_per_s"] / out["fp64"]["solves_per_s"],
               eig_rel_err_fp32_vs_fp64=fp32_vs_fp64_err(vals["fp32"], vals["fp64"]))
    return out


def serving_main(args):
    import synth
    import paper_2201_07498_amd as lz
    t = time.perf_counter()
    pool = serving_pool(args.pool)
    pool_dev = []
    for m_ in pool:
        d = dict(rp=pinned(m_["rp"]), col=pinned(m_["col"]))
        for p in ("fp64", "fp32", "bf16"):
            d[p] = pinned(synth.to_storage(m_["val"], p).view(np.int16) if p == "bf16"
                          else synth.to_storage(m_["val"], p))
        pool_dev.append(d)
    reqs = serving_requests(pool, args.requests)
    print(f"[serving] pool of {len(pool)} matrices (n {min(p['n'] for p in pool)}..{max(p['n'] for p in pool)}), "
          f"{len(reqs)} requests, prepared in {time.perf_counter() - t:.1f}s", file=sys.stderr, flush=True)
    budget = int(args.budget_gb * (1 << 30))
    burst = np.zeros(len(reqs))
    warm_up_serving(lz, pool_dev, reqs, ("fp64", "fp32", "bf16"), budget, args)
    runs = {}
    for name, force in (("fp64", "fp64"), ("fp32", "fp32"), ("mix", None)):
        el, lat, out, st = run_stream(lz, pool_dev, reqs, burst, force, budget, args.slots, not args.no_graphs)
        runs[name] = dict(elapsed=el, lat=lat, out=out, stats=st)
        print(f"[serving] saturation {name}: {len(reqs) / el:.1f} solves/s, p50 {np.percentile(lat, 50):.1f} ms, "
              f"p99 {np.percentile(lat, 99):.1f} ms, arena peak {st['arena_peak'] / 2**30:.1f} GiB",
              file=sys.stderr, flush=True)
    # Poisson arrivals of the mix at fractions of the measured FP64 capacity.
    cap = len(reqs) / runs["fp64"]["elapsed"]
    sweep = []
    for frac in (() if args.saturation_only else (0.5, 0.8, 1.0, 1.5)):
        rate = frac * cap
        arr = np.cumsum(np.random.default_rng(7).exponential(1.0 / rate, len(reqs)))
        el, lat, out, st = run_stream(lz, pool_dev, reqs, arr, None, budget, args.slots, not args.no_graphs)
        sweep.append({"rate_per_s": rate, "fraction_of_fp64_capacity": frac, "solves_per_s": len(reqs) / el,
                      "latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))}})
        print(f"[serving] poisson mix at {rate:.1f} req/s ({frac}x FP64 capacity): {len(reqs) / el:.1f} solves/s, "
              f"p50 {np.percentile(lat, 50):.1f} ms, p99 {np.percentile(lat, 99):.1f} ms", file=sys.stderr, flush=True)
    f = lambda r: {"solves_per_s": len(reqs) / r["elapsed"],
                   "latency_ms": {"p50": float(np.percentile(r["lat"], 50)),
                                  "p99": float(np.percentile(r["lat"], 99))}}
    line = {
        "metric": METRIC,
        "value": len(reqs) / runs["fp32"]["elapsed"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": len(reqs),
        "warmup": 0,
        "ms_per_step": runs["fp32"]["elapsed"] / len(reqs) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "serving", "description": "request stream: R-MAT/ER, n log-uniform in [1e4, 2e6], "
                   "degree U[4,32], K in {4,8,16}, m=3K", "requests": len(reqs), "pool": len(pool),
                   "slots": args.slots, "graphs": not args.no_graphs, "budget_gb": args.budget_gb,
                   "parallelism": "single-gpu"},
        "fp32": f(runs["fp32"]), "fp64": f(runs["fp64"]), "mix": f(runs["mix"]),
        "poisson_mix": sweep,
        "speedup_fp32_vs_fp64": runs["fp64"]["elapsed"] / runs["fp32"]["elapsed"],
        "eig_rel_err_fp32_vs_fp64": fp32_vs_fp64_err(runs["fp32"]["out"], runs["fp64"]["out"]),
        "arena_peak_gib": runs["mix"]["stats"]["arena_peak"] / 2 ** 30,
    }
    print(json.dumps(line), flush=True)


def study_reorth(args, W, lz, torch, device_csr, eig_rel_err):
    """Sec. IV-D accuracy measures (orthogonality of the basis and of the Ritz
    vectors, mean pairwise angle, residuals) and solve time for each
    reorthogonalisation mode, per storage precision and K (m = 3K).  The
    eigenvalue error is against the FP64 two-pass run of the same K."""
    rp, col, val = W["rp"], W["col"], W["val"]
    n, nnz = rp.size - 1, int(rp[-1])
    precs = tuple(dict.fromkeys(("fp64",) + tuple(W["precisions"])))
    ks = (8, 16, 32)
    ws = torch.empty(max(lz.workspace_size(n, nnz, 32, 64, mode_of(p)[0]) for p in precs),
                     dtype=torch.uint8, device="cuda:0")
    rows, ref = [], {}
    for p in precs:
        prec, arith = mode_of(p)
        dcsr = device_csr(rp, col, val, prec, torch.device("cuda:0"))
        for K in ks:
            m = min(3 * K, 64)
            out = (torch.empty(K, dtype=torch.float64, device="cuda:0"),
                   torch.empty(K, n, dtype=torch.float64, device="cuda:0"))
            for mode in ("twice", "selective", "once", "none"):
                try:
                    lz.topk(*dcsr, K, m, prec, seed=0, reorth=mode, workspace=ws, out=out, arith=arith)
                except lz.LanczosError as e:       # e.g. no convergence without reorthogonalisation
                    torch.cuda.synchronize()
                    rows.append({"precision": p, "reorth": mode, "K": K, "m": m, "error": str(e)})
                    print(f"[study] {p} {mode} K={K}: {e}", file=sys.stderr, flush=True)
                    continue
                torch.cuda.synchronize()
                reps = max(1, min(args.steps, 5))
                t = time.perf_counter()
                for _ in range(reps):
                    vals, _, rep = lz.topk(*dcsr, K, m, prec, seed=0, reorth=mode, workspace=ws, out=out, arith=arith)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t) / reps
                v = vals.cpu().numpy()
                if p == "fp64" and mode == "twice":
                    ref[K] = v
                row = {"precision": p, "reorth": mode, "K": K, "m": m, "ms_per_solve": dt * 1e3,
                       "status": rep["status"], "restarts": rep["restarts"],
                       "ortho_loss": rep["ortho_loss"], "ritz_ortho_loss": rep["ritz_ortho_loss"],
                       "mean_angle_deg": rep["mean_angle_deg"], "resid_max": float(np.max(rep["resid"])),
                       "resid_median": float(np.median(rep["resid"])),
                       "eig_rel_err_vs_fp64_twice": eig_rel_err(v, ref[K]) if K in ref else None}
                rows.append(row)
                print(f"[study] {p} {mode:9s} K={K:2d} m={m:2d}: {dt * 1e3:7.2f} ms  ortho {row['ortho_loss']:.1e}"
                      f"  ritz ortho {row['ritz_ortho_loss']:.1e}  angle {row['mean_angle_deg']:.3f}"
                      f"  resid max {row['resid_max']:.1e}  eig err {row['eig_rel_err_vs_fp64_twice']}",
                      file=sys.stderr, flush=True)
        del dcsr
    print(json.dumps({"study": "reorth", "workload": args.workload, "n": n, "nnz": nnz, "rows": rows}), flush=True)


def study_precision(args, lz, torch, device_csr, eig_rel_err):
    """Sec. IV-D precision trade-off: per matrix, solve time and error of the
    all-double (DDD), FP32-storage/FP64-arithmetic (FDF) and all-FP32 (FFF)
    configurations.  Errors are against the FP64 oracle: Ritz values, basis
    orthogonality, and the residual ||A y - theta y|| of the leading pair
    (the pair every configuration converges)."""
    import oracle
    import synth
    mats = [("er n=1e4", lambda: synth.er(10000, 9.0, seed=0)),
            ("er n=1e5", lambda: synth.er(100000, 9.0, seed=1)),
            ("rmat 14", lambda: synth.rmat(14, 8, seed=2)),
            ("rmat 16", lambda: synth.rmat(16, 8, seed=3)),
            ("rmat 18", lambda: synth.rmat(18, 8, seed=4))]
    K, m = 8, 24
    rows = []
    for name, gen in mats:
        rp, col, val = gen()
        val = synth.round_values(val, "fp32")          # every configuration sees one matrix
        n, nnz = rp.size - 1, int(rp[-1])
        ref = oracle.topk(rp, col, val, K, m, seed=0)
        for label, mode in (("DDD", "fp64"), ("FDF", "fp32"), ("FFF", "fp32-fff")):
            prec, arith = mode_of(mode)
            dcsr = device_csr(rp, col, val, prec, torch.device("cuda:0"))
            lz.topk(*dcsr, K, m, prec, seed=0, arith=arith)
            torch.cuda.synchronize()
            reps = max(1, min(args.steps, 10))
            t = time.perf_counter()
            for _ in range(reps):
                vals, _, rep = lz.topk(*dcsr, K, m, prec, seed=0, arith=arith)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / reps
            row = {"matrix": name, "n": n, "nnz": nnz, "config": label, "ms_per_solve": dt * 1e3,
                   "eig_rel_err": eig_rel_err(vals.cpu().numpy(), ref["vals"]),
                   "ortho_loss": rep["ortho_loss"], "ritz_ortho_loss": rep["ritz_ortho_loss"],
                   "lead_abs_resid": float(rep["abs_resid"][0]), "oracle_lead_abs_resid": float(ref["abs_resid"][0])}
            rows.append(row)
            print(f"[study] {name:9s} {label}: {dt * 1e3:7.3f} ms  eig err {row['eig_rel_err']:.2e}  ortho "
                  f"{row['ortho_loss']:.1e}  lead resid {row['lead_abs_resid']:.2e} (oracle "
                  f"{row['oracle_lead_abs_resid']:.2e})", file=sys.stderr, flush=True)
            del dcsr
    print(json.dumps({"study": "precision", "K": K, "m": m, "rows": rows}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat26")
    ap.add_argument("--cache", default=None, help="directory keeping the generated matrix between runs (.npy)")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving saturation leg")
    ap.add_argument("--serving-requests", type=int, default=256,
                    help="requests of the serving saturation leg of the default benchmark")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--requests", type=int, default=512, help="serving: number of requests")
    ap.add_argument("--pool", type=int, default=32, help="serving: distinct matrices")
    ap.add_argument("--slots", type=int, default=8, help="serving: requests in flight")
    ap.add_argument("--budget-gb", type=float, default=64.0, help="serving: HBM arena")
    ap.add_argument("--no-graphs", action="store_true", help="serving: launch kernels directly, no hipGraph")
    ap.add_argument("--saturation-only", action="store_true", help="serving: skip the Poisson arrival sweep")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run a plain copy kernel (1 GiB read + 1 GiB written, three launches) whose "
                         "FETCH_SIZE/WRITE_SIZE counters calibrate the traffic of the other kernels")
    ap.add_argument("--precisions", default=None, help="comma list overriding the workload's precisions")
    ap.add_argument("--host", action="store_true",
                    help="matrix entries in pinned host memory, streamed at every SpMV (lanczos_topk_host)")
    ap.add_argument("--resident", default="0,0.25,0.5,0.75,1",
                    help="host: comma list of the shares of entries kept on the device (slabs of nnz/8)")
    ap.add_argument("--slab-nnz", type=int, default=0,
                    help="host: entries per streamed slab for every run (0: library default, nnz/8 for the sweep)")
    ap.add_argument("--study", default=None, choices=["reorth", "precision"],
                    help="reorth: accuracy and time of the reorthogonalisation modes (none/once/twice/"
                         "selective) for K in {8, 16, 32}, m = 3K, on the workload; precision: all-double, "
                         "FP32 storage and all-FP32 arithmetic on seeded ER and R-MAT matrices against the "
                         "oracle; each prints one JSON line")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the multi-GPU "
              "row-partitioned path is a design, not built", file=sys.stderr)
        sys.exit(2)

    if args.workload == "serving":
        return serving_main(args)
    import torch
    import paper_2201_07498_amd as lz
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from gpu_util import device_csr, eig_rel_err, topk_pair_err

    if args.calibrate_copy:
        src = torch.rand(1 << 28, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.add(src, 0.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    t = time.perf_counter()
    print(f"[bench] generating workload {args.workload}", file=sys.stderr, flush=True)
    W = workload(args.workload, args.cache)
    if args.precisions:
        W["precisions"] = tuple(args.precisions.split(","))
    rp, col, val, K, m = W["rp"], W["col"], W["val"], W["K"], W["m"]
    n, nnz = rp.size - 1, int(rp[-1])
    print(f"[bench] workload {args.workload}: n={n} nnz={nnz} K={K} m={m} (gen {time.perf_counter() - t:.1f}s)",
          file=sys.stderr, flush=True)
    dev = torch.device("cuda:0")
    if args.study == "reorth":
        return study_reorth(args, W, lz, torch, device_csr, eig_rel_err)
    if args.study == "precision":
        return study_precision(args, lz, torch, device_csr, eig_rel_err)
    if args.host:
        return host_main(args, W, lz, torch, eig_rel_err)
    ws_bytes = max(lz.workspace_size(n, nnz, K, m, mode_of(p)[0]) for p in W["precisions"])
    ws = torch.empty(ws_bytes, dtype=torch.uint8, device=dev)

    results = {}
    for p in W["precisions"]:
        dcsr = device_csr(rp, col, val, mode_of(p)[0], dev)
        torch.cuda.synchronize()
        r = run_mode(lz, dcsr, K, m, p, args.steps, args.warmup, ws)
        t_spmv = float(np.mean([x["t_spmv_ms"] for x in r["reps"]]))
        t_orth = float(np.mean([x["t_orth_ms"] for x in r["reps"]]))
        r.update(t_spmv_ms=t_spmv, t_orth_ms=t_orth,
                 t_lanczos_ms=float(np.mean([x["t_lanczos_ms"] for x in r["reps"]])),
                 t_finish_ms=float(np.mean([x["t_finish_ms"] for x in r["reps"]])),
                 t_setup_ms=float(np.mean([x["t_setup_ms"] for x in r["reps"]])),
                 spmv_bytes=spmv_bytes(n, nnz, p))
        r["spmv_gbps"] = r["spmv_bytes"] / (t_spmv * 1e-3) / 1e9
        results[p] = r
        print(f"[bench] {p}: {args.steps / r['elapsed']:.2f} solves/s, spmv {t_spmv * 1e3:.1f} us "
              f"({r['spmv_gbps']:.0f} GB/s), orth {t_orth * 1e3:.1f} us/step", file=sys.stderr, flush=True)
        del dcsr

    head = W["precisions"][0]
    R = results[head]
    rep = R["reps"][-1]
    line = {
        "metric": METRIC,
        "value": args.steps / R["elapsed"],
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": R["elapsed"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "fp32": "f32", "bf16": "bf16", "fp32-fff": "f32"}[head],
        "data": "synthetic",
        "config": {"workload": args.workload, "description": W["desc"], "n": n, "nnz": nnz, "K": K, "m": m,
                   "precision": head, "reorth": "twice", "parallelism": "single-gpu"},
        "spmv_gbps": R["spmv_gbps"],
        "latency_ms": {"p50": float(np.percentile(R["lat"], 50) * 1e3),
                       "p99": float(np.percentile(R["lat"], 99) * 1e3)},
        "phases_ms": {"setup": R["t_setup_ms"], "lanczos": R["t_lanczos_ms"], "spmv_per_step": R["t_spmv_ms"],
                      "orth_per_step": R["t_orth_ms"], "finish": R["t_finish_ms"]},
        "lanczos_steps_per_s": m / (R["t_lanczos_ms"] * 1e-3) if R["t_lanczos_ms"] > 0 else None,
        "resid_max": float(np.max(rep["resid"])),
        "ortho_loss": rep["ortho_loss"],
        "jacobi_sweeps": rep["jacobi_sweeps"],
        "relabelled": rep["reordered"],
        "spmv_layout": layout_name(rep["spmv_layout"]),
        "roofline": {"bound": "hbm", "kernel": f"k_spmv_step (Lanczos step SpMV; {layout_name(rep['spmv_layout'])})",
                     "achieved": R["spmv_gbps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": R["spmv_gbps"] / HBM_PEAK_GBPS, "traffic": None,
                     "bytes_per_launch": R["spmv_bytes"]},
    }
    for p, r in results.items():
        if p == head:
            continue
        line[p] = {"solves_per_s": args.steps / r["elapsed"], "spmv_gbps": r["spmv_gbps"],
                   "latency_ms": {"p50": float(np.percentile(r["lat"], 50) * 1e3),
                                  "p99": float(np.percentile(r["lat"], 99) * 1e3)},
                   "phases_ms": {"lanczos": r["t_lanczos_ms"], "spmv_per_step": r["t_spmv_ms"],
                                 "orth_per_step": r["t_orth_ms"], "finish": r["t_finish_ms"]}}
        line[f"speedup_{head}_vs_{p}"] = line["value"] / line[p]["solves_per_s"]
        if p != "fp64" and "fp64" in results:
            line[p]["eig_rel_err_vs_fp64_gpu"] = eig_rel_err(r["vals"], results["fp64"]["vals"])

    line["roofline"]["traffic"] = measured_traffic(args.workload, head, rep["spmv_layout"] & 15 == 4)
    if "fp64" in results and head != "fp64":
        # The FP64 run is the reference of the reduced-precision mode.
        line[f"eig_rel_err_{head}_vs_fp64_gpu"] = eig_rel_err(R["vals"], results["fp64"]["vals"])
    G = golden(args.workload)
    if G is not None and G["n"] == n and G["nnz"] == nnz and G["recipe"]["K"] == K and G["recipe"]["m"] == m:
        # Against the oracle's stored solve of this matrix, in Top-K order
        # with ties in modulus (within 1e-6) compared as sets.
        ref = G["fp64"]
        for p, r in results.items():
            e = topk_pair_err(r["vals"], np.asarray(ref["vals"]), 1e-6, np.asarray(ref["theta"]))
            line["eig_rel_err" if p == head else f"eig_rel_err_{p}"] = float(e.max())
        line["eig_rel_err_reference"] = "FP64 oracle solve of the same matrix (tests/golden)"
    if not args.no_cpu:
        import oracle
        if nnz <= 64_000_000:
            t = time.perf_counter()
            ref = oracle.topk(rp, col, val, K, m, seed=0, report=False)
            dt = time.perf_counter() - t
            line["cpu_baseline"] = {"value": 1.0 / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
                                    "sample": f"one whole FP64 oracle solve of the same workload ({dt:.1f} s)"}
            for p, r in results.items():
                key = "eig_rel_err" if p == head else f"eig_rel_err_{p}"
                line[key] = eig_rel_err(r["vals"], ref["vals"])
            line["eig_rel_err_reference"] = "FP64 oracle solve of the same matrix, run here"
        else:
            # Bounded sample: the oracle's first two Lanczos steps on the whole
            # matrix, scaled to m steps (its Jacobi and Ritz parts are not
            # timed).  Later steps reorthogonalise against more basis vectors,
            # so a whole oracle solve takes longer than this estimate.
            steps = 2
            t = time.perf_counter()
            oracle.lanczos(rp, col, val, steps, seed=0)
            dt = (time.perf_counter() - t) / steps * m
            line["cpu_baseline"] = {"value": 1.0 / dt, "unit": "solves/s", "cores": 1, "kind": "oracle",
                                    "sample": f"the FP64 oracle's first {steps} Lanczos steps on the whole matrix "
                                              f"(one host core), scaled to m={m} steps ({dt:.0f} s per solve; "
                                              f"later steps cost more, so this overstates the oracle's rate)"}
    if args.workload == "rmat26" and not args.no_serving and args.gpus == 1:
        del ws
        torch.cuda.empty_cache()
        line["serving_saturation"] = serving_saturation(args)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
