"""Writes the oracle's expected values for the large benchmark workloads.

The GPU tests at these sizes cannot afford the FP64 oracle at run time (about
a minute per solve at R-MAT scale 23 and four minutes at scale 26 on one host
core), so this script runs it once and stores what the tests compare against.
It calls only the seeded input generators (``synth``) and the CPU oracle
(``oracle``); nothing here comes from the GPU library.

Stored per workload (JSON, floats written exactly):
  * the recipe (generator call, rounding, K, m, seed) and n, nnz;
  * the oracle solve (Algorithm 1 with two modified Gram-Schmidt passes, Jacobi
    on T, Top-K by modulus, Ritz vectors and the Sec. IV-D report): the K
    eigenvalues, all m Ritz values, alpha, beta, absolute and relative
    residuals, orthogonality losses, restarts;
  * Ritz-vector entries at seeded sample rows and at each vector's entry of
    largest modulus (the sign rule), so vectors can be compared entry by entry
    without storing n*K values;
  * optionally the same solve with the Lanczos phase emulating a reduced
    storage precision (``oracle.topk(..., emulate=...)``: stored vectors
    rounded to BF16 or FP32, SpMV accumulated in FP32), which predicts how far
    that mode's Ritz values can be from the FP64 ones.

Workloads:
  rmat21  R-MAT scale 21, edge factor 4, seed 5, weights rounded to BF16; K = 4,
          m = 16; FP64 oracle and BF16 emulation
  rmat20  R-MAT scale 20, edge factor 8, FP32-rounded weights, D^-1/2 A D^-1/2,
          rounded to FP32 then to BF16 (the BF16-mode input); K = 16, m = 48;
          FP64 oracle and BF16 emulation
  rmat23  R-MAT scale 23, edge factor 16, weights rounded to BF16; K = 24,
          m = 64; FP64 oracle and BF16 emulation
  rmat26  R-MAT scale 26, edge factor 16, weights rounded to FP32; K = 8,
          m = 32; FP64 oracle (needs about 90 GB of host memory)

Usage: python tests/golden/make_golden.py WORKLOAD [--out DIR]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

N_SAMPLE_ROWS = 256
SAMPLE_SEED = 20220118


def inputs(name: str):
    if name == "rmat20":
        rp, c, v = synth.rmat(20, 8, seed=0)
        v = synth.normalize_sym(rp, c, synth.round_values(v, "fp32"))
        v = synth.round_values(synth.round_values(v, "fp32"), "bf16")
        return rp, c, v, 16, 48, ("bf16",), dict(
            generator="synth.rmat(20, 8, seed=0)",
            values="round fp32, normalize_sym, round fp32, round bf16")
    if name == "rmat21":
        rp, c, v = synth.rmat(21, 4, seed=5)
        v = synth.round_values(v, "bf16")
        return rp, c, v, 4, 16, ("bf16",), dict(generator="synth.rmat(21, 4, seed=5)", values="round bf16")
    if name == "rmat23":
        rp, c, v = synth.rmat(23, 16, seed=0)
        v = synth.round_values(v, "bf16")
        return rp, c, v, 24, 64, ("bf16",), dict(generator="synth.rmat(23, 16, seed=0)", values="round bf16")
    if name == "rmat26":
        rp, c, v = synth.rmat(26, 16, seed=0)
        v = synth.round_values(v, "fp32")
        return rp, c, v, 8, 32, (), dict(generator="synth.rmat(26, 16, seed=0)", values="round fp32")
    raise SystemExit(f"unknown workload {name}")


def sample_rows(n: int) -> np.ndarray:
    rng = np.random.default_rng(SAMPLE_SEED)
    return np.sort(rng.choice(n, size=min(N_SAMPLE_ROWS, n), replace=False)).astype(np.int64)


def summarise(ref: dict, rows: np.ndarray) -> dict:
    Y = ref["vecs"]
    arg = np.argmax(np.abs(Y), axis=0)          # lowest row on ties
    K = Y.shape[1]
    return dict(
        vals=ref["vals"].tolist(), theta=ref["theta"].tolist(), idx=ref["idx"].tolist(),
        alpha=ref["alpha"].tolist(), beta=ref["beta"].tolist(),
        abs_resid=ref["abs_resid"].tolist(), rel_resid=ref["rel_resid"].tolist(),
        resid_estimate=ref["resid_estimate"].tolist(),
        ortho_loss=ref["ortho_loss"], ritz_ortho_loss=ref["ritz_ortho_loss"],
        mean_angle_deg=ref["mean_angle_deg"], restarts=int(ref["restarts"]), sweeps=int(ref["sweeps"]),
        sample_vecs=Y[rows, :].tolist(),
        argmax_rows=arg.tolist(), argmax_vals=Y[arg, np.arange(K)].tolist())


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", choices=["rmat20", "rmat21", "rmat23", "rmat26"])
    ap.add_argument("--out", default=HERE)
    args = ap.parse_args()
    oracle.set_progress(True)
    t = time.perf_counter()
    print(f"[golden] generating {args.workload}", flush=True)
    rp, c, v, K, m, emulations, recipe = inputs(args.workload)
    n, nnz = rp.size - 1, int(rp[-1])
    print(f"[golden] n={n} nnz={nnz} K={K} m={m} ({time.perf_counter() - t:.0f} s)", flush=True)
    rows = sample_rows(n)
    out = dict(workload=args.workload, recipe=dict(recipe, K=K, m=m, seed=0, passes=2), n=n, nnz=nnz,
               sample_rows=rows.tolist())
    t = time.perf_counter()
    ref = oracle.topk(rp, c, v, K, m, seed=0)
    print(f"[golden] FP64 oracle solve {time.perf_counter() - t:.0f} s; vals {ref['vals'][:4]}", flush=True)
    out["fp64"] = summarise(ref, rows)
    del ref
    for e in emulations:
        t = time.perf_counter()
        ref = oracle.topk(rp, c, v, K, m, seed=0, emulate=e)
        print(f"[golden] {e}-emulated oracle solve {time.perf_counter() - t:.0f} s", flush=True)
        out[f"emul_{e}"] = summarise(ref, rows)
        del ref
    path = os.path.join(args.out, f"{args.workload}.json")
    with open(path + ".tmp", "w") as fh:
        json.dump(out, fh)
    os.replace(path + ".tmp", path)
    print(f"[golden] wrote {path}", flush=True)


if __name__ == "__main__":
    main()
