"""Serving loop (continuous batching) on the GPU: results are identical alone
and in a concurrent mix, admission respects the HBM budget, oversized
requests are rejected, and latency timestamps are consistent."""
import numpy as np
import pytest

import oracle
import synth
from gpu_util import bf16_bounds, device_csr, eig_rel_err, topk_pair_err

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_2201_07498_amd as lz  # noqa: E402


def make_requests():
    reqs = []
    specs = [("er", 6000, 9.0, 4, 12, "fp64", 1), ("rmat", 5000, 12.0, 8, 24, "fp32", 2),
             ("rmat", 20000, 7.0, 8, 24, "bf16", 3), ("rmat", 30000, 20.0, 16, 48, "fp64", 4),
             ("er", 3000, 15.0, 4, 12, "fp32", 5), ("rmat", 12000, 6.0, 4, 12, "fp64", 6)]
    for kind, n, d, K, m, prec, seed in specs:
        if kind == "er":
            rp, c, v = synth.er(n, d, seed=seed)
        else:
            rp, c, v = synth.rmat_n(n, d, seed=seed)
        v = synth.round_values(v, prec)
        reqs.append(dict(rp=rp, col=c, val=v, K=K, m=m, prec=prec, seed=seed))
    return reqs


REQS = make_requests()


def solo(q):
    drp, dc, dv = device_csr(q["rp"], q["col"], q["val"], q["prec"])
    vals, vecs, rep = lz.topk(drp, dc, dv, q["K"], q["m"], q["prec"], seed=q["seed"])
    torch.cuda.synchronize()
    return vals.cpu().numpy(), vecs.cpu().numpy(), rep


def submit_all(srv, reqs):
    tickets = []
    for q in reqs:
        tickets.append(srv.submit(q["rp"], q["col"], synth.to_storage(q["val"], q["prec"]), q["K"], q["m"],
                                  q["prec"], seed=q["seed"], want_vectors=True))
    return tickets


@pytest.mark.parametrize("use_graphs", [True, False])
def test_mix_equals_alone_bitwise(use_graphs):
    alone = [solo(q) for q in REQS]
    budget = 4 * max(lz.request_footprint(q["rp"].size - 1, q["col"].size, q["K"], q["m"], q["prec"]) for q in REQS)
    with lz.Server(budget, max_slots=4, use_graphs=use_graphs) as srv:
        tickets = submit_all(srv, REQS)
        for q, t, (va, Ya, rep) in zip(REQS, tickets, alone):
            vals, vecs, res = srv.wait(t)
            print(f"n={q['rp'].size - 1} {q['prec']} slot={res['slot']} latency "
                  f"{res['t_done_ms'] - res['t_submit_ms']:.2f} ms device {res['device_ms']:.2f} ms")
            assert res["status"] == 0
            assert np.array_equal(vals, va), (vals, va)
            assert np.array_equal(vecs, Ya)
            assert res["m_eff"] == q["m"]
            assert res["resid_max"] == float(np.max(rep["resid"]))
            assert np.array_equal(res["resid"], rep["resid"])
            assert res["t_submit_ms"] <= res["t_admit_ms"] <= res["t_done_ms"] and res["device_ms"] > 0
        st = srv.stats()
        assert st["completed"] == len(REQS) and st["active"] == 0 and st["queued"] == 0
        assert st["arena_peak"] <= st["arena_bytes"] and st["arena_in_use"] == 0


def test_results_match_oracle_in_the_mix():
    # FP64 and FP32 against the FP64 oracle at 1e-10 / 1e-6.  BF16 in Top-K
    # order against the FP64 oracle with the per-pair bound: 1e-3 on the pairs
    # the oracle has converged (three of the eight here), the BF16 emulation
    # and the residuals elsewhere; its residuals come from the same request
    # solved alone, which the mix reproduces bit for bit.
    alone = {i: solo(q) for i, q in enumerate(REQS) if q["prec"] == "bf16"}
    with lz.Server(1 << 30, max_slots=3) as srv:
        tickets = submit_all(srv, REQS)
        for i, (q, t) in enumerate(zip(REQS, tickets)):
            vals, vecs, res = srv.wait(t)
            if q["prec"] != "bf16":
                ref = oracle.topk(q["rp"], q["col"], q["val"], q["K"], q["m"], seed=q["seed"], report=False)
                tol = {"fp64": 1e-10, "fp32": 1e-6}[q["prec"]]
                assert eig_rel_err(vals, ref["vals"]) <= tol, (q["prec"], eig_rel_err(vals, ref["vals"]))
                continue
            ref = oracle.topk(q["rp"], q["col"], q["val"], q["K"], q["m"], seed=q["seed"])
            emul = oracle.topk(q["rp"], q["col"], q["val"], q["K"], q["m"], seed=q["seed"], emulate="bf16",
                               report=False)
            va, _, rep = alone[i]
            assert np.array_equal(vals, va)
            bound, conv, emul_err = bf16_bounds(ref, emul["vals"], rep["abs_resid"])
            errs = topk_pair_err(vals, np.asarray(ref["vals"]), 1e-3, np.asarray(ref["theta"]))
            print(f"serving bf16: errors {errs}, bounds {bound}, {conv.sum()} converged")
            assert conv.sum() >= 3
            assert np.all(errs <= bound), (errs, bound)


def test_small_budget_serialises_and_rejects_oversized():
    foot = [lz.request_footprint(q["rp"].size - 1, q["col"].size, q["K"], q["m"], q["prec"]) for q in REQS]
    budget = int(1.2 * max(foot))
    with lz.Server(budget, max_slots=4) as srv:
        tickets = submit_all(srv, REQS)
        done = [srv.wait(t)[2] for t in tickets]
        assert all(r["status"] == 0 for r in done)
        st = srv.stats()
        assert st["arena_peak"] <= budget
        # A request that can never fit is refused at submission.
        rp, c, v = synth.er(200000, 9.0, seed=9)
        with pytest.raises(lz.LanczosError) as ei:
            srv.submit(rp, c, v, 8, 24, "fp64")
        assert ei.value.code == -5
        assert srv.stats()["rejected"] == 1


def test_invalid_requests_rejected():
    with lz.Server(1 << 26, max_slots=2) as srv:
        rp, c, v = synth.er(100, 5.0, seed=1)
        with pytest.raises(lz.LanczosError):
            srv.submit(rp, c, v, 8, 4, "fp64")          # m < K
        with pytest.raises(lz.LanczosError):
            srv.submit(rp, c, v, 4, 65, "fp64")         # m > max steps
        t = srv.submit(rp, c, v, 2, 6, "fp64")
        vals, _, res = srv.wait(t)
        assert res["status"] == 0 and vals.shape == (2,)


def test_concurrent_submitters_match_alone():
    # Three host threads share one server: each submits its requests and waits
    # for them while the others do the same (the library's calls release the
    # interpreter lock, so submissions, completions and the slot threads
    # interleave).  Every result equals the solve run alone.
    import threading

    alone = [solo(q) for q in REQS]
    budget = 3 * max(lz.request_footprint(q["rp"].size - 1, q["col"].size, q["K"], q["m"], q["prec"]) for q in REQS)
    errors = []
    with lz.Server(budget, max_slots=3) as srv:
        def client(indices):
            try:
                for _ in range(2):
                    tickets = [(i, srv.submit(REQS[i]["rp"], REQS[i]["col"],
                                              synth.to_storage(REQS[i]["val"], REQS[i]["prec"]), REQS[i]["K"],
                                              REQS[i]["m"], REQS[i]["prec"], seed=REQS[i]["seed"],
                                              want_vectors=True)) for i in indices]
                    for i, t in tickets:
                        vals, vecs, res = srv.wait(t)
                        va, Ya, rep = alone[i]
                        assert res["status"] == 0, (i, res["status"])
                        assert np.array_equal(vals, va), i
                        assert np.array_equal(vecs, Ya), i
                        assert np.array_equal(res["resid"], rep["resid"]), i
                        srv.release(t)
            except Exception as exc:          # reported on the main thread
                errors.append(exc)

        threads = [threading.Thread(target=client, args=(list(range(k, len(REQS), 3)),)) for k in range(3)]
        for th in threads:
            th.start()
        for th in threads:
            th.join(timeout=120)
        assert not any(th.is_alive() for th in threads)
        assert not errors, errors
        st = srv.stats()
        assert st["completed"] == 2 * len(REQS) and st["active"] == 0 and st["queued"] == 0
        assert st["arena_in_use"] == 0 and st["arena_peak"] <= st["arena_bytes"]
