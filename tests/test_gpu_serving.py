"""Serving loop: continuous batching across requests of several resident
models.  Each request's result must equal a lone plan execution of the same
model bit for bit (the server fixes the M2L slot split) and meet the FP32
bar against the FP64 oracle, batching must actually combine requests, and
the HBM budget must reject a request that cannot fit."""
import numpy as np
import pytest

import synth
from _helpers import gpu_tree, oracle_tree
from oracle import fmm as ofmm, operators as oops

pytestmark = pytest.mark.gpu


def _models():
    from paper_1903_02153_amd import bbfmm
    specs = [(12000, 0, 1.0, 4, "uniform", 5), (20000, 1, 0.1, 5, "clustered", 5),
             (6000, 2, 0.05, 6, "slab", 4)]
    out = []
    for i, (n, kid, prm, order, kind, depth) in enumerate(specs):
        pts, _ = synth.random_cloud(n, 70 + i, kind=kind)
        t = gpu_tree(pts, kid, prm, order, fixed_depth=depth)
        o = bbfmm.precompute_operators(t, 1e-5)
        out.append((t, o, n, pts, (kid, prm, order, depth)))
    return out


def test_mix_equals_alone_and_batches():
    import torch
    from paper_1903_02153_amd import bbfmm
    models = _models()
    srv = bbfmm.Server(hbm_budget_bytes=4 << 30, max_inflight=2, r_max=32)
    ids = [srv.add(t, o) for t, o, *_ in models]
    rng = np.random.default_rng(5)
    inputs = []
    for q in range(40):
        m = int(rng.integers(0, len(models)))
        r = int(rng.choice([1, 2, 4, 8]))
        n = models[m][2]
        sig = torch.from_numpy(rng.standard_normal((n, r)).astype(np.float32)).cuda()
        inputs.append((m, sig, torch.empty_like(sig)))
    torch.cuda.synchronize()
    # a burst: requests arriving while both slots are busy are batched
    reqs = [(m, sig, phi, srv.submit(ids[m], sig, phi)) for m, sig, phi in inputs]
    stats = [srv.wait(rid) for _, _, _, rid in reqs]
    torch.cuda.synchronize()
    # Batch invariance: with the M2L slot split and the near-field path fixed
    # (the server uses split 2, the MFMA near field for batches of width
    # >= 2 and the per-lane one for a lone r = 1 request), a column's
    # arithmetic does not depend on the batch, so every request equals a
    # lone plan execution bit for bit.
    lone = {}
    for (m, sig, phi, _), st in zip(reqs, stats):
        t, o = models[m][:2]
        r = sig.shape[1]
        path = 1 if st["batch_r"] == 1 else 2
        if (m, r, path) not in lone:
            lone[(m, r, path)] = bbfmm.Plan(t, o, r, m2l_split=2, p2p_mfma=path)
        alone = torch.empty_like(sig)
        lone[(m, r, path)].execute(sig, alone)
        torch.cuda.synchronize()
        assert torch.equal(phi, alone), (m, r, st["batch_r"])
        assert st["t_submit"] <= st["t_admit"] <= st["t_done"]
    # every served column against the FP64 oracle, per model in one block
    for m, (_, _, n, pts, (kid, prm, order, depth)) in enumerate(models):
        mine = [(sig, phi) for mm, sig, phi, _ in reqs if mm == m]
        if not mine:
            continue
        ot = oracle_tree(pts, fixed_depth=depth)
        oo = oops.precompute(ot, kid, prm, order, 1e-5)
        sig_all = np.concatenate([sig.cpu().numpy() for sig, _ in mine], axis=1)
        got = np.concatenate([phi.cpu().numpy() for _, phi in mine], axis=1)
        ref = ofmm.matvec(ot, oo, pts, sig_all, kid, prm)
        err = ofmm.rel_l2_cols(got.astype(np.float64), ref).max()
        print(f"model {m}: {sig_all.shape[1]} served columns, max rel err vs oracle {err:.2e}")
        assert err < 1e-5
    assert any(st["batch_r"] > sig.shape[1] for (_, sig, _, _), st in zip(reqs, stats))
    c = srv.stats()
    assert c["requests_done"] == len(reqs) and 0 < c["batches"] < len(reqs)
    assert 0 < c["plans_created"] and c["bytes_peak"] <= 4 << 30
    srv.close()


def test_budget_rejects_oversized_request():
    import torch
    from paper_1903_02153_amd import bbfmm
    t, o, n = _models()[1][:3]
    srv = bbfmm.Server(hbm_budget_bytes=1 << 20, max_inflight=2, r_max=8)
    mid = srv.add(t, o)
    sig = torch.ones((n, 4), device="cuda")
    phi = torch.empty_like(sig)
    rid = srv.submit(mid, sig, phi)
    with pytest.raises(bbfmm.BBFMMError, match="BUDGET"):
        srv.wait(rid)
    srv.close()


def test_cancel_pending_and_destroy_with_waiter():
    """A request still queued can be cancelled (its wait reports CANCELLED
    and its phi is untouched); destroying the server while another thread
    waits completes that wait (with a result or CANCELLED) before the
    server's state is freed."""
    import threading
    import torch
    from paper_1903_02153_amd import bbfmm
    models = _models()
    t, o, n = models[1][0], models[1][1], models[1][2]
    srv = bbfmm.Server(hbm_budget_bytes=4 << 30, max_inflight=1, r_max=32)
    mid = srv.add(t, o)
    sig = torch.randn(n, 8, device="cuda")
    outs = [torch.full_like(sig, float("nan")) for _ in range(12)]
    rids = [srv.submit(mid, sig, outs[q]) for q in range(12)]
    cancelled = []
    for q in reversed(range(12)):          # the latest are the likeliest still queued
        try:
            srv.cancel(rids[q])
            cancelled.append(q)
        except bbfmm.BBFMMError as e:
            assert e.status == 1           # already admitted
    for q in range(12):
        if q in cancelled:
            with pytest.raises(bbfmm.BBFMMError) as ei:
                srv.wait(rids[q])
            assert ei.value.status == 7
            torch.cuda.synchronize()
            assert torch.isnan(outs[q]).all()
        else:
            srv.wait(rids[q])
            torch.cuda.synchronize()
            assert torch.isfinite(outs[q]).all()
    print(f"cancelled {len(cancelled)} of 12 queued requests")
    with pytest.raises(bbfmm.BBFMMError):
        srv.cancel(rids[0])                # already waited: unknown
    # destroy while a thread waits
    more = [srv.submit(mid, sig, torch.empty_like(sig)) for _ in range(6)]
    seen = []
    ready = [threading.Event() for _ in more]

    def waiter(q, rid):
        try:
            ready[q].set()
            srv.wait(rid)
            seen.append("done")
        except bbfmm.BBFMMError as e:
            seen.append(e.status)

    th = [threading.Thread(target=waiter, args=(q, rid)) for q, rid in enumerate(more)]
    for x in th:
        x.start()
    for e in ready:
        assert e.wait(30)
    import time
    time.sleep(0.5)                        # the waiters are inside bbfmm_server_wait
    srv.close()
    for x in th:
        x.join(timeout=60)
    assert not any(x.is_alive() for x in th)
    assert len(seen) == 6 and all(v in ("done", 7) for v in seen), seen


def test_concurrent_clients():
    """Four client threads submit and wait at the same time (each wait may
    run while another thread's submit grows the request table); every
    result equals a lone plan execution of its request bit for bit."""
    import threading
    import torch
    from paper_1903_02153_amd import bbfmm
    models = _models()
    srv = bbfmm.Server(hbm_budget_bytes=4 << 30, max_inflight=3, r_max=16)
    ids = [srv.add(t, o) for t, o, *_ in models]
    rng = np.random.default_rng(9)
    jobs = []
    for q in range(48):
        m = int(rng.integers(0, len(models)))
        r = int(rng.choice([1, 2, 4]))
        sig = torch.from_numpy(rng.standard_normal((models[m][2], r)).astype(np.float32)).cuda()
        jobs.append((m, sig, torch.empty_like(sig)))
    torch.cuda.synchronize()
    stats, errors = {}, []

    def client(k):
        try:
            for q in range(k, len(jobs), 4):
                m, sig, phi = jobs[q]
                rid = srv.submit(ids[m], sig, phi)
                stats[q] = srv.wait(rid)
        except Exception as e:          # reported below, on the main thread
            errors.append(repr(e))

    th = [threading.Thread(target=client, args=(k,)) for k in range(4)]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout=120)
    assert not any(x.is_alive() for x in th) and not errors, errors
    torch.cuda.synchronize()
    lone = {}
    for q, (m, sig, phi) in enumerate(jobs):
        t, o = models[m][:2]
        path = 1 if stats[q]["batch_r"] == 1 else 2
        key = (m, sig.shape[1], path)
        if key not in lone:
            lone[key] = bbfmm.Plan(t, o, sig.shape[1], m2l_split=2, p2p_mfma=path)
        alone = torch.empty_like(sig)
        lone[key].execute(sig, alone)
        torch.cuda.synchronize()
        assert torch.equal(phi, alone), (q, m, sig.shape[1], stats[q])
    for p in lone.values():
        p.close()
    assert srv.stats()["requests_done"] == len(jobs)
    srv.close()


def test_fft_model_served():
    """A resident model whose operators are the FFT M2L's spectra (equally
    spaced nodes): served requests of several widths equal a lone plan
    execution bit for bit (each column's M2L runs in its own workgroups)
    and meet the FP32 bar against the oracle on the same nodes."""
    import torch
    from paper_1903_02153_amd import bbfmm
    pts, _ = synth.random_cloud(10000, 90, kind="uniform")
    t = gpu_tree(pts, 0, 1.0, 4, fixed_depth=4)
    o = bbfmm.precompute_operators(t, 1e-5, bbfmm.M2L_FFT)
    srv = bbfmm.Server(hbm_budget_bytes=4 << 30, max_inflight=2, r_max=16)
    mid = srv.add(t, o)
    rng = np.random.default_rng(11)
    reqs = []
    for q in range(12):
        r = int(rng.choice([1, 2, 4]))
        sig = torch.from_numpy(rng.standard_normal((10000, r)).astype(np.float32)).cuda()
        phi = torch.empty_like(sig)
        reqs.append((sig, phi, srv.submit(mid, sig, phi)))
    stats = [srv.wait(rid) for _, _, rid in reqs]
    torch.cuda.synchronize()
    for (sig, phi, _), st in zip(reqs, stats):
        path = 1 if st["batch_r"] == 1 else 2
        plan = bbfmm.Plan(t, o, sig.shape[1], m2l_split=2, p2p_mfma=path)
        alone = torch.empty_like(sig)
        plan.execute(sig, alone)
        torch.cuda.synchronize()
        plan.close()
        assert torch.equal(phi, alone), (sig.shape[1], st["batch_r"])
    ot = oracle_tree(pts, fixed_depth=4)
    oo = oops.precompute(ot, 0, 1.0, 4, 0.0, nodes="uniform")
    sig_all = np.concatenate([s.cpu().numpy() for s, _, _ in reqs], axis=1)
    got = np.concatenate([p.cpu().numpy() for _, p, _ in reqs], axis=1)
    ref = ofmm.matvec(ot, oo, pts, sig_all, 0, 1.0)
    err = ofmm.rel_l2_cols(got.astype(np.float64), ref).max()
    print(f"FFT model: {sig_all.shape[1]} served columns, max rel err vs oracle {err:.2e}")
    assert err < 1e-5
    srv.close()
