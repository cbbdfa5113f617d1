"""Resource handling of the C ABI on the GPU: the allocator hook (torch's
caching allocator owns the library's device memory, an allocator that
returns NULL gives OUT_OF_MEMORY and leaks nothing), the asynchronous
bbfmm_matvec with its per-(r, stream) workspace cache, the ordering of one
plan's products across streams, and plans freed while their product runs."""
import numpy as np
import pytest

import synth
from _helpers import assert_parity, gpu_tree, oracle_tree, run_plan
from oracle import fmm as ofmm, operators as oops

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _cloud(nn=20000, seed=7, r=2):
    return synth.random_cloud(nn, seed, r=r, kind="clustered")


def _live():
    import gc
    from paper_1903_02153_amd import bbfmm
    gc.collect()
    return bbfmm.runtime_counters()


def test_torch_allocator_owns_the_device_memory():
    """With the default binding every device byte of a tree, its operators
    and a plan comes from torch's caching allocator and goes back to it."""
    import torch
    from paper_1903_02153_amd import bbfmm
    pts, sig = _cloud()
    alloc = bbfmm.TorchAllocator()
    base = _live()
    tp = torch.from_numpy(pts).cuda()
    tree = bbfmm.build_tree(tp, bbfmm.K_EXP, 0.2, cheb_order=4, fixed_depth=4, allocator=alloc)
    ops = bbfmm.precompute_operators(tree, 1e-5)
    phi = run_plan(tree, ops, sig)
    held = _live()
    print(f"torch allocator: {alloc.allocs} allocations, {len(alloc.live)} live; counters {held}")
    assert alloc.allocs > 0 and len(alloc.live) == held["device_buffers"] - base["device_buffers"]
    assert sum(alloc.live.values()) == held["device_bytes"] - base["device_bytes"]
    ot = oracle_tree(pts, fixed_depth=4)
    oo = oops.precompute(ot, 1, 0.2, 4, 1e-5)
    assert_parity(phi.cpu().numpy(), ofmm.matvec(ot, oo, pts, sig, 1, 0.2), TOL, "torch allocator")
    ops.close()
    tree.close()
    assert not alloc.live and alloc.allocs == alloc.frees
    assert _live()["device_buffers"] == base["device_buffers"]


@pytest.mark.parametrize("stage", ["build", "precompute", "plan"])
def test_allocator_returning_null_gives_out_of_memory(stage):
    """An allocator that returns NULL at its k-th call (k swept over the
    calls the stage makes) makes the call fail with OUT_OF_MEMORY; every
    buffer obtained before the failure is returned and no handle is left."""
    import torch
    from paper_1903_02153_amd import bbfmm
    pts, sig = _cloud(6000, 8, r=3)
    tp = torch.from_numpy(pts).cuda()
    ts = torch.from_numpy(sig).cuda()
    good = bbfmm.TorchAllocator()
    base = _live()
    # how many allocations the stage makes when nothing fails
    probe = bbfmm.TorchAllocator()
    t = bbfmm.build_tree(tp, bbfmm.K_INV_R, 1.0, cheb_order=4, fixed_depth=4,
                         allocator=probe if stage == "build" else good)
    o = bbfmm.precompute_operators(t, 1e-5, allocator=probe if stage == "precompute" else None)
    p = bbfmm.Plan(t, o, 3, allocator=probe if stage == "plan" else None)
    torch.cuda.synchronize()
    total = probe.allocs
    p.close()
    o.close()
    t.close()
    assert total > 0 and not probe.live
    ks = sorted(set([0, 1, total // 3, total // 2, total - 1]))
    for k in ks:
        bad = bbfmm.TorchAllocator(fail_after=k)
        t = o = None
        with pytest.raises(bbfmm.BBFMMError) as ei:
            t = bbfmm.build_tree(tp, bbfmm.K_INV_R, 1.0, cheb_order=4, fixed_depth=4,
                                 allocator=bad if stage == "build" else good)
            o = bbfmm.precompute_operators(t, 1e-5, allocator=bad if stage == "precompute" else None)
            bbfmm.Plan(t, o, 3, allocator=bad if stage == "plan" else None)
        assert ei.value.status == 2, str(ei.value)
        if o is not None:
            o.close()
        if t is not None:
            t.close()
        torch.cuda.synchronize()
        print(f"{stage}: NULL at allocation {k} of {total}: {bad.allocs} obtained, "
              f"{bad.frees} returned")
        assert bad.allocs == k and bad.frees == k and not bad.live
        assert _live()["device_buffers"] == base["device_buffers"]
        assert _live()["plans"] == base["plans"]
    # the library still works afterwards
    t = bbfmm.build_tree(tp, bbfmm.K_INV_R, 1.0, cheb_order=4, fixed_depth=4, allocator=good)
    o = bbfmm.precompute_operators(t, 1e-5)
    phi = run_plan(t, o, ts)
    ot = oracle_tree(pts, fixed_depth=4)
    oo = oops.precompute(ot, 0, 1.0, 4, 1e-5)
    assert_parity(phi.cpu().numpy(), ofmm.matvec(ot, oo, pts, sig, 0, 1.0), TOL, "after OOM")


def test_matvec_is_asynchronous_and_reuses_its_workspace():
    """bbfmm_matvec enqueues and returns; repeated products on one stream
    allocate nothing; products on two streams agree; freeing the operators
    releases the cached workspaces."""
    import torch
    from paper_1903_02153_amd import bbfmm
    pts, sig = _cloud(30000, 9, r=1)
    tree = gpu_tree(pts, bbfmm.K_INV_R, 1.0, 5, fixed_depth=5)
    ops = bbfmm.precompute_operators(tree, 1e-5)
    ts = torch.from_numpy(sig).cuda()
    ref = run_plan(tree, ops, ts)
    torch.cuda.synchronize()
    base = _live()
    out = [torch.empty_like(ts) for _ in range(8)]
    bbfmm.matvec(tree, ops, ts, out[0])
    first = _live()
    for q in range(1, 8):
        bbfmm.matvec(tree, ops, ts, out[q])
    again = _live()
    torch.cuda.synchronize()
    assert again["device_buffers"] == first["device_buffers"] > base["device_buffers"]
    for q in range(8):
        assert torch.equal(out[q], ref), q
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a, b = torch.empty_like(ts), torch.empty_like(ts)
    torch.cuda.synchronize()
    for _ in range(3):
        bbfmm.matvec(tree, ops, ts, a, stream=s1)
        bbfmm.matvec(tree, ops, ts, b, stream=s2)
    torch.cuda.synchronize()
    assert torch.equal(a, ref) and torch.equal(b, ref)
    ops.close()
    assert _live()["device_buffers"] < first["device_buffers"]
    assert _live()["plans"] == base["plans"]


def test_one_plan_on_two_streams_is_ordered():
    """Products of one plan enqueued alternately on two streams (no caller
    synchronisation between them) each see a whole workspace of their own
    turn: with sigma scaled by powers of two (exact in FP32, so the product
    scales exactly) every output equals the single-stream result times the
    scale, bit for bit."""
    import torch
    from paper_1903_02153_amd import bbfmm
    pts, sig = _cloud(25000, 10, r=3)
    tree = gpu_tree(pts, bbfmm.K_EXP, 0.2, 5, fixed_depth=5)
    ops = bbfmm.precompute_operators(tree, 1e-5)
    ts = torch.from_numpy(sig).cuda()
    ref = run_plan(tree, ops, ts, overlap=2, p2p_mfma=1)
    plan = bbfmm.Plan(tree, ops, 3, overlap=2, p2p_mfma=1)
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    sigs = [ts * float(2 ** q) for q in range(6)]
    outs = [torch.empty_like(ts) for _ in range(6)]
    torch.cuda.synchronize()
    for q in range(6):
        plan.execute(sigs[q], outs[q], stream=streams[q % 2])
    torch.cuda.synchronize()
    for q in range(6):
        assert torch.equal(outs[q], ref * float(2 ** q)), q
    plan.close()


def test_plan_freed_while_its_product_runs():
    """Freeing a plan right after enqueueing a product waits for it (the
    counter records that it was still running); the result is complete."""
    import torch
    from paper_1903_02153_amd import bbfmm
    pts, sig = _cloud(60000, 11, r=4)
    tree = gpu_tree(pts, bbfmm.K_INV_R, 1.0, 5, fixed_depth=5)
    ops = bbfmm.precompute_operators(tree, 1e-5)
    ts = torch.from_numpy(sig).cuda()
    ref = run_plan(tree, ops, ts, overlap=2, p2p_mfma=1)
    base = _live()
    for q in range(3):
        phi = torch.full_like(ts, float("nan"))
        plan = bbfmm.Plan(tree, ops, 4, overlap=2, p2p_mfma=1)
        plan.execute(ts, phi)
        plan.close()                  # no synchronisation before the free
        torch.cuda.synchronize()
        assert torch.equal(phi, ref), q
    now = _live()
    print(f"plans freed in flight: {now['plans_freed_in_flight'] - base['plans_freed_in_flight']} of 3")
    for key in ("device_buffers", "plans", "events"):
        assert now[key] == base[key], (key, base, now)
