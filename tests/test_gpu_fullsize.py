"""Full-size parity for the two larger workload shapes, in the launch
configuration of a batched plan (all r right-hand sides in one execution):

* 2^21 points in 64 Gaussian clusters, exp(-r/0.1), order 6, leaf-size rule
  (64 points) capped at 7 levels, r = 16, M2L in split-BF16x3;
* a jittered 200x200x25 slab of 10^6 points, exp(-r^2/0.05^2), order 7,
  7 levels, r = 64, M2L in per-cell-scaled FP16.

The tree is compared bit for bit.  phi is compared with the FP64 oracle bbFMM
(same tree, order and SVD tolerance) on 1024 sampled rows and the first and
last columns, for the workload's own M2L precision and for the FP32 path.
The oracle's far field is evaluated in full; its near field only for the
sampled rows."""
import numpy as np
import pytest

import synth
from _helpers import compare_trees, gpu_tree, oracle_tree
from oracle import fmm as ofmm, operators as oops

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

TOL_FP32 = 1e-5
# Scaled FP16 rounds both M2L operands to 11 significant bits; on the far
# field this gives ~1e-3 relative error per product, reduced by averaging over
# the k terms of a row and by the near field's share of phi.
TOL = {synth.PREC_FP32: TOL_FP32, synth.PREC_BF16X3: TOL_FP32, synth.PREC_FP16_SCALED: 1e-3}


def _run(w, precision):
    import torch
    from paper_1903_02153_amd import bbfmm
    gt = gpu_tree(w.points, w.kernel_id, w.kernel_param, w.order, leaf_size=w.leaf_size,
                  max_depth=w.max_depth, fixed_depth=w.fixed_depth)
    go = bbfmm.precompute_operators(gt, w.eps, precision)
    plan = bbfmm.Plan(gt, go, w.r)
    sig = torch.from_numpy(w.sigma).cuda()
    phi = torch.empty_like(sig)
    plan.execute(sig, phi)
    torch.cuda.synchronize()
    return gt, phi.cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module", params=["clustered-2M", "slab-1M"])
def workload(request):
    w = synth.cfg_clustered_2m() if request.param == "clustered-2M" else synth.cfg_slab_1m()
    ot = oracle_tree(w.points, leaf_size=w.leaf_size, max_depth=w.max_depth,
                     fixed_depth=w.fixed_depth)
    oo = oops.precompute(ot, w.kernel_id, w.kernel_param, w.order, w.eps)
    cols = [0, w.r - 1]
    rows = w.sample_rows[::4]
    ref = ofmm.matvec(ot, oo, w.points, w.sigma[:, cols], w.kernel_id, w.kernel_param,
                      rows=rows)
    return w, ot, cols, rows, ref


@pytest.mark.parametrize("which", ["own", "fp32"])
def test_full_size_batched(workload, which):
    w, ot, cols, rows, ref = workload
    prec = w.precision if which == "own" else synth.PREC_FP32
    gt, phi = _run(w, prec)
    compare_trees(gt, ot)
    got = phi[rows][:, cols]
    assert np.all(np.isfinite(phi))
    err = ofmm.rel_l2_cols(got, ref)
    print(f"{w.name} precision {prec}: depth {ot.depth}, rel err per column {err}")
    assert err.max() < TOL[prec]
