"""Shared helpers for the GPU parity tests (oracle on one side, the HIP
library through its C ABI on the other; no code is shared between them)."""
import numpy as np

from oracle import fmm as ofmm, operators as oops, tree as otree


def oracle_tree(pts, leaf_size=64, max_depth=22, fixed_depth=0):
    return otree.build_tree(pts, leaf_size=leaf_size, max_depth=max_depth,
                            fixed_depth=fixed_depth)


def gpu_tree(pts, kid, prm, n, leaf_size=64, max_depth=22, fixed_depth=0):
    import torch
    from paper_1903_02153_amd import bbfmm
    tp = torch.from_numpy(np.ascontiguousarray(pts, dtype=np.float32)).cuda()
    return bbfmm.build_tree(tp, kid, prm, cheb_order=n, leaf_size=leaf_size,
                            max_depth=max_depth, fixed_depth=fixed_depth)


def gpu_matvec(tree, ops, sig):
    import torch
    from paper_1903_02153_amd import bbfmm
    ts = torch.from_numpy(np.ascontiguousarray(sig, dtype=np.float32)).cuda()
    phi = bbfmm.matvec(tree, ops, ts)
    torch.cuda.synchronize()
    return phi.cpu().numpy().astype(np.float64)


# Element-wise bar beside the per-column relative L2 bar: every element of a
# column within ELEM_FACTOR x (the L2 bar) x the column's largest |phi|.
ELEM_FACTOR = 10.0


def assert_parity(got, ref, tol, label=""):
    """Per-column relative L2 error < tol and, element by element,
    |got - ref| <= ELEM_FACTOR * tol * max|ref| of the column.  Prints both."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if got.ndim == 1:
        got, ref = got[:, None], ref[:, None]
    assert got.shape == ref.shape, (got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{label}: non-finite output"
    l2 = ofmm.rel_l2_cols(got, ref)
    scale = np.abs(ref).max(axis=0)
    scale[scale == 0] = 1.0
    elem = np.abs(got - ref).max(axis=0) / scale
    print(f"{label}: max column rel L2 {l2.max():.2e}, max element err / column max "
          f"{elem.max():.2e} ({got.shape[0]} rows x {got.shape[1]} columns)")
    assert l2.max() < tol, (label, l2)
    assert elem.max() <= ELEM_FACTOR * tol, (label, elem)
    return l2, elem


def run_plan(tree, ops, sig, **options):
    """One product with a plan of these options; the plan is held until the
    device has finished and then freed."""
    import torch
    from paper_1903_02153_amd import bbfmm
    ts = sig if isinstance(sig, torch.Tensor) else \
        torch.from_numpy(np.ascontiguousarray(sig, dtype=np.float32)).cuda()
    phi = torch.empty((tree.info().n_targets, ts.shape[1]), dtype=ts.dtype, device=ts.device)
    plan = bbfmm.Plan(tree, ops, ts.shape[1], **options)
    plan.execute(ts, phi)
    torch.cuda.synchronize()
    plan.close()
    return phi


def compare_trees(gt, ot):
    """Bit-exact comparison of every tree array against the oracle."""
    info = gt.info()
    assert info.depth == ot.depth
    assert np.float32(info.side) == ot.side and np.float32(info.scale) == ot.scale
    assert np.array_equal(np.array(info.lo[:], np.float32), ot.lo)
    assert np.array_equal(gt.export("perm"), ot.perm)
    for lvl in range(ot.depth):
        lv = ot.levels[lvl]
        assert info.cells[lvl] == len(lv.keys)
        assert np.array_equal(gt.export("keys", lvl), lv.keys)
        assert np.array_equal(gt.export("pb", lvl), lv.pb)
        assert np.array_equal(gt.export("pe", lvl), lv.pe)
        assert np.array_equal(gt.export("parent", lvl), lv.parent)
        assert np.array_equal(gt.export("cb", lvl), lv.cb)
        assert np.array_equal(gt.export("ce", lvl), lv.ce)
    assert np.array_equal(gt.export("nbr_off"), ot.nbr_off)
    assert np.array_equal(gt.export("nbr_idx"), ot.nbr_idx)
    for lvl in range(2, ot.depth):
        pr = ot.pairs[lvl]
        assert info.pairs[lvl] == len(pr["t"])
        assert np.array_equal(gt.export("pair_t", lvl), pr["t"])
        assert np.array_equal(gt.export("pair_tgt", lvl), pr["tgt"])
        assert np.array_equal(gt.export("pair_src", lvl), pr["src"])
        assert np.array_equal(gt.export("pair_goff", lvl), pr["group_off"])
