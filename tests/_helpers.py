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
