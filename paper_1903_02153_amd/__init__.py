"""MI355X (gfx950) black-box FMM kernel matvec: phi = K sigma.

The compute path is the HIP library ``libbbfmm.so`` (sources in ``csrc/``,
C ABI in ``include/bbfmm.h``); ``bbfmm`` is its Python binding.
"""
from .bbfmm import (BBFMMError, Ops, Plan, Tree, build_tree, lib, matvec,  # noqa: F401
                    ops_import, precompute_operators)
