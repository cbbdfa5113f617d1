"""The C-ABI library loads, exports every symbol include/bbfmm.h declares,
and rejects invalid arguments before touching the GPU (CPU-only tests)."""
import ctypes
import os
import re

import pytest

from paper_1903_02153_amd import bbfmm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bbfmm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return set(re.findall(r"\b(bbfmm_[a-z_]+)\s*\(", text))


def test_header_declares_the_paper_api():
    names = declared_functions()
    for fn in ("bbfmm_build_tree", "bbfmm_precompute_operators", "bbfmm_matvec"):
        assert fn in names


def test_library_exports_every_declared_symbol():
    lib = bbfmm.lib()
    names = declared_functions()
    assert names, "no declarations parsed"
    for name in sorted(names):
        assert hasattr(lib, name), name
    assert names == set(bbfmm.SIGNATURES)


def test_invalid_arguments_rejected_without_gpu():
    lib = bbfmm.lib()
    p = bbfmm.TreeParams(0, 1.0, 4, 64, 22, 0)
    out = ctypes.c_void_p()
    assert lib.bbfmm_build_tree(None, 10, ctypes.byref(p), None, None, ctypes.byref(out)) == 1
    assert b"NULL" in lib.bbfmm_last_error()
    fake = ctypes.c_void_p(0x1000)
    assert lib.bbfmm_build_tree(fake, 0, ctypes.byref(p), None, None, ctypes.byref(out)) == 1
    bad = bbfmm.TreeParams(0, 1.0, 9, 64, 22, 0)
    assert lib.bbfmm_build_tree(fake, 10, ctypes.byref(bad), None, None, ctypes.byref(out)) == 1
    assert b"cheb_order" in lib.bbfmm_last_error()
    bad = bbfmm.TreeParams(7, 1.0, 4, 64, 22, 0)
    assert lib.bbfmm_build_tree(fake, 10, ctypes.byref(bad), None, None, ctypes.byref(out)) == 1
    bad = bbfmm.TreeParams(0, 1.0, 4, 64, 23, 0)
    assert lib.bbfmm_build_tree(fake, 10, ctypes.byref(bad), None, None, ctypes.byref(out)) == 1
    bad = bbfmm.TreeParams(1, -1.0, 4, 64, 22, 0)
    assert lib.bbfmm_build_tree(fake, 10, ctypes.byref(bad), None, None, ctypes.byref(out)) == 1
    assert out.value is None
    assert lib.bbfmm_precompute_operators(None, 1e-5, 0, None, None, ctypes.byref(out)) == 1
    # thresholds the FP64 Gram route cannot resolve are refused before anything else
    assert lib.bbfmm_precompute_operators(None, 1e-9, 0, None, None, ctypes.byref(out)) == 1
    assert b"svd_eps" in lib.bbfmm_last_error()
    assert lib.bbfmm_plan_create(None, None, 1, ctypes.byref(out)) == 1
    assert lib.bbfmm_plan_execute(None, None, None, None) == 1
    info = bbfmm.TreeInfo()
    assert lib.bbfmm_tree_info_get(None, ctypes.byref(info)) == 1
    # free functions accept NULL
    lib.bbfmm_tree_free(None)
    lib.bbfmm_ops_free(None)
    lib.bbfmm_plan_free(None)


def test_dense_products_reject_invalid_arguments_without_gpu():
    """The dense products of the eigendecomposition check sizes and
    pointers before touching the device."""
    lib = bbfmm.lib()
    fake = ctypes.c_void_p(0x1000)
    assert lib.bbfmm_dense_atb(None, fake, 10, 4, fake, None, None) == 1
    assert b"NULL" in lib.bbfmm_last_error()
    assert lib.bbfmm_dense_atb(fake, fake, 0, 4, fake, None, None) == 1
    assert lib.bbfmm_dense_atb(fake, fake, 10, 0, fake, None, None) == 1
    assert lib.bbfmm_dense_atb(fake, fake, 10, 1025, fake, None, None) == 1
    assert b"m must be" in lib.bbfmm_last_error()
    assert lib.bbfmm_dense_atb(fake, fake, 10, 4, fake, None, None) == 1   # not device memory
    assert b"device" in lib.bbfmm_last_error()
    assert lib.bbfmm_dense_ab(fake, 10, 4, None, 3, fake, None) == 1
    assert lib.bbfmm_dense_ab(fake, 10, 4, fake, 0, fake, None) == 1
    assert lib.bbfmm_dense_ab(fake, -1, 4, fake, 3, fake, None) == 1


def test_allocator_hook_checked_and_counters_without_gpu():
    """An allocator hook needs both functions; the runtime counters are
    readable without a GPU and start with nothing live."""
    lib = bbfmm.lib()
    a = bbfmm.TorchAllocator()
    half = bbfmm.AllocatorHook(a._alloc_cb, bbfmm._FREE_FN(), None)
    p = bbfmm.TreeParams(0, 1.0, 4, 64, 22, 0)
    out = ctypes.c_void_p()
    fake = ctypes.c_void_p(0x1000)
    assert lib.bbfmm_build_tree(fake, 10, ctypes.byref(p), ctypes.byref(half), None,
                                ctypes.byref(out)) == 1
    assert b"allocator" in lib.bbfmm_last_error()
    assert out.value is None and a.allocs == 0
    c = bbfmm.runtime_counters()
    assert set(c) == {"device_buffers", "device_bytes", "plans", "streams", "events",
                      "plans_freed_in_flight"}
    assert c["device_buffers"] == 0 and c["device_bytes"] == 0 and c["plans"] == 0


@pytest.mark.parametrize("field,value", [("m2l_split", 9), ("m2l_min_waves", 17),
                                         ("p2p_max_split", 3), ("p2p_mfma", 3), ("overlap", -1),
                                         ("p2p_waves", -5), ("m2l_occupancy", 5),
                                         ("m2l_layout", 3), ("m2l_schedule", 3),
                                         ("m2l_block", -1), ("m2l_rtile", 48),
                                         ("m2l_xcd", 3), ("leaf_fused", 3), ("p2p_pack", -1),
                                         ("m2l_mfma", 3)])
def test_plan_options_validated_without_gpu(field, value):
    """Every launch-shape option is range-checked before any handle or
    device memory is touched; the message names the option."""
    lib = bbfmm.lib()
    opt = bbfmm.PlanOptions()
    setattr(opt, field, value)
    out = ctypes.c_void_p()
    assert lib.bbfmm_plan_create_ex(None, None, 4, ctypes.byref(opt), None, None,
                                     ctypes.byref(out)) == 1
    assert field.encode() in lib.bbfmm_last_error()
    assert out.value is None


def test_autotune_rejects_invalid_arguments_without_gpu():
    lib = bbfmm.lib()
    best = bbfmm.PlanOptions()
    ms = ctypes.c_double()
    assert lib.bbfmm_plan_autotune(None, None, 1, None, None, None, 3, ctypes.byref(best),
                                   ctypes.byref(ms)) == 1
    assert b"NULL" in lib.bbfmm_last_error()


def test_binding_refuses_cpu_tensors():
    import torch
    with pytest.raises(TypeError):
        bbfmm.build_tree(torch.zeros((10, 3)))


def test_missing_library_fails_loudly(monkeypatch):
    monkeypatch.setattr(bbfmm, "_lib_handle", None)
    monkeypatch.setattr(bbfmm, "LIB_PATH", "/nonexistent/libbbfmm.so")
    with pytest.raises(RuntimeError, match="missing"):
        bbfmm.lib()


def test_server_rejects_invalid_arguments_without_gpu():
    lib = bbfmm.lib()
    out = ctypes.c_void_p()
    assert lib.bbfmm_server_create(0, 4, 16, ctypes.byref(out)) == 1
    assert lib.bbfmm_server_create(1 << 30, 0, 16, ctypes.byref(out)) == 1
    assert lib.bbfmm_server_create(1 << 30, 4, 0, ctypes.byref(out)) == 1
    assert out.value is None
    assert lib.bbfmm_server_destroy(None) == 0
