"""C ABI checks that need no GPU: the library builds, loads, exports every symbol the
header declares, and host-side misuse returns status codes instead of aborting."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ttie.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2606_06511_amd import build_lib, ttie

    if not os.path.exists(build_lib.LIB):
        build_lib.build()
    return ttie.lib()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ttie_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    # the calls of the boundary: version and errors, context, workspace, broad phase,
    # evaluation, the two-call Hessian, matrix-free products, batches
    for fn in ["ttie_version", "ttie_last_error", "ttie_create", "ttie_destroy", "ttie_workspace_size",
               "ttie_set_workspace", "ttie_get_status", "ttie_broadphase", "ttie_eval", "ttie_bsr_symbolic",
               "ttie_bsr_numeric", "ttie_hvp", "ttie_bsr_mv", "ttie_get_hits", "ttie_batch_broadphase",
               "ttie_batch_eval", "ttie_eval_static"]:
        assert fn in names, fn


def test_library_exports_every_declared_symbol(lib):
    from paper_2606_06511_amd import build_lib, ttie

    out = subprocess.run(["nm", "-D", "--defined-only", build_lib.LIB], capture_output=True, text=True, check=True)
    exported = set(re.findall(r"\bT (ttie_\w+)", out.stdout))
    for fn in declared_functions():
        assert fn in exported, fn
        assert fn in ttie.SIGNATURES, fn


def test_version_string(lib):
    assert lib.ttie_version().decode().startswith("ttie ")


def test_host_side_errors_without_gpu(lib):
    import torch

    from paper_2606_06511_amd import ttie

    if torch.cuda.is_available():
        pytest.skip("checks the no-device path")
    h = ctypes.c_void_p()
    assert lib.ttie_create(0, ctypes.byref(h)) == 6  # TTIE_ERR_NO_DEVICE
    assert h.value is None
    assert lib.ttie_last_error().decode() != ""
    assert lib.ttie_create(0, None) == 1
    assert lib.ttie_destroy(None) == 1
    size = ctypes.c_size_t()
    lim = ttie.Limits(10, 10, 10, 10, 10)
    assert lib.ttie_workspace_size(None, ctypes.byref(lim), ctypes.byref(size)) == 1
    assert lib.ttie_eval(None, None, None, None, 0, None, None, None, None, None, None, None, None, 0, None,
                         None, None) == 1
    assert lib.ttie_broadphase(None, None, 0, None, None, 0, None, None) == 1
    assert lib.ttie_hvp(None, None, None, None, 0, None) == 1
    with pytest.raises(ttie.TTIEError):
        ttie.Context(0)
