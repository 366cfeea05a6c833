"""CPU checks of the C-ABI library: it loads, exports every function that
include/emx.h declares, rejects bad handles and arguments before touching the
device, and the Python binding fails loudly when the library is missing.
No kernel is launched here."""

import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "emx.h")
LIB = os.path.join(ROOT, "paper_1501_03879_amd", "libemx.so")


def _ensure_built():
    if not os.path.exists(LIB):
        from paper_1501_03879_amd import build
        build.build(force=False)
    return C.CDLL(LIB)


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:em_status_t|const char \*)\s*(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ("em_create", "em_destroy", "em_solve_batch", "em_solve_plain", "nlem_denoise",
                 "nlem_denoise_multi", "nlem_denoise_ex", "nlm_denoise", "em_solve_batch_ex", "em_solve_plain_ex",
                 "em_sync", "nlem_autotune", "nlem_plan", "nlem_plan_get", "nlem_plan_set", "em_batch_autotune",
                 "em_batch_plan_get", "em_batch_plan_set", "em_kernel_timing", "em_kernel_timing_read",
                 "em_status_string", "em_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = _ensure_built()
    for name in declared_functions():
        assert hasattr(lib, name), f"libemx.so does not export {name}"


def test_struct_sizes_match_the_header():
    from synth.pointsets import INSTANCE_DTYPE
    import paper_1501_03879_amd as emx
    assert INSTANCE_DTYPE.itemsize == 32                     # em_instance_t
    assert C.sizeof(emx.NlemImage) == 8 * 3 + 4 * 6          # nlem_image_t
    assert C.sizeof(emx.NlemOptions) == 4 * 8                # nlem_options_t
    assert C.sizeof(emx.EmOptions) == 4 * 4 + 8 * 2 + 4 * 8 + 8 + 8 * 2 + 8   # em_options_t
    assert C.sizeof(emx.NlemPlan) == 4 * 6                   # nlem_plan_t
    assert C.sizeof(emx.BatchPlan) == 8 + 4 * 4              # em_batch_plan_t


def test_null_handle_is_rejected_without_device_work():
    lib = _ensure_built()
    vp = C.c_void_p
    lib.em_solve_batch.argtypes = [vp, vp, C.c_int64, vp, vp, vp, C.c_float, C.c_float, C.c_float,
                                   C.c_int32, C.c_float, C.c_int32, vp, vp]
    lib.nlem_denoise.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                 C.c_float, C.c_float, C.c_float, C.c_float, C.c_int32, C.c_float, vp, vp]
    lib.em_sync.argtypes = [vp, vp]
    lib.em_destroy.argtypes = [vp]
    assert lib.em_solve_batch(None, None, 1, None, None, None, 0, 1, 1, 1, 0, 0, None, None) == -1
    assert lib.nlem_denoise(None, None, None, 0, 8, 8, 1, 1, 1.0, 0, 255, 1e-3, 1, 0, None, None) == -1
    lib.em_solve_batch_ex.argtypes = [vp, vp, C.c_int64, vp, vp, vp, vp, vp, vp]
    assert lib.em_solve_batch_ex(None, None, 1, None, None, None, None, None, None) == -1
    lib.em_solve_plain_ex.argtypes = [vp, vp, C.c_int64, vp, vp, vp, vp, vp, vp, vp]
    assert lib.em_solve_plain_ex(None, None, 1, None, None, None, None, None, None, None) == -1
    lib.nlem_denoise_ex.argtypes = [vp, vp, C.c_int32, vp, vp]
    assert lib.nlem_denoise_ex(None, None, 0, None, None) == -1
    lib.nlm_denoise.argtypes = [vp, vp, vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                                C.c_float, vp]
    assert lib.nlm_denoise(None, None, None, 0, 8, 8, 1, 1, 1.0, None) == -1
    lib.nlem_autotune.argtypes = [vp, vp, vp, vp, C.c_int32, vp]
    assert lib.nlem_autotune(None, None, None, None, 1, None) == -1
    lib.nlem_plan.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, vp]
    assert lib.nlem_plan(None, 3, 10, 0, None) == -1
    lib.nlem_plan_get.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp]
    assert lib.nlem_plan_get(None, 3, 10, 0, 0, None) == -1
    lib.nlem_plan_set.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32, C.c_int32, vp]
    assert lib.nlem_plan_set(None, 3, 10, 0, 0, None) == -1
    lib.em_batch_autotune.argtypes = [vp, vp, C.c_int64, vp, vp, vp, vp, vp, vp, C.c_int32, vp]
    assert lib.em_batch_autotune(None, None, 1, None, None, None, None, None, None, 1, None) == -1
    lib.em_batch_plan_get.argtypes = [vp, C.c_int32, C.c_int32, vp]
    assert lib.em_batch_plan_get(None, 0, 0, None) == -1
    lib.em_batch_plan_set.argtypes = [vp, C.c_int32, C.c_int32, vp]
    assert lib.em_batch_plan_set(None, 0, 0, None) == -1
    lib.em_kernel_timing.argtypes = [vp, C.c_int32]
    assert lib.em_kernel_timing(None, 1) == -1
    lib.em_kernel_timing_read.argtypes = [vp, vp, vp]
    assert lib.em_kernel_timing_read(None, None, None) == -1
    assert lib.em_sync(None, None) == -1
    assert lib.em_destroy(None) == 0
    lib.em_create.argtypes = [C.POINTER(vp), C.c_int]
    assert lib.em_create(None, 0) == -1


def test_status_strings():
    lib = _ensure_built()
    lib.em_status_string.restype = C.c_char_p
    lib.em_status_string.argtypes = [C.c_int]
    assert lib.em_status_string(0) == b"EM_OK"
    assert lib.em_status_string(-1) == b"EM_ERR_INVALID_ARG"
    assert lib.em_status_string(-2) == b"EM_ERR_UNSUPPORTED"
    assert lib.em_status_string(-4) == b"EM_ERR_HIP"


def test_binding_fails_loudly_without_library(monkeypatch):
    import paper_1501_03879_amd as emx
    monkeypatch.setattr(emx, "LIB_PATH", os.path.join(ROOT, "no_such_libemx.so"))
    monkeypatch.setattr(emx, "_lib", None)
    with pytest.raises(RuntimeError, match="build the HIP library"):
        emx.load_library()


def test_instances_tensor_bytes_roundtrip():
    import torch
    import synth
    import paper_1501_03879_amd as emx
    b = synth.make_pointset_batch(3, 17, n_hi=40)
    t = emx.instances_tensor(b.inst, "cpu")
    assert t.dtype == torch.int64 and t.shape == (17, 4)
    back = t.numpy().view(synth.pointsets.INSTANCE_DTYPE).reshape(-1)
    np.testing.assert_array_equal(back, b.inst)


def test_c_client_links_against_the_library():
    """The C example client is plain C on include/emx.h, linked to libemx.so
    in the package directory; without arguments it prints its usage and
    exits 1 before any HIP call (runs without a GPU)."""
    import subprocess
    from paper_1501_03879_amd import build
    _ensure_built()
    if not os.path.exists(build.CLIENT):
        build.build_client()
    r = subprocess.run([build.CLIENT], capture_output=True, text=True, timeout=60)
    assert r.returncode == 1 and "usage:" in r.stderr
    ldd = subprocess.run(["ldd", build.CLIENT], capture_output=True, text=True, timeout=60).stdout
    assert os.path.realpath(LIB) in {os.path.realpath(tok) for tok in ldd.split() if tok.endswith("libemx.so")}
