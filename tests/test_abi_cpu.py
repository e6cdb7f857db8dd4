"""CPU checks of the C ABI boundary: the library loads, exports every entry
point that include/rid.h declares, and rejects bad arguments before touching
the GPU (no compute call is made here)."""
import ctypes
import os
import re

import pytest

import paper_1205_3830_amd as rid

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rid.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:rid_status|const char \*|int)\s*(rid_\w+)\s*\(",
                                 src, flags=re.M)))


def test_header_declares_the_five_steps():
    names = _declared()
    for n in ["rid_sketch", "rid_pivqr", "rid_interp", "rid_residual", "rid_decompose"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = rid.load()
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(rid.EXPORTED) == _declared()


def test_status_strings():
    assert rid.rid_status_string(rid.RID_OK) == "RID_OK"
    assert rid.rid_status_string(rid.RID_ERR_RANK) == "RID_ERR_RANK"
    assert rid.rid_status_string(99) == "RID_ERR_UNKNOWN"


def test_null_handle_and_bad_args_rejected_without_gpu():
    lib = rid.load()
    P = ctypes.c_void_p
    assert lib.rid_create(None, 0) == rid.RID_ERR_INVALID_ARG
    assert lib.rid_destroy(None) == rid.RID_OK
    assert lib.rid_pivqr(None, None, 10, 20, 5, P(16), 10, P(16), None, 1e-12) == \
        rid.RID_ERR_INVALID_ARG
    assert lib.rid_interp(None, None, 20, 5, P(16), 5, P(16), P(16), 5) == \
        rid.RID_ERR_INVALID_ARG
    assert lib.rid_reserve(None, 1, 1, 1, 1) == rid.RID_ERR_INVALID_ARG
    assert lib.rid_last_hip_error(None) == 0
    # the serving entry points check their arguments before touching a device
    cfg = rid.rid_server_config(1 << 30, 1 << 20, 1, 1, 8)
    admit = rid.ADMIT_FN(lambda *a: 1)
    done = rid.DONE_FN(lambda *a: None)
    h = rid._P()
    assert lib.rid_server_create(None, 0, ctypes.byref(cfg), admit, done, None) == \
        rid.RID_ERR_INVALID_ARG
    assert lib.rid_server_create(ctypes.byref(h), 0, None, admit, done, None) == \
        rid.RID_ERR_INVALID_ARG
    for bad in (rid.rid_server_config(0, 1, 1, 1, 8), rid.rid_server_config(1, 1, 1, 0, 8),
                rid.rid_server_config(1, 1, -1, 1, 8), rid.rid_server_config(1, 1, 1, 1, 0)):
        assert lib.rid_server_create(ctypes.byref(h), 0, ctypes.byref(bad), admit, done,
                                     None) == rid.RID_ERR_INVALID_ARG
    req = rid.rid_request(100, 50, 5, 10, rid.RID_C128, rid.RID_FP64, 0, 4, 1, 1e-12, 0)
    t = rid._U64(0)
    assert lib.rid_server_submit(None, ctypes.byref(req), ctypes.byref(t)) == \
        rid.RID_ERR_INVALID_ARG
    assert lib.rid_server_drain(None) == rid.RID_ERR_INVALID_ARG
    assert lib.rid_server_stats(None, None, None, None) == rid.RID_ERR_INVALID_ARG
    assert lib.rid_server_destroy(None) == rid.RID_ERR_INVALID_ARG
    assert lib.rid_set_batch_plan(None, 1024, 1 << 18, 8) == rid.RID_ERR_INVALID_ARG
    assert lib.rid_set_qr(None, 0) == rid.RID_ERR_INVALID_ARG
    assert lib.rid_get_batch_plan(None, None, None, None) == rid.RID_ERR_INVALID_ARG
    assert lib.rid_tune_batched(None, None, 0, 0, None, 1, 1, None, None, None) == \
        rid.RID_ERR_INVALID_ARG
    assert lib.rid_svd(None, None, 0, 100, 50, 5, P(16), 100, P(16), P(16), 5, P(16), 100,
                       P(16), P(16), 50, None) == rid.RID_ERR_INVALID_ARG


def test_binding_functions_carry_the_c_names():
    for name in rid.EXPORTED:
        assert callable(getattr(rid, name)), name


def test_package_has_no_cpu_fallback():
    # the product package never imports the oracle
    pkg = os.path.join(ROOT, "paper_1205_3830_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "rid_oracle" not in text, f
