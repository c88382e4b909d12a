"""C ABI checks that need no GPU: the library loads, exports every function
declared in include/*.h, and rejects bad arguments before touching a device."""

import ctypes
import os
import re

import pytest

from paper_2604_07276_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"^\s*(?:const\s+)?\w+\s*\**\s*(dp_\w+)\s*\(", src,
                                flags=re.M))
    return sorted(names)


def test_header_lists_the_abi():
    names = _declared_functions()
    assert set(names) == set(binding.EXPORTED), names


def test_library_exports_every_declared_symbol():
    lib = binding.load_library()
    for name in _declared_functions():
        assert hasattr(lib, name), name


def _create(path, rcut=6.0, sel=120):
    lib = binding.load_library()
    h = ctypes.c_void_p()
    rc = lib.dp_create(path.encode() if path is not None else None, rcut, sel, ctypes.byref(h))
    return rc, lib.dp_last_error().decode()


def test_create_rejects_missing_file(tmp_path):
    rc, msg = _create(str(tmp_path / "nope.bin"))
    assert rc == -5 and "cannot open" in msg


def test_create_rejects_foreign_file(tmp_path):
    p = tmp_path / "junk.bin"
    p.write_bytes(b"not a weights file at all")
    rc, msg = _create(str(p))
    assert rc == -5


def test_create_rejects_bad_sel_and_rcut(weights_path):
    assert _create(weights_path, sel=0)[0] == -1
    assert _create(weights_path, sel=129)[0] == -1
    assert _create(weights_path, rcut=-1.0)[0] == -1
    assert _create(None)[0] == -1


def test_calls_with_null_handle_fail_cleanly():
    lib = binding.load_library()
    assert lib.dp_compute(None, None, None, None, 0, 0, None, None, None, None) == -1
    assert lib.dp_sync(None) == -1
    assert lib.dp_set_precision(None, 0) == -1
    assert lib.dp_debug_nlist(None, None, None) == -1
    lib.dp_destroy(None)


def test_create_without_device_reports_device_error(weights_path):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    rc, msg = _create(weights_path)
    assert rc == -6, msg


def test_trainer_calls_reject_bad_arguments(weights_path):
    lib = binding.load_library()
    h = ctypes.c_void_p()
    assert lib.dp_train_create(weights_path.encode(), 6.0, 120, None, ctypes.byref(h)) == -1
    opt = binding.TrainOptions(1.0, 100.0, 1.5, 0.999, 1e-8, 0)  # beta1 out of range
    assert lib.dp_train_create(weights_path.encode(), 6.0, 120, ctypes.byref(opt),
                               ctypes.byref(h)) == -1
    opt = binding.TrainOptions(1.0, 100.0, 0.9, 0.999, 1e-8, 5)  # unknown precision
    assert lib.dp_train_create(weights_path.encode(), 6.0, 120, ctypes.byref(opt),
                               ctypes.byref(h)) == -1
    n = ctypes.c_int32()
    assert lib.dp_train_params(None, None, ctypes.byref(n)) == -1
    assert lib.dp_train_save(None, b"x") == -1
    assert lib.dp_train_gradient(None, None, None, None, 1, 1, None, None, None, None,
                                 None) == -1
    lib.dp_train_destroy(None)
    out = (ctypes.c_double * 2)()
    assert lib.dp_force_error(None, None, -1, out, None) == -1
    assert lib.dp_force_error(None, None, 0, out, None) == 0 and out[0] == 0.0


def test_memory_budget_calls_reject_bad_arguments():
    lib = binding.load_library()
    assert lib.dp_set_memory_budget(None, 1.0) == -1
    b = ctypes.c_int64()
    r = ctypes.c_int32()
    assert lib.dp_memory_info(None, ctypes.byref(b), ctypes.byref(r)) == -1
