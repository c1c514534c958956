"""The C-ABI library loads and exports every function include/sfd.h declares (no compute calls)."""

import ctypes
import os
import re

import numpy as np
import pytest

pytestmark = pytest.mark.cpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    with open(os.path.join(ROOT, "include", "sfd.h")) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sfd_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    from paper_1602_00412_amd import sfd

    if not os.path.exists(sfd.LIB_PATH):
        from paper_1602_00412_amd.build import build

        build()
    lib = ctypes.CDLL(sfd.LIB_PATH)
    names = _declared()
    assert len(names) >= 10
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(sfd.EXPORTS)


def test_strerror_and_argument_errors_without_a_gpu():
    from paper_1602_00412_amd import sfd

    lib = sfd.load()
    assert lib.sfd_strerror(sfd.SFD_E_INDEX) == b"column index out of range"
    h = ctypes.c_void_p()
    # argument checks run before any device call
    assert lib.sfd_create(10, 0, 0.25, 0, ctypes.byref(h)) == sfd.SFD_E_ARG
    assert lib.sfd_create(10, 11, 0.25, 0, ctypes.byref(h)) == sfd.SFD_E_ARG
    assert lib.sfd_create(100, 5, 1.5, 0, ctypes.byref(h)) == sfd.SFD_E_ARG
    assert lib.sfd_create(1 << 30, 5, 0.25, 0, ctypes.byref(h)) == sfd.SFD_E_ARG
    assert lib.sfd_destroy(None) == sfd.SFD_OK
    assert lib.sfd_merge(None, None) == sfd.SFD_E_ARG
    res = sfd.EvalResult()
    assert lib.sfd_evaluate(10, 5, None, None, None, None, 0, 0, 0, 0, None, ctypes.byref(res)) == sfd.SFD_E_ARG
    assert lib.sfd_evaluate(10, 0, None, None, None, None, 0, 0, 0, 0, None, None) == sfd.SFD_E_ARG


def test_batch_argument_errors_without_a_gpu():
    from paper_1602_00412_amd import sfd

    lib = sfd.load()
    h = ctypes.c_void_p()
    assert lib.sfd_batch_create(0, 100, 5, 0.25, 0, ctypes.byref(h)) == sfd.SFD_E_ARG
    assert lib.sfd_batch_create(4, 10, 11, 0.25, 0, ctypes.byref(h)) == sfd.SFD_E_ARG
    assert lib.sfd_batch_create(4, 100, 5, 0.0, 0, ctypes.byref(h)) == sfd.SFD_E_ARG
    assert lib.sfd_batch_destroy(None) == sfd.SFD_OK
    assert lib.sfd_batch_sketch(None, None, 0) == sfd.SFD_E_ARG
    assert lib.sfd_batch_append_csr(None, 0, None, None, None, None, None, 0) == sfd.SFD_E_ARG
    assert lib.sfd_batch_set_option(None, sfd.OPT_DELTA, 0.1) == sfd.SFD_E_ARG


def test_binding_constants_match_the_header():
    # every option / precision / algorithm / memory constant of the binding has the header's value
    from paper_1602_00412_amd import sfd

    with open(os.path.join(ROOT, "include", "sfd.h")) as f:
        text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
    values = {name: int(v) for name, v in re.findall(r"\bSFD_([A-Z0-9_]+)\s*=\s*(-?\d+)", text)}
    for prefix in ("OPT_", "PRECISION_", "ALGO_", "MEM_"):
        names = [n for n in values if n.startswith(prefix)]
        assert names
        for n in names:
            assert getattr(sfd, n) == values[n], n


def test_evaluate_binding_checks_its_arguments_without_a_gpu():
    # host tensors and wrong dtypes are refused before the library is called
    import torch

    from paper_1602_00412_amd import sfd

    p = torch.zeros(2, dtype=torch.int64)
    i = torch.zeros(1, dtype=torch.int32)
    v = torch.zeros(1, dtype=torch.float32)
    with pytest.raises(TypeError):
        sfd.evaluate(p, i, v, 4)
    with pytest.raises(TypeError):
        sfd.evaluate(p, i.to(torch.int64), v, 4)


def test_output_buffers_are_checked_without_a_gpu():
    # a caller-supplied output must hold exactly the sketch's FP32 values contiguously, in the
    # memory kind asked for; anything else is refused before the library is called
    import torch

    from paper_1602_00412_amd import sfd

    good = np.empty((3, 5), np.float32)
    assert sfd._out_ptr(good, (3, 5), False) == good.ctypes.data
    ro = np.empty((3, 5), np.float32)
    ro.flags.writeable = False
    for bad in (np.empty((3, 4), np.float32), np.empty((3, 5), np.float64), np.empty((5, 3), np.float32).T, ro,
                torch.empty((3, 5))):
        with pytest.raises(TypeError):
            sfd._out_ptr(bad, (3, 5), False)
    with pytest.raises(TypeError):
        sfd._out_ptr(torch.empty((3, 5), dtype=torch.float32), (3, 5), True)  # host tensor, device asked


def test_missing_library_fails_loudly():
    # no fallback: without the built HIP library the binding raises instead of computing anything
    import subprocess
    import sys

    code = ("import paper_1602_00412_amd.sfd as s\n"
            "try:\n    s.load('/nonexistent/libsfd.so')\nexcept RuntimeError as e:\n    print('raised', e)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.startswith("raised"), r.stdout + r.stderr
