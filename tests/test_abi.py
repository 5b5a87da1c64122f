"""CPU-side checks of the C ABI: the library loads, exports every symbol the
header declares, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import pytest

from paper_2004_12484_amd import enuf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(enuf_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    lib = enuf.load_library()
    names = _declared()
    assert "enuf_create" in names and "enuf_energy_forces" in names
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(enuf.EXPORTS) >= {n for n in names if n.startswith("enuf_") and not n.startswith("enuf_mlp")}


def _create(box=(10.0, 10.0, 10.0), n=100, alpha=1.0, rc=3.0, M=(32, 32, 32), p=4, prec=0):
    lib = enuf.load_library()
    h = ctypes.c_void_p()
    st = lib.enuf_create(ctypes.byref(h), (ctypes.c_double * 3)(*box), n, alpha, rc,
                         (ctypes.c_int32 * 3)(*M), p, prec, None)
    return st, h


@pytest.mark.parametrize("kw,status", [
    (dict(n=0), enuf.ENUF_EINVAL),
    (dict(n=-5), enuf.ENUF_EINVAL),
    (dict(box=(10.0, 0.0, 10.0)), enuf.ENUF_EINVAL),
    (dict(box=(10.0, float("nan"), 10.0)), enuf.ENUF_EINVAL),
    (dict(alpha=0.0), enuf.ENUF_EINVAL),
    (dict(alpha=float("inf")), enuf.ENUF_EINVAL),
    (dict(rc=-1.0), enuf.ENUF_EINVAL),
    (dict(M=(32, 48, 32)), enuf.ENUF_EINVAL),
    (dict(M=(4, 32, 32)), enuf.ENUF_EINVAL),
    (dict(M=(2048, 32, 32)), enuf.ENUF_EINVAL),
    (dict(p=5), enuf.ENUF_EINVAL),
    (dict(p=8, M=(8, 32, 32)), enuf.ENUF_EINVAL),
    (dict(prec=7), enuf.ENUF_EINVAL),
    (dict(rc=5.1), enuf.ENUF_EUNSUPPORTED),
])
def test_create_rejects_invalid_arguments(kw, status):
    st, h = _create(**kw)
    assert st == status
    assert not h.value
    assert enuf.load_library().enuf_last_error(None)


def test_null_handles():
    lib = enuf.load_library()
    assert lib.enuf_destroy(None) == enuf.ENUF_EINVAL
    assert lib.enuf_set_option(None, 0, 1.0) == enuf.ENUF_EINVAL
    assert lib.enuf_energy_forces(None, None, None, None, None, None) == enuf.ENUF_EINVAL
    assert lib.enuf_energy_grad(None, 1.0, None, None) == enuf.ENUF_EINVAL
    assert lib.enuf_create(None, None, 1, 1.0, 1.0, None, 4, 0, None) == enuf.ENUF_EINVAL


def test_status_strings():
    lib = enuf.load_library()
    for s in range(7):
        assert lib.enuf_status_string(s)
    assert lib.enuf_status_string(99) == b"unknown status"


def test_valid_request_without_device_is_device_error():
    lib = enuf.load_library()
    if lib.enuf_device_count() > 0:
        pytest.skip("a GPU is present")
    st, h = _create()
    assert st == enuf.ENUF_EDEVICE
    assert not h.value


def test_python_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(RuntimeError):
        enuf.Enuf((10.0, 10.0, 10.0), 10, 1.0, 3.0, (16, 16, 16), 4)
