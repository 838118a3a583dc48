"""C-ABI checks that need no GPU: the library loads, exports every entry
point that include/rt.h declares, and rejects bad parameters before touching
the device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rt.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(rt_[a-z_]+)\s*\(", txt)))


def test_header_declares_the_four_hot_path_calls():
    names = declared_functions()
    for f in ("rt_build_cells", "rt_gradient", "rt_transport", "rt_adjoint"):
        assert f in names


def test_library_exports_every_declared_symbol():
    from paper_2302_12727_amd import rt
    L = rt.load_library()
    missing = [f for f in declared_functions() if not hasattr(L, f)]
    assert not missing, missing
    assert set(declared_functions()) == set(rt.EXPORTED)


@pytest.mark.parametrize("field,value,msg", [
    ("n", 0, "n must be"),
    ("groups", 0, "groups"),
    ("groups", 9, "groups"),
    ("precision", 7, "precision"),
    ("box", -1.0, "box"),
    ("eta", 0.0, "eta"),
    ("c_red", float("nan"), "c_red"),
    ("cfl", 0.0, "cfl"),
])
def test_create_rejects_bad_params(field, value, msg):
    from paper_2302_12727_amd import rt
    L = rt.load_library()
    p = rt.rt_params(1000, 3, 0, 1.0, 1.2348, 1.825742, 1.0, 0.9, None)
    setattr(p, field, value)
    out = ctypes.c_void_p()
    st = L.rt_create(ctypes.byref(p), ctypes.byref(out))
    assert st == rt.RT_EINVAL
    assert out.value is None
    assert msg in L.rt_last_error(None).decode()


def test_null_arguments_rejected():
    from paper_2302_12727_amd import rt
    L = rt.load_library()
    assert L.rt_create(None, None) == rt.RT_EINVAL
    assert L.rt_sync(None) == rt.RT_EINVAL
    assert L.rt_transport(None, None, None, None, None, None, None, None, None) == rt.RT_EINVAL


def test_product_path_fails_loudly_without_library(tmp_path, monkeypatch):
    from paper_2302_12727_amd import rt
    monkeypatch.setattr(rt, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(rt, "_lib", None)
    with pytest.raises(ImportError):
        rt.load_library()
