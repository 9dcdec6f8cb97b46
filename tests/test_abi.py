"""CPU checks of the C-ABI library: it loads, exports every function that
include/lbm.h declares, the binding covers the same names, and argument
validation fails cleanly without touching a device."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def declared_functions(path):
    text = open(path).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(lbm\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_core_calls():
    names = declared_functions(os.path.join(ROOT, "include", "lbm.h"))
    for core in ("lbm_create", "lbm_step", "lbm_moments", "lbm_probe", "lbm_destroy"):
        assert core in names


def test_library_exports_every_declared_symbol():
    from paper_2211_05009_amd import lbm
    lib = ct.CDLL(lbm.LIB_PATH)
    for h in HEADERS:
        for name in declared_functions(h):
            assert hasattr(lib, name), f"{name} declared in {os.path.basename(h)} but not exported"


def test_binding_covers_every_declared_symbol():
    from paper_2211_05009_amd import lbm
    names = declared_functions(os.path.join(ROOT, "include", "lbm.h"))
    assert sorted(lbm.SIGNATURES) == names
    for name in names:
        assert callable(getattr(lbm, name))


def test_argument_validation_without_device():
    from paper_2211_05009_amd import lbm
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(1, 10, 100.0, 0.1, "f64")
    assert e.value.code == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(10, 10, -1.0, 0.1, "f64")
    assert e.value.code == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(10, 10, 100.0, 0.6, "f64")        # |u| >= c_s
    assert e.value.code == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create_tau(10, 10, 0.5, 0.1, "f64")      # tau <= 1/2
    assert e.value.code == lbm.LBM_EINVAL
    with pytest.raises(lbm.LbmError) as e:
        lbm.lbm_create(10, 10, 100.0, 0.1, 7)
    assert e.value.code == lbm.LBM_EINVAL
    assert "lbm" in lbm.lbm_version()
    # NULL handle is rejected, lbm_destroy(NULL) is a no-op
    assert lbm._lib.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert lbm._lib.lbm_destroy(None) == lbm.LBM_OK
