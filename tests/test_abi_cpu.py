"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
symbol the header declares, and rejects invalid configurations before touching
the device."""
import ctypes
import os
import re

import pytest

from paper_1408_6299_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nkreg.h")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nkreg_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = _lib.load()
    names = declared_symbols()
    assert len(names) >= 20
    for name in names:
        assert hasattr(lib, name), name
    assert set(names) == set(_lib.SIGNATURES), set(names) ^ set(_lib.SIGNATURES)


def test_version_and_status_strings():
    lib = _lib.load()
    assert lib.nkreg_version().decode().startswith("nkreg")
    for code in range(-9, 1):
        assert lib.nkreg_status_string(code).decode() != "unknown status"


def make_cfg(**kw):
    c = _lib.Config()
    c.dim = kw.get("dim", 2)
    n = kw.get("n", (64, 64, 1))
    for i in range(3):
        c.n[i] = n[i]
    c.nt = kw.get("nt", 16)
    c.nc = kw.get("nc", 1)
    c.reg = kw.get("reg", 1)
    c.incompressible = kw.get("incompressible", 0)
    c.beta = kw.get("beta", 1e-2)
    c.precision = kw.get("precision", 32)
    c.checkpoint_every = kw.get("checkpoint_every", 0)
    c.trajectory_slots = kw.get("trajectory_slots", 1)
    c.cfl_max = 0.0
    return c


@pytest.mark.parametrize("kw,code", [
    (dict(dim=4), _lib.EINVAL),
    (dict(reg=3), _lib.EINVAL),
    (dict(beta=0.0), _lib.EINVAL),
    (dict(beta=-1.0), _lib.EINVAL),
    (dict(nt=0), _lib.EINVAL),
    (dict(nc=0), _lib.EINVAL),
    (dict(nc=17), _lib.EINVAL),
    (dict(precision=16), _lib.EINVAL),
    (dict(n=(48, 64, 1)), _lib.ESHAPE),
    (dict(n=(63, 64, 1)), _lib.ESHAPE),
    (dict(n=(4, 64, 1)), _lib.ESHAPE),
    (dict(n=(1024, 64, 1)), _lib.ESHAPE),
    (dict(dim=3, n=(64, 64, 12)), _lib.ESHAPE),
    (dict(checkpoint_every=-1), _lib.EINVAL),
    (dict(checkpoint_every=2, trajectory_slots=-1), _lib.EINVAL),
])
def test_invalid_configs_are_rejected_before_any_device_work(kw, code):
    lib = _lib.load()
    h = ctypes.c_void_p()
    st = lib.nkreg_create(ctypes.byref(make_cfg(**kw)), None, ctypes.byref(h))
    assert st == code
    assert not h.value
    assert lib.nkreg_last_error().decode()


def test_null_arguments_are_rejected():
    lib = _lib.load()
    assert lib.nkreg_create(None, None, None) == _lib.EINVAL
    h = ctypes.c_void_p()
    assert lib.nkreg_create(None, None, ctypes.byref(h)) == _lib.EINVAL
    assert lib.nkreg_destroy(None) == _lib.OK
    assert lib.nkreg_hessian_matvec(None, None, None) == _lib.EINVAL
    assert lib.nkreg_batch_create(-1, None, None, ctypes.byref(h)) == _lib.EINVAL
    assert lib.nkreg_batch_wrap(-1, None, ctypes.byref(h)) == _lib.EINVAL
    assert lib.nkreg_batch_item(None, 0, ctypes.byref(h)) == _lib.EINVAL
    assert lib.nkreg_batch_set_state(None, None) == _lib.EINVAL
    assert lib.nkreg_batch_pcg(None, None, None, 1e-3, 10, None, None) == _lib.EINVAL


def test_launch_floor_validates_its_arguments_before_any_device_work():
    lib = _lib.load()
    us = ctypes.c_double()
    for args in ((0, 512, 256, 200, None, None), (4, 512, 256, 200, None, ctypes.byref(us)),
                 (1, 100, 256, 200, None, ctypes.byref(us)), (2, 512, 8192, 200, None, ctypes.byref(us)),
                 (3, 512, 256, 1, None, ctypes.byref(us))):
        assert lib.nkreg_launch_floor(*args) == _lib.EINVAL, args


def test_batch_create_validates_every_configuration_before_any_device_work():
    lib = _lib.load()
    cfgs = (_lib.Config * 2)(make_cfg(), make_cfg(n=(48, 64, 1)))
    h = ctypes.c_void_p()
    assert lib.nkreg_batch_create(2, cfgs, None, ctypes.byref(h)) == _lib.ESHAPE
    assert not h.value
    cfgs = (_lib.Config * 2)(make_cfg(), make_cfg(beta=-1.0))
    assert lib.nkreg_batch_create(2, cfgs, None, ctypes.byref(h)) == _lib.EINVAL


def test_check_raises_with_message():
    with pytest.raises(_lib.NkregError) as ei:
        _lib.check(_lib.ESTATE, "where")
    assert ei.value.status == _lib.ESTATE


def test_product_path_has_no_oracle_or_cpu_fallback():
    """The package never imports the oracle and refuses to load without libnkreg.so."""
    pkg = os.path.join(ROOT, "paper_1408_6299_amd")
    for fn in os.listdir(pkg):
        if fn.endswith(".py"):
            src = open(os.path.join(pkg, fn)).read()
            assert "oracle" not in src.replace("oracle is the oracle", ""), fn
            assert "import numpy" not in src or fn == "build.py", fn
    with pytest.raises(ImportError):
        _lib.load.__wrapped__ if hasattr(_lib.load, "__wrapped__") else None
        saved = _lib._lib
        try:
            _lib._lib = None
            _lib.load(os.path.join(ROOT, "no_such_lib.so"))
        finally:
            _lib._lib = saved
