"""The C ABI library loads on the CPU host and exports every function that
include/polyflood.h declares (no compute call: there is no GPU here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_1807_05298_amd", "libpolyflood.so")


def _declared():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(pf_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_header_declares_entry_points():
    names = _declared()
    assert "pf_create" in names and "pf_step" in names and len(names) >= 10


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_binding_loads_and_defaults():
    from paper_1807_05298_amd import polyflood as pf
    o = pf.default_opts()
    assert o.restart == 30 and o.max_newton == 12 and o.inexact == 1
    for n in pf.EXPORTED:
        assert hasattr(pf._lib, n)


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_workspace_size_and_validation_on_host():
    """pf_workspace_size runs on the host only; invalid models are rejected."""
    from paper_1807_05298_amd import inputs as I
    from paper_1807_05298_amd import polyflood as pf
    c = I.case_c1()
    nbytes = pf.workspace_size(c)
    n = c.n
    assert nbytes > 63 * n * 8            # at least the Jacobian
    bad = c.copy()
    bad.wells[0].ix = 99
    with pytest.raises(pf.PFError) as e:
        pf.workspace_size(bad)
    assert e.value.status == pf.PF_EINVAL
    with pytest.raises(pf.PFError):
        pf.workspace_size(c, pf.default_opts(restart=100))


@pytest.mark.skipif(not os.path.exists(LIB), reason="library not built")
def test_fusion_and_server_argument_checks_on_host():
    """The fusion-group and server entry points reject bad arguments before
    touching the device."""
    from paper_1807_05298_amd import polyflood as pf
    lib = pf._lib
    vp = ctypes.c_void_p
    assert lib.pf_fusion_step(None, 1, None, None, None) == pf.PF_EINVAL
    assert lib.pf_fusion_join(None, None) == pf.PF_EINVAL
    assert lib.pf_fusion_leave(None) == pf.PF_EINVAL
    assert lib.pf_fusion_stats(None, None, None, None) == pf.PF_EINVAL
    assert lib.pf_fusion_create(None, None) == pf.PF_EINVAL
    out = vp()
    # more fusion groups than slots, a misaligned arena, too many slots
    assert lib.pf_server_create(vp(256), 1 << 20, 2, 3, ctypes.byref(out)) == pf.PF_EINVAL
    assert lib.pf_server_create(vp(100), 1 << 20, 2, 0, ctypes.byref(out)) == pf.PF_EINVAL
    assert lib.pf_server_create(vp(256), 1 << 20, 65, 0, ctypes.byref(out)) == pf.PF_EINVAL
    assert lib.pf_server_release(None, 1) == pf.PF_EINVAL
