"""The C ABI without a GPU: the library loads, exports every declared entry
point, and rejects invalid parameter sets before touching the device."""
import ctypes as C
import os
import re

import pytest

from paper_1109_6672_amd import lbddf, workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "lbddf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lb_[a-z_]+)\s*\(", src)))


@pytest.mark.parametrize("path", [lbddf.LIB_PATH, lbddf.LIB_PATH_FP64])
def test_library_exports_every_declared_symbol(path):
    names = _declared()
    assert "lb_create" in names and "lb_step" in names and len(names) >= 18
    if not os.path.exists(path):
        pytest.skip(f"{os.path.basename(path)} not built")
    lib = C.CDLL(path)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) <= set(lbddf._SIGS), set(names) - set(lbddf._SIGS)


def test_state_bytes_layout():
    p = W.periodic(100, 30)
    n32 = lbddf.state_bytes(p)
    n16 = lbddf.state_bytes(dict(p, storage="f16"))
    pitch = 128
    assert n32 >= 2 * 18 * 4 * pitch * 30 and n16 >= 2 * 18 * 2 * pitch * 30
    assert n16 < n32


@pytest.mark.parametrize("change,msg", [
    (dict(tau_f=0.5), "tau_f"),
    (dict(R=0.3), "R*T0"),
    (dict(s_q=2.0), "s_q"),
    (dict(energy="internal", heating=True), "heating"),
    (dict(nx=0), "nx"),
    (dict(Pr=-1.0), "positive"),
])
def test_invalid_parameters_are_rejected(change, msg):
    p = W.periodic(16, 16)
    p.update(change)
    with pytest.raises(lbddf.LBError) as e:
        lbddf.validate(p)
    assert e.value.status == lbddf.LB_EINVAL and msg in str(e.value)


def test_invalid_sides_are_rejected():
    p = W.periodic(16, 16)
    p["sides"] = [W.side("wall"), W.side(), W.side(), W.side()]
    with pytest.raises(lbddf.LBError, match="both sides"):
        lbddf.validate(p)
    p = W.channel(nx=16, ny=8)
    p["sides"][2] = W.side("wall")
    p["sides"][3] = W.side("wall")
    with pytest.raises(lbddf.LBError, match="periodic y"):
        lbddf.validate(p)
    p = W.cavity(3, 1e3, 0.1, 0.1)
    with pytest.raises(lbddf.LBError, match="adiabatic"):
        lbddf.validate(p)
    p = W.couette(U=0.7)
    with pytest.raises(lbddf.LBError, match="c_s"):
        lbddf.validate(p)


def test_create_rejects_small_or_missing_buffers():
    lib = lbddf.load()
    s = lbddf.make_params(W.periodic(16, 16))
    h = C.c_void_p()
    assert lib.lb_create(C.byref(s), None, 0, None, C.byref(h)) == lbddf.LB_EINVAL
    assert lib.lb_create(C.byref(s), C.c_void_p(256), 16, None, C.byref(h)) == lbddf.LB_ENOMEM
    assert not h.value


def test_workload_recipes_validate():
    for p in (W.couette(), W.cavity(128, 1e4, 0.02, 0.02), W.cavity(64, 1e5, 1.2, 0.01, sutherland=True),
              W.periodic(1024), W.channel(), W.couette_paper(1, 0.35)):
        lbddf.validate(p)


def test_server_rejects_bad_pools_without_touching_the_device():
    lib = lbddf.load()
    h = C.c_void_p()
    assert lib.lbs_create(None, 1 << 30, 0, 10, None, C.byref(h)) == lbddf.LB_EINVAL
    assert lib.lbs_create(C.c_void_p(256), 1024, 0, 10, None, C.byref(h)) == lbddf.LB_ENOMEM
    assert lib.lbs_create(C.c_void_p(256), 1 << 30, 7, 10, None, C.byref(h)) == lbddf.LB_EINVAL
    assert lib.lbs_create(C.c_void_p(256), 1 << 30, 0, 0, None, C.byref(h)) == lbddf.LB_EINVAL
    assert not h.value
