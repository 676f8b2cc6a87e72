"""CPU-side checks of the C ABI boundary: the library loads and exports every
entry point that include/vopp.h declares; validation errors need no GPU."""

import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vopp.h")


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"\b(vopp_[a-z0-9_]+)\s*\(", src)
    return sorted(set(names))


def test_header_declares_the_plan_entry_point():
    names = declared_functions()
    assert "vopp_plan" in names
    assert len(names) >= 10


def test_library_exports_every_declared_symbol():
    from paper_2510_27191_amd import vopp
    L = vopp.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert set(vopp.EXPORTS) <= set(declared_functions())
    assert L.vopp_version().decode().startswith("vopp")


def _tab_desc(inst, **over):
    from paper_2510_27191_amd import vopp
    arrs = dict(rowptr=np.ascontiguousarray(inst["rowptr"], np.int32),
                col=np.ascontiguousarray(inst["col"], np.int32),
                tprob=np.ascontiguousarray(inst["tprob"], np.float32),
                zprob=np.ascontiguousarray(inst["zprob"], np.float32),
                reward=np.ascontiguousarray(inst["reward"], np.float32))
    arrs.update({k: v for k, v in over.items() if k in arrs})
    d = vopp.vopp_tabular_desc(over.get("nS", inst["nS"]), over.get("nA", inst["nA"]),
                               over.get("nO", inst["nO"]),
                               *[a.ctypes.data_as(C.c_void_p) for a in arrs.values()],
                               None, over.get("gamma", inst["gamma"]))
    return d, arrs


@pytest.mark.parametrize("bad", [
    dict(nA=0), dict(nA=4097), dict(nO=0), dict(gamma=1.0), dict(gamma=0.0),
    dict(col="oob"), dict(tprob="unnormalised"), dict(zprob="negative"),
])
def test_invalid_models_rejected_before_device_work(bad):
    from paper_2510_27191_amd import instances as I
    from paper_2510_27191_amd import vopp
    inst = I.tabular_dense(0, 5, 3, 4)
    over = dict(bad)
    if over.get("col") == "oob":
        c = inst["col"].copy()
        c[3] = 5
        over["col"] = c
    if over.get("tprob") == "unnormalised":
        t = inst["tprob"].copy()
        t[0] += 0.1
        over["tprob"] = t
    if over.get("zprob") == "negative":
        z = inst["zprob"].copy()
        z[1] = -z[1]
        over["zprob"] = z
    d, keep = _tab_desc(inst, **over)
    h = C.c_void_p()
    st = vopp.lib().vopp_pomdp_tabular(C.byref(d), C.byref(h))
    assert st == vopp.VOPP_E_INVALID
    assert h.value is None
    assert vopp.lib().vopp_last_error().decode()


def test_null_arguments_rejected():
    from paper_2510_27191_amd import vopp
    L = vopp.lib()
    assert L.vopp_pomdp_tabular(None, None) == vopp.VOPP_E_INVALID
    assert L.vopp_pomdp_nav2d(None, None) == vopp.VOPP_E_INVALID
    act = C.c_int32()
    prm = vopp.params(16)
    assert L.vopp_plan(None, None, 1, 1, 1, C.byref(prm), None, None, C.byref(act),
                       None, None, None) == vopp.VOPP_E_INVALID
    assert L.vopp_pomdp_num_actions(None) == 0
    assert L.vopp_plan_footprint(None, C.byref(prm), 1, 1) == 0
