"""The C-ABI library (CPU checks: no kernel is launched here)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", h)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names.update(re.findall(r"^\s*(?:int|void|const char\s*\*)\s*(pic_\w+)\s*\(", src, re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_2109_04469_amd import capi

    return capi.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 35
    assert "pic_batch_step" in names and "pic_mlp_train_step" in names and "pic_load_profile" in names
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_library_is_the_in_tree_build(lib):
    from paper_2109_04469_amd import capi

    assert os.path.dirname(capi.LIB_PATH) == os.path.join(ROOT, "paper_2109_04469_amd")


def _structs(**over):
    from paper_2109_04469_amd.discharge import make_params, make_xsec
    from pic_inputs import workloads, xsec

    p = dict(workloads.get("c1_small")["params"])
    p.update(over)
    xs = xsec.argon_synthetic()
    pp = make_params(p)
    xx, keep = make_xsec(xs)
    return pp, xx, keep


def test_workspace_size_and_validation(lib):
    from paper_2109_04469_amd import capi

    pp, xx, keep = _structs()
    n = ctypes.c_uint64()
    assert lib.pic_workspace_bytes(ctypes.byref(pp), ctypes.byref(xx), ctypes.byref(n)) == 0
    # at least the four ping-pong SoA streams of both species
    assert n.value >= 2 * 2 * 4 * 8 * 40_000
    for bad in (dict(n_cells=1), dict(n_cells=5000), dict(gap_m=0.0), dict(reflection=1.5),
                dict(gamma_see=-0.1), dict(capacity=(-1, 10)), dict(ion_subcycle=0),
                dict(eepf_bins=0), dict(steps_per_cycle=0), dict(flags=1 << 10)):
        pp, xx, keep = _structs(**bad)
        assert lib.pic_workspace_bytes(ctypes.byref(pp), ctypes.byref(xx), ctypes.byref(n)) == \
            capi.PIC_EINVAL, bad
    # a larger grid or capacity needs more workspace
    pp, xx, keep = _structs(capacity=(80_000, 80_000))
    m = ctypes.c_uint64()
    assert lib.pic_workspace_bytes(ctypes.byref(pp), ctypes.byref(xx), ctypes.byref(m)) == 0
    assert m.value > n.value


def test_strerror_covers_codes(lib):
    for s in range(0, -7, -1):
        msg = lib.pic_strerror(s).decode()
        assert msg and msg != "unknown status"


def test_init_rejects_bad_workspace(lib):
    pp, xx, keep = _structs()
    h = ctypes.c_void_p()
    assert lib.pic_init(ctypes.byref(pp), ctypes.byref(xx), None, 0, None, ctypes.byref(h)) == -1
