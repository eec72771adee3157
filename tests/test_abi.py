"""CPU checks of the C ABI: the library loads, exports every declared symbol,
and its host-side validation behaves (no device call is made here)."""

import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2103_04081_amd", "libcpdmi.so")

pytestmark = pytest.mark.skipif(not os.path.exists(LIB), reason="libcpdmi.so not built")


def declared_symbols():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        names.update(re.findall(r"CPD_API\s+[\w\s\*]+?\b(cpd_\w+)\s*\(", text))
    return sorted(names)


def test_headers_declare_entry_points():
    names = declared_symbols()
    for must in ("cpd_init", "cpd_sample", "cpd_step", "cpd_step_replay", "cpd_fit",
                 "cpd_workspace_size", "cpd_read_state", "cpd_write_state"):
        assert must in names, must


def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_symbols() if not hasattr(lib, n)]
    assert not missing, missing


def test_workspace_size_and_validation():
    import paper_2103_04081_amd as P
    p = P.make_problem([300, 300, 300], 10, 256)
    o = P.make_options(storage="f32")
    n = P.cpd_workspace_size(p, o)
    # three padded FP32 copies of 300^3 (rows of 320) plus small state
    assert 3 * 90000 * 320 * 4 < n < 3 * 90000 * 320 * 4 + (1 << 20)
    ob = P.make_options(storage="bf16")
    assert P.cpd_workspace_size(p, ob) < n
    with pytest.raises(P.CpdError) as e:
        P.cpd_workspace_size(P.make_problem([300, 300, 300], 0, 256), o)
    assert e.value.status == -1
    with pytest.raises(P.CpdError):
        P.cpd_workspace_size(P.make_problem([300, 300, 300], 10, 0), o)
    with pytest.raises(P.CpdError):
        P.cpd_workspace_size(P.make_problem([5], 2, 4), o)
    with pytest.raises(P.CpdError):
        P.cpd_workspace_size(p, P.make_options(sampler=7))
    # a plan that cannot fit the on-chip budget is refused up front
    with pytest.raises(P.CpdError) as e:
        P.cpd_workspace_size(P.make_problem([4096, 64, 64], 64, 4096), o)
    assert "LDS" in str(e.value)
    # every mode-major copy must stay addressable with 32-bit byte offsets
    with pytest.raises(P.CpdError) as e:
        P.cpd_workspace_size(P.make_problem([4096, 4096, 128], 8, 64), o)
    assert "4 GiB" in str(e.value)
