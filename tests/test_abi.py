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
                 "cpd_workspace_size", "cpd_read_state", "cpd_write_state", "cpd_destroy",
                 "cpd_batch_workspace_size", "cpd_batch_create", "cpd_batch_step",
                 "cpd_batch_fits", "cpd_batch_run", "cpd_batch_member_info",
                 "cpd_batch_destroy", "cpd_server_create", "cpd_submit", "cpd_poll",
                 "cpd_server_stats", "cpd_server_destroy", "cpd_variance"):
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


def test_step_path_selection():
    import paper_2103_04081_amd as P
    # B beyond the persistent kernel: AUTO plans the grid step, whose
    # workspace adds up to eight R x I_max parts per gather block
    p_small = P.make_problem([300, 300, 300], 10, 256)
    p_big = P.make_problem([300, 300, 300], 10, 65536)
    o = P.make_options()
    n_small = P.cpd_workspace_size(p_small, o)
    n_big = P.cpd_workspace_size(p_big, o)
    # (slices of 128 to 512 fibres)
    assert n_big - n_small >= 65536 // 512 * 10 * 300 * 4
    assert n_big - n_small < 8 * 65536 // 128 * 10 * 300 * 4 + (1 << 16)
    # the grid path can be asked for at any B; the persistent one only up to 4096
    assert P.cpd_workspace_size(p_small, P.make_options(path="grid")) > n_small
    with pytest.raises(P.CpdError) as e:
        P.cpd_workspace_size(p_big, P.make_options(path="persistent"))
    assert "4096" in str(e.value)
    with pytest.raises(P.CpdError):
        P.cpd_workspace_size(p_small, P.make_options(path=3))
    with pytest.raises(P.CpdError) as e:
        P.cpd_workspace_size(p_big, P.make_options(ksplit=[2, 0, 0]))
    assert "grid" in str(e.value)
    with pytest.raises(P.CpdError):
        P.cpd_workspace_size(P.make_problem([300, 300, 300], 10, P.cpdmi.MAX_BATCH + 1), o)
    # batched members and served requests use the persistent step
    with pytest.raises(P.CpdError) as e:
        P.cpd_batch_workspace_size([p_small, p_big], [o, o])
    assert "persistent" in str(e.value)


def test_ksplit_option_validation():
    import paper_2103_04081_amd as P
    p = P.make_problem([40, 300, 33], 10, 256)
    # mode 0: 3 row tiles of 16 -> at most 2 parts per tile over 8 waves
    P.cpd_workspace_size(p, P.make_options(ksplit=[2, 1, 0]))
    with pytest.raises(P.CpdError) as e:
        P.cpd_workspace_size(p, P.make_options(ksplit=[4, 0, 0]))
    assert "ksplit[0]" in str(e.value)
    with pytest.raises(P.CpdError):
        P.cpd_workspace_size(p, P.make_options(ksplit=[0, 2, 0]))  # 19 tiles: no split
    with pytest.raises(P.CpdError):
        P.cpd_workspace_size(p, P.make_options(ksplit=[-1, 0, 0]))


def test_batch_workspace_size():
    import paper_2103_04081_amd as P
    dims = [[50, 60, 70], [31, 17, 9, 12], [200, 100, 50]]
    ps = [P.make_problem(d, 8, 128) for d in dims]
    os_ = [P.make_options(storage="bf16") for _ in dims]
    single = sum(P.cpd_workspace_size(p, o) for p, o in zip(ps, os_))
    n = P.cpd_batch_workspace_size(ps, os_)
    assert single < n < single + len(dims) * 256 + (1 << 16)
    # members must share the storage type and the round length
    with pytest.raises(P.CpdError):
        P.cpd_batch_workspace_size(ps, os_[:2] + [P.make_options(storage="f32")])
    with pytest.raises(P.CpdError):
        P.cpd_batch_workspace_size(ps, os_[:2] + [P.make_options(storage="bf16", fit_every=7)])
    # a bad member is named
    bad = ps[:1] + [P.make_problem([31, 17, 9, 12], 0, 128)] + ps[2:]
    with pytest.raises(P.CpdError) as e:
        P.cpd_batch_workspace_size(bad, os_)
    assert "member 1" in str(e.value)


def test_rescale_option_validation():
    import paper_2103_04081_amd as P
    p = P.make_problem([30, 20, 10], 4, 64)
    P.cpd_workspace_size(p, P.make_options(rescale_every=1))
    with pytest.raises(P.CpdError) as e:
        P.cpd_workspace_size(p, P.make_options(rescale_every=-1))
    assert "rescale_every" in str(e.value)
    # batched members are single-round persistent steps: no rescaling
    ps = [p, p]
    P.cpd_batch_workspace_size(ps, [P.make_options(), P.make_options()])
    with pytest.raises(P.CpdError) as e:
        P.cpd_batch_workspace_size(ps, [P.make_options(), P.make_options(rescale_every=5)])
    assert "member 1" in str(e.value) and "rescale_every" in str(e.value)


def test_wide_rank_planning():
    """Ranks 65..128 plan the grid step (also at the paper's Pavia shape, whose
    factor rows exceed LDS); the leverage sampler, the persistent path and
    ranks beyond 128 are refused."""
    import paper_2103_04081_amd as P
    o = P.make_options(sampler="euclidean")
    n_auto = P.cpd_workspace_size(P.make_problem([610, 340, 103], 100, 20), o)
    n_grid = P.cpd_workspace_size(P.make_problem([610, 340, 103], 100, 20),
                                  P.make_options(sampler="euclidean", path="grid"))
    assert n_auto == n_grid
    P.cpd_workspace_size(P.make_problem([40, 33, 29], 128, 60), P.make_options(sampler="uniform"))
    with pytest.raises(P.CpdError) as e:
        P.cpd_workspace_size(P.make_problem([40, 33, 29], 70, 60), P.make_options(sampler="leverage"))
    assert "leverage" in str(e.value)
    with pytest.raises(P.CpdError) as e:
        P.cpd_workspace_size(P.make_problem([40, 33, 29], 70, 60),
                             P.make_options(sampler="euclidean", path="persistent"))
    assert "R <= 64" in str(e.value)
    with pytest.raises(P.CpdError):
        P.cpd_workspace_size(P.make_problem([40, 33, 29], 129, 60), o)
