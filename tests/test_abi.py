"""Host-side checks of the C ABI: the library loads, exports every declared symbol, and rejects
invalid arguments before any device work (these run without a GPU)."""

import ctypes
import os
import re

import numpy as np
import pytest

import paper_2007_14135_amd as nd
from paper_2007_14135_amd import _abi

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nssdoa.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nssdoa_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = nd.load()
    names = _declared_functions()
    assert "nssdoa_estimate" in names and len(names) >= 10
    for n in names:
        assert hasattr(lib, n), n


def test_status_strings():
    lib = nd.load()
    for s in range(6):
        assert lib.nssdoa_status_string(s)
    assert lib.nssdoa_status_string(99) == b"unknown status"


def _ula(M):
    p = np.zeros((M, 3))
    p[:, 0] = 0.5 * np.arange(M)
    return p


@pytest.mark.parametrize("arrays,grids,msg", [
    ([np.zeros((1, 3))], [(-90, 0.1, 1800)], "M=1"),
    ([np.zeros((65, 3))], [(-90, 0.1, 1800)], "M=65"),
    ([_ula(8)], [(-90, 0.1, 2)], "L=2"),
    ([_ula(8)], [(-90, 0.0, 1800)], "step=0"),
    ([_ula(8)], [(-90, -0.1, 1800)], "step<0"),
    ([_ula(8)], [(-90, float("nan"), 1800)], "step nan"),
    ([np.full((8, 3), np.inf)], [(-90, 0.1, 1800)], "non-finite positions"),
    ([_ula(8)], [(0, 1.0, 360, 1, 1.0, 0.0, 90)], "2-D polar step 0"),
    ([_ula(8)], [(0, 1.0, 360, 1, float("nan"), 1.0, 90)], "2-D polar start nan"),
    ([_ula(8)], [(0, 1.0, 360, 1, 1.0, 1.0, -1)], "n_polar < 0"),
    ([_ula(8)], [(0, 1.0, 360, 1, 1.0, 1.0, 4097)], "n_polar > 4096"),
    ([_ula(8)], [(0, 0.001, 360000, 1, 1.0, 0.01, 4096)], "2-D grid beyond 2^24 points"),
])
def test_plan_rejects_invalid(arrays, grids, msg):
    with pytest.raises(nd.NssdoaError) as e:
        nd.Plan(arrays, grids)
    assert e.value.status == _abi.EINVAL, msg


@pytest.mark.parametrize("kw", [dict(eig_tol=0.0), dict(eig_max_iter=0), dict(eig_method=3), dict(c64_scan=3), dict(refine_halfwidth=0),
                                dict(refine_halfwidth=17), dict(lowq_tau=-1.0), dict(extra_candidates=17),
                                dict(scan_rows=16), dict(scan_rows=100), dict(scan_rows=32768)])
def test_plan_rejects_bad_options(kw):
    with pytest.raises(nd.NssdoaError) as e:
        nd.Plan([_ula(8)], [(-90, 0.1, 1800)], nd.Options(**kw))
    assert e.value.status == _abi.EINVAL


@pytest.mark.parametrize("frame,alg,prec,max_D,msg", [
    ((3, 0, 1024, 2, 0, 1024, 0), "music", "c64", 4, "unknown array"),
    ((0, 3, 1024, 2, 0, 1024, 0), "music", "c64", 4, "unknown grid"),
    ((0, 0, 0, 2, 0, 1024, 0), "music", "c64", 4, "N=0"),
    ((0, 0, 1024, 0, 0, 1024, 0), "music", "c64", 4, "D=0"),
    ((0, 0, 1024, 8, 0, 1024, 0), "music", "c64", 8, "D=M"),
    ((0, 0, 1024, 5, 0, 1024, 0), "music", "c64", 4, "D>max_D"),
    ((0, 0, 1024, 2, 0, 1000, 0), "music", "c64", 4, "ldx<N"),
    ((0, 0, 1024, 2, -1, 1024, 0), "music", "c64", 4, "negative x_off"),
    ((0, 0, 1024, 2, 0, 1024, -5), "music", "c64", 4, "negative spec_off"),
    ((0, 0, 1024, 2, 0, 1024, 0), "music", "c64", 65, "max_D>64"),
    ((2, 0, 1024, 2, 0, 1024, 0), "music", "c64", 4, "M=12 not allowed for the FP32 scan"),
])
def test_batch_rejects_invalid(frame, alg, prec, max_D, msg):
    plan = nd.Plan([_ula(8), _ula(16), _ula(12)], [(-90, 0.1, 1800)])
    with pytest.raises(nd.NssdoaError) as e:
        nd.Batch(plan, alg, prec, [frame], max_D)
    assert e.value.status == _abi.EINVAL, msg


@pytest.mark.parametrize("prec", ["c64", "bf16", "f16"])
def test_matrix_core_scans_need_supported_M(prec):
    plan = nd.Plan([_ula(12)], [(-90, 0.1, 1800)])
    with pytest.raises(nd.NssdoaError) as e:
        nd.Batch(plan, "music", prec, [(0, 0, 1024, 2, 0, 1024, 0)], 4)
    assert e.value.status == _abi.EINVAL


def test_null_handles_rejected():
    lib = nd.load()
    n = ctypes.c_size_t()
    assert lib.nssdoa_workspace_size(None, ctypes.byref(n)) == _abi.EINVAL
    assert lib.nssdoa_estimate(None, None, 0, None, 0, None, None, None, None, 0, None) == _abi.EINVAL
    assert lib.nssdoa_estimate_noalloc(None, None, 0, None, 0, None, None, None, None) == _abi.EINVAL
    assert lib.nssdoa_noalloc_workspace_limit(None) == _abi.EINVAL
    assert lib.nssdoa_noalloc_workspace_limit(ctypes.byref(n)) == _abi.OK and n.value == 64 << 20
    assert lib.nssdoa_plan_destroy(None) == _abi.OK
    assert lib.nssdoa_batch_destroy(None) == _abi.OK
    assert lib.nssdoa_plan_create(None, None, 0, None, 0, None) == _abi.EINVAL


def test_plan_accepts_scan_rows():
    nd.Plan([_ula(8)], [(-90, 0.1, 1800)], nd.Options(scan_rows=1024)).close()


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_2d_grids_need_c64_or_c128(prec):
    # azimuth x polar-angle grids run on the FP32-accuracy and FP64 scans only
    plan = nd.Plan([_ula(8)], [(0, 1.0, 360, 1, 61.0, 1.0, 30)])
    with pytest.raises(nd.NssdoaError) as e:
        nd.Batch(plan, "music", prec, [(0, 0, 1024, 2, 0, 1024, 0)], 4)
    assert e.value.status == _abi.EUNSUPPORTED


def test_2d_grid_struct_layout():
    # the C struct: start, step, L, circular, polar start, polar step, n_polar, reserved
    assert ctypes.sizeof(_abi.Grid) == 48 and _abi.Grid.n_polar.offset == 40
    assert _abi.PEAK_DTYPE.itemsize == 32 and _abi.PEAK_DTYPE.fields["polar_deg"][1] == 24
    nd.Plan([_ula(8)], [(0, 1.0, 360, 1, 1.0, 1.0, 90), (-90, 0.1, 1800)]).close()
