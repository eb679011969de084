"""Host-only checks of the C ABI (no GPU): exported symbols and descriptor validation."""

import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cs.h")

cs = pytest.importorskip("paper_2604_08463_amd")
from paper_2604_08463_amd import _lib  # noqa: E402


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cs_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libcs.so not built (run __graft_entry__.build())")
    return _lib.load()


def test_library_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 19
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(line.split()[-1] for line in out.splitlines() if line.strip())
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    assert sorted(_lib.EXPORTS) == names


def test_library_is_built_for_gfx950(lib):
    out = subprocess.run(["strings", _lib.LIB_PATH], capture_output=True, text=True).stdout
    assert "gfx950" in out


def _desc(F=15, P=100, B=2, **over):
    freqs = np.linspace(40.0, 400.0, F)
    ninv = np.ones(2 * F)
    ncl = np.tile(np.array([3, 2, 2], dtype=np.int32), (B, 1))
    d = _lib.Desc()
    d.nfreq, d.npix, d.nitems = F, P, B
    d.freqs_ghz = freqs.ctypes.data_as(C.POINTER(C.c_double))
    d.nu0_dust_ghz, d.nu0_sync_ghz, d.tcmb_k = 353.0, 23.0, 2.7255
    d.precision, d.d_dtype = 0, 0
    d.d = C.c_void_p(0x1000)  # never dereferenced by cs_problem_create
    d.d_item_stride = 2 * F * P
    d.ninv_mode = 0
    d.ninv_band = ninv.ctypes.data_as(C.POINTER(C.c_double))
    d.labels = C.c_void_p(0x2000)
    d.labels_item_stride = 0
    d.nclusters = ncl.ctypes.data_as(C.POINTER(C.c_int32))
    for k, v in over.items():
        setattr(d, k, v)
    return d, (freqs, ninv, ncl)


def _create(lib, d):
    h = C.c_void_p()
    rc = lib.cs_problem_create(C.byref(d), C.byref(h))
    return rc, h


def test_create_valid_and_workspace_size(lib):
    d, keep = _desc()
    rc, h = _create(lib, d)
    assert rc == 0
    off = np.zeros(3, dtype=np.int64)
    assert lib.cs_problem_param_offsets(h, off.ctypes.data_as(C.POINTER(C.c_int64))) == 0
    assert off.tolist() == [0, 7, 14]
    nb = C.c_size_t()
    assert lib.cs_problem_workspace_bytes(h, C.byref(nb)) == 0
    assert nb.value > 2 * 2 * 15 * 128 * 8  # holds at least the packed FP64 data
    # evaluation before prepare is a state error, reported without touching the device
    f = C.c_void_p(0x3000)
    assert lib.cs_likelihood(h, f, f, None, None) == _lib.CS_E_STATE
    lib.cs_problem_destroy(h)


@pytest.mark.parametrize("field,value,code", [
    ("nfreq", 0, _lib.CS_E_INVALID),
    ("nfreq", 33, _lib.CS_E_UNSUPPORTED),
    ("npix", 0, _lib.CS_E_INVALID),
    ("nitems", 0, _lib.CS_E_INVALID),
    ("tcmb_k", 0.0, _lib.CS_E_INVALID),
    ("precision", 7, _lib.CS_E_INVALID),
    ("d_item_stride", 5, _lib.CS_E_INVALID),
    ("labels_item_stride", 7, _lib.CS_E_INVALID),
    ("ninv_mode", 4, _lib.CS_E_INVALID),
    ("d", None, _lib.CS_E_INVALID),
])
def test_create_rejects_bad_descriptors(lib, field, value, code):
    d, keep = _desc(**{field: value})
    rc, h = _create(lib, d)
    assert rc == code
    assert not h.value
    assert len(lib.cs_last_error()) > 0


def test_create_rejects_bad_weights_and_counts(lib):
    d, (freqs, ninv, ncl) = _desc()
    ninv[3] = 0.0
    assert _create(lib, d)[0] == _lib.CS_E_INVALID
    d, (freqs, ninv, ncl) = _desc()
    ncl[1, 0] = 4  # shared labels need equal counts
    assert _create(lib, d)[0] == _lib.CS_E_INVALID
    d, (freqs, ninv, ncl) = _desc()
    ncl[0, 2] = 0
    assert _create(lib, d)[0] == _lib.CS_E_INVALID


def test_sort_key_width_limit(lib):
    d, (freqs, ninv, ncl) = _desc(P=1 << 20, B=1)
    ncl[:] = (1 << 20, 1 << 20, 1 << 20)  # 4 x 20 bits > 63
    assert _create(lib, d)[0] == _lib.CS_E_UNSUPPORTED


def test_status_strings(lib):
    for s in range(7):
        assert lib.cs_status_str(s)


def test_optimizer_options_validation(lib):
    o = _lib.OptimOpts()
    assert lib.cs_optim_default_opts(C.byref(o)) == 0
    assert (o.m, o.max_iter, o.iters_per_graph, o.max_backtracks, o.fp64_polish) == (10, 1000, 8, 30, 1)
    assert o.gtol_rel == 1e-8 and o.c1 == 1e-4
    assert o.solver == _lib.SOLVER_LBFGS
    assert (o.lr, o.beta1, o.beta2, o.eps, o.topk) == (0.01, 0.9, 0.999, 1e-16, 0.0)


def test_schedule_validation(lib):
    d, keep = _desc()
    rc, h = _create(lib, d)
    s = _lib.Schedule(3, 0, 1)
    assert lib.cs_problem_set_schedule(h, C.byref(s)) == _lib.CS_E_INVALID
    s = _lib.Schedule(8, 4, 0, 3)  # staging modes are 0, 1 and 2
    assert lib.cs_problem_set_schedule(h, C.byref(s)) == _lib.CS_E_INVALID
    s = _lib.Schedule(8, 4, 0, 2)
    assert lib.cs_problem_set_schedule(h, C.byref(s)) == 0
    s = _lib.Schedule(8, 4, 0)
    assert lib.cs_problem_set_schedule(h, C.byref(s)) == 0
    g = _lib.Schedule()
    assert lib.cs_problem_get_schedule(h, C.byref(g)) == 0
    assert (g.waves_per_block, g.blocks_per_cu, g.xcd_remap) == (8, 4, 0)
    lib.cs_problem_destroy(h)


def test_optimizer_switch_default(lib):
    o = _lib.OptimOpts()
    assert lib.cs_optim_default_opts(C.byref(o)) == 0
    assert o.switch_rel == 1e-4


@pytest.mark.parametrize("nitems,nranks", [(64, 8), (1024, 7), (5, 3), (3, 5), (0, 2), (1, 1)])
def test_item_range_is_contiguous_floor_chunking(lib, nitems, nranks):
    # worker k takes [floor(k N / P), floor((k+1) N / P)): the ranges tile [0, N) in order
    ends = []
    for k in range(nranks):
        b, e = C.c_int32(), C.c_int32()
        assert lib.cs_item_range(k, nranks, nitems, C.byref(b), C.byref(e)) == 0
        assert (b.value, e.value) == ((k * nitems) // nranks, ((k + 1) * nitems) // nranks)
        ends.append((b.value, e.value))
    assert ends[0][0] == 0 and ends[-1][1] == nitems
    assert all(ends[i][1] == ends[i + 1][0] for i in range(nranks - 1))
    b, e = C.c_int32(), C.c_int32()
    assert lib.cs_item_range(nranks, nranks, nitems, C.byref(b), C.byref(e)) == _lib.CS_E_INVALID


def test_descriptor_slice_offsets_item_arrays(lib):
    F, P, B = 15, 100, 6
    d, (freqs, ninv, ncl) = _desc(F=F, P=P, B=B)
    ncl[:] = np.arange(3 * B, dtype=np.int32).reshape(B, 3) + 1
    d.labels_item_stride = 3 * P
    d.d_dtype = 1  # FP32: 4-byte elements
    out = _lib.Desc()
    assert lib.cs_problem_desc_slice(C.byref(d), 2, 5, C.byref(out)) == 0
    assert out.nitems == 3 and out.nfreq == F and out.npix == P
    assert out.d == 0x1000 + 2 * (2 * F * P) * 4
    assert out.labels == 0x2000 + 2 * 3 * P * 4
    got = np.ctypeslib.as_array(out.nclusters, shape=(3, 3))
    assert np.array_equal(got, ncl[2:5])
    # shared arrays (stride 0) stay shared
    d.d_item_stride = 0
    assert lib.cs_problem_desc_slice(C.byref(d), 1, 2, C.byref(out)) == 0
    assert out.d == 0x1000
    for b, e in ((0, 0), (3, 2), (-1, 2), (4, 7)):
        assert lib.cs_problem_desc_slice(C.byref(d), b, e, C.byref(out)) == _lib.CS_E_INVALID
