"""The C-ABI library loads and exports every entry point its header declares (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xm.h")
LIB = os.path.join(ROOT, "paper_2502_04640_amd", "libxm.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(xm_[A-Za-z_0-9]+)\s*\(", text)))


def test_header_declares_the_four_calls():
    names = declared_functions()
    for n in ("xm_build_Q", "xm_bm_solve", "xm_round", "xm_certify"):
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libxm.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libxm.so not built")
def test_last_error_empty_and_default_opts():
    lib = ctypes.CDLL(LIB)
    lib.xm_last_error.restype = ctypes.c_char_p
    assert lib.xm_last_error() == b""
    from paper_2502_04640_amd.api import _SolveOpts
    o = _SolveOpts()
    lib.xm_default_opts(ctypes.byref(o))
    assert (o.r0, o.r_max, o.compute, o.lift) == (5, 7, 0, 1.0)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libxm.so not built")
def test_null_arguments_are_rejected_without_gpu():
    # argument checks run before any HIP call
    lib = ctypes.CDLL(LIB)
    lib.xm_build_Q.restype = ctypes.c_int
    lib.xm_last_error.restype = ctypes.c_char_p
    out = ctypes.c_void_p(0)
    code = lib.xm_build_Q(ctypes.c_int32(1), ctypes.c_int32(1), ctypes.c_int64(1), None, None, None, 0, None, 0,
                          ctypes.c_uint32(0), None, ctypes.byref(out))
    assert code == -1 and b"N must be" in lib.xm_last_error()
    lib.xm_get_info.restype = ctypes.c_int
    assert lib.xm_get_info(None, None) == -1


@pytest.mark.skipif(not os.path.exists(LIB), reason="libxm.so not built")
def test_product_kind_calls_reject_bad_arguments_without_gpu():
    # argument checks of the product-kernel selectors run before any HIP call
    lib = ctypes.CDLL(LIB)
    lib.xm_last_error.restype = ctypes.c_char_p
    for fn in (lib.xm_set_spmm_kind, lib.xm_set_product_kind, lib.xm_get_product_kind, lib.xm_spmm_timing,
               lib.xm_spmm_stats):
        fn.restype = ctypes.c_int
    assert lib.xm_set_spmm_kind(None, 0, 1) == -1
    assert lib.xm_set_product_kind(None, 0, 0, 1) == -1
    k = ctypes.c_int(-7)
    assert lib.xm_get_product_kind(None, 1, 0, ctypes.byref(k)) == -1
    assert k.value == -7  # output untouched on failure
    assert lib.xm_spmm_timing(None, 1) == -1
    assert lib.xm_spmm_stats(None, None, 0) == -1
    assert lib.xm_last_error() != b""


def test_stats_struct_matches_header():
    # the ctypes mirror of xm_spmm_counters has as many slots as the header declares
    text = open(HEADER).read()
    slots = int(re.search(r"#define XM_STATS_SLOTS (\d+)", text).group(1))
    from paper_2502_04640_amd.api import _SpmmStats
    assert len(_SpmmStats().launches) == slots == len(_SpmmStats().total_ms) == len(_SpmmStats().bytes_per_launch)


def _struct_fields(name):
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    body = re.search(r"typedef struct \{([^}]*)\}\s*" + name + r"\s*;", text).group(1)
    fields = []
    for decl in body.split(";"):
        decl = decl.strip()
        if not decl:
            continue
        typ, names = decl.split(None, 1)
        fields += [(n.strip(), typ) for n in names.split(",")]
    return fields


@pytest.mark.parametrize("cname,pyname", [("xm_cert", "_Cert"), ("xm_solve_info", "_SolveInfo"),
                                          ("xm_solve_opts", "_SolveOpts"), ("xm_adjoint_info", "_AdjInfo")])
def test_ctypes_structs_match_header(cname, pyname):
    # field names, order and C types of the ctypes mirrors follow the header
    from paper_2502_04640_amd import api
    cmap = {"double": ctypes.c_double, "int32_t": ctypes.c_int32, "xm_dtype": ctypes.c_int32}
    fields = _struct_fields(cname)
    mirror = getattr(api, pyname)._fields_
    assert [n for n, _ in fields] == [n for n, _ in mirror]
    for (n, t), (_, pt) in zip(fields, mirror):
        assert ctypes.sizeof(cmap[t]) == ctypes.sizeof(pt), (n, t, pt)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libxm.so not built")
def test_memory_pool_calls_without_gpu():
    # the pool's accounting needs no device: nothing is live or cached before any call
    lib = ctypes.CDLL(LIB)
    lib.xm_memory_info.restype = ctypes.c_int
    live, cached = ctypes.c_int64(-1), ctypes.c_int64(-1)
    assert lib.xm_memory_info(ctypes.byref(live), ctypes.byref(cached)) == 0
    assert live.value == 0 and cached.value == 0
    assert lib.xm_memory_info(None, None) == -1


def test_noalloc_scratch_size_matches_header():
    import re as _re
    text = open(HEADER).read()
    mib = int(_re.search(r"#define XM_NOALLOC_SCRATCH_MIB (\d+)", text).group(1))
    from paper_2502_04640_amd import api
    assert api.XM_NOALLOC_SCRATCH_BYTES == mib << 20
