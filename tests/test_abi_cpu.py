"""CPU-side checks of the C-ABI boundary: the library loads and exports
every function include/mpcare.h declares; the binding's table matches the
header; option defaults follow the values of Sec. 5.  No GPU work."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mpcare.h")
LIB = os.path.join(ROOT, "paper_2607_14742_amd", "libmpcare.so")


def header_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:care_status|void|const char\s*\*)\s+(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libmpcare.so not built")


def test_header_declares_the_four_solver_entry_points():
    names = header_functions()
    for f in ("care_solve", "lyap_lradi", "care_residual_factor", "lowrank_truncate"):
        assert f in names


@needs_lib
def test_library_exports_every_declared_symbol():
    lib = C.CDLL(LIB)
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2607_14742_amd._lib import SIGNATURES
    assert sorted(SIGNATURES) == header_functions()


def test_struct_layouts_match_header_order():
    from paper_2607_14742_amd._lib import care_opts, care_stats
    src = open(HEADER).read()
    body = src[src.index("typedef struct {\n  int32_t inner_prec;"):src.index("} care_opts;")]
    fields = re.findall(r"(?:int32_t|int64_t|double|const double\*)\s+([\w, ]+);", body)
    flat = [f.strip() for grp in fields for f in grp.split(",")]
    assert flat == [f for f, _ in care_opts._fields_]
    body = src[src.index("typedef struct {\n  int32_t iter0_outer"):src.index("} care_stats;")]
    fields = re.findall(r"(?:int32_t|int64_t|double)\s+([\w, \[\]0-9]+);", body)
    flat = [re.sub(r"\[\d+\]", "", f.strip()) for grp in fields for f in grp.split(",")]
    assert flat == [f for f, _ in care_stats._fields_]


@needs_lib
def test_struct_sizes_match_the_compiled_library():
    from paper_2607_14742_amd import _lib as L
    lib = L.load()
    sizes = (C.c_int64 * 6)()
    assert lib.care_struct_sizes(sizes, 6) == L.CARE_OK
    mine = [C.sizeof(t) for t in (L.care_csr, L.care_shift, L.care_opts, L.care_stats, L.care_instance,
                                  L.care_instance_result)]
    assert list(sizes) == mine
    assert lib.care_struct_sizes(sizes, 7) == L.CARE_ERR_ARG


@needs_lib
def test_opts_defaults_follow_the_paper():
    from paper_2607_14742_amd import _lib as L
    lib = L.load()
    o = L.care_opts()
    lib.care_opts_default(C.byref(o), L.CARE_FP32)
    assert o.inner_prec == L.CARE_FP32
    assert o.k_max == 20 and o.j_max == 50
    assert o.eta_r_rel == 1e-4
    assert abs(o.eta_s_rel - 10 * 2.0 ** -53) < 1e-30
    assert o.stagnation == 0.999
    assert o.tau_L0 == 0.0 and o.refine_forcing == 0.25
    # library choices outside the paper: panel autotuner and column compaction
    # on, BiCGStab inner solves, one shift set for the whole solve
    assert o.spmm_tune == 1 and o.krylov_compact == 1 and o.adi_rotate == 1 and o.krylov_block_tol == -1
    assert o.krylov_method == 0 and o.shift_update == 0


@needs_lib
def test_null_context_is_an_argument_error():
    from paper_2607_14742_amd import _lib as L
    lib = L.load()
    r = C.c_int32(0)
    st = lib.care_solve(None, None, None, 0, None, 0, 1e-10, None, 0, None, None, 0, 0, C.byref(r), None)
    assert st == L.CARE_ERR_ARG
    assert b"context" in lib.care_last_error()
