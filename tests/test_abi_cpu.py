"""CPU checks of the C-ABI library: it loads, exports every declared entry point,
and rejects bad arguments on the host before touching any device memory."""
import ctypes
import os
import re

import pytest

import paper_2312_07008_amd as dp
from paper_2312_07008_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    src = open(os.path.join(ROOT, "include", "dfpt2.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:int|const char\*)\s+(\w+)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("library not built")
    return dp.load()


def test_exports_every_declared_symbol(lib):
    names = _declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
        assert n in _lib.SIGNATURES, n


def test_stage_names_match_header():
    """The Python stage list follows the header's DFPT2_STAGE_* values, in order."""
    src = open(os.path.join(ROOT, "include", "dfpt2.h")).read()
    vals = {m.group(1).lower(): int(m.group(2)) for m in re.finditer(r"DFPT2_STAGE_(\w+)\s*=\s*(\d+)", src)}
    nstage = int(re.search(r"DFPT2_NSTAGE\s*=\s*(\d+)", src).group(1))
    assert sorted(vals.values()) == list(range(nstage))
    assert [name for name, _ in sorted(vals.items(), key=lambda kv: kv[1])] == _lib.STAGES


def test_version_and_status_strings(lib):
    assert b"gfx950" in lib.dfpt2_version()
    assert lib.dfpt2_status_string(0) == b"ok"
    assert lib.dfpt2_status_string(-2) == b"workspace too small"


def test_workspace_sizes(lib):
    n1 = dp.workspace_size(dp.make_opts(10, 0, 60, 200, 0.5))
    n3 = dp.workspace_size(dp.make_opts(80, 0, 1200, 4000, 0.5))
    assert 0 < n1 < n3
    assert dp.fno_truncate_workspace_size(60) > 0
    assert dp.pt2_correction_workspace_size(dp.make_opts(10, 0, 60, 200, 0.5), 40) > 0
    # the split-BF16 density keeps BF16 slices of four matrices per pair of a batch
    b_fp64_d = dp.workspace_size(dp.make_opts(80, 0, 1200, 4000, 0.5, precision=1, slices_gemm2=1))
    b_bf16_d = dp.workspace_size(dp.make_opts(80, 0, 1200, 4000, 0.5, precision=1))
    assert b_bf16_d - b_fp64_d >= 4 * 4 * 2 * 512 * 1216 * 1216
    # INT8 digits: 5 bytes per element of B instead of 8 for four BF16 slices
    b_i8 = dp.workspace_size(dp.make_opts(80, 0, 1200, 4000, 0.5, precision=3))
    assert b_bf16_d - b_i8 >= 3 * 80 * 1216 * 4000 - 80 * 1216 * 4
    # the exactness limit of the INT8 level sums: n_aux_pad * 5 * 2^14 < 2^31
    assert dp.workspace_size(dp.make_opts(10, 0, 60, 26208, 0.5, precision=3)) > 0
    assert dp.workspace_size(dp.make_opts(10, 0, 60, 20000, 0.5, precision=3, slices_gemm1=4)) > 0


@pytest.mark.parametrize("bad", [dict(s=0.0), dict(s=-1.0), dict(s=float("nan")), dict(n_vir=0),
                                 dict(n_aux=0), dict(n_core=0, n_act=0), dict(n_core=-1),
                                 dict(precision=7), dict(density_convention=3), dict(slices_gemm1=9),
                                 dict(pair_batch=-5), dict(slices_gemm2=3), dict(precision=1, slices_gemm2=5),
                                 dict(precision=1, slices_gemm1=5), dict(precision=2, slices_gemm2=2),
                                 dict(precision=3, slices_gemm1=2), dict(precision=3, slices_gemm1=6),
                                 dict(precision=3, slices_gemm2=6), dict(precision=3, n_aux=26209)])
def test_invalid_options_rejected(lib, bad):
    kw = dict(n_core=10, n_act=0, n_vir=60, n_aux=200, s=0.5)
    kw.update({k: v for k, v in bad.items() if k in kw})
    extra = {k: v for k, v in bad.items() if k not in kw}
    o = dp.make_opts(kw["n_core"], kw["n_act"], kw["n_vir"], kw["n_aux"], kw["s"], **extra)
    n = ctypes.c_size_t(0)
    st = lib.dfpt2_workspace_size(ctypes.byref(o), ctypes.byref(n))
    assert st == _lib.ERR_INVALID_ARG
    assert lib.dfpt2_last_error()


def test_null_pointers_rejected_before_launch(lib):
    o = dp.make_opts(10, 0, 60, 200, 0.5)
    st = lib.dfpt2_build_vv_density(ctypes.byref(o), None, None, None, None, None, None, None, None,
                                    None, None, 0, None)
    assert st == _lib.ERR_INVALID_ARG
    kept = ctypes.c_int64(0)
    st = lib.fno_truncate(None, 60, 0.985, 0.0, None, None, ctypes.byref(kept), None, None, 0, None)
    assert st == _lib.ERR_INVALID_ARG


def test_workspace_too_small_rejected(lib):
    o = dp.make_opts(10, 0, 60, 200, 0.5)
    fake = ctypes.c_void_p(16)  # never dereferenced: the size check fails first
    st = lib.dfpt2_build_vv_density(ctypes.byref(o), fake, fake, None, fake, None, fake, fake, None, None,
                                    fake, 10, None)
    assert st == _lib.ERR_WORKSPACE


def test_bad_threshold_rejected(lib):
    fake = ctypes.c_void_p(16)
    kept = ctypes.c_int64(0)
    for p_o in (0.0, -0.1, 1.5, float("nan")):
        st = lib.fno_truncate(fake, 60, p_o, 0.0, fake, fake, ctypes.byref(kept), None, fake, 1 << 30, None)
        assert st == _lib.ERR_INVALID_ARG
    st = lib.fno_truncate(fake, 60, 0.98, -1.0, fake, fake, ctypes.byref(kept), None, fake, 1 << 30, None)
    assert st == _lib.ERR_INVALID_ARG


def test_correction_rejects_bad_kept_count(lib):
    o = dp.make_opts(10, 0, 60, 200, 0.5)
    n = ctypes.c_size_t(0)
    assert lib.pt2_correction_workspace_size(ctypes.byref(o), 0, ctypes.byref(n)) == _lib.ERR_INVALID_ARG
    assert lib.pt2_correction_workspace_size(ctypes.byref(o), 61, ctypes.byref(n)) == _lib.ERR_INVALID_ARG


@pytest.mark.parametrize("rule,param", [(7, 0.5), (1, 0.0), (1, 1.5), (0, 0.0), (3, 2.5), (3, 0.0), (3, 61.0),
                                        (2, float("nan"))])
def test_truncation_rule_arguments_rejected(lib, rule, param):
    kept = ctypes.c_int64(0)
    buf = ctypes.create_string_buffer(64)
    st = lib.fno_truncate_rule(buf, 60, rule, param, 0.0, buf, buf, ctypes.byref(kept), None, buf, 1 << 30, None)
    assert st == _lib.ERR_INVALID_ARG
    assert lib.dfpt2_last_error()


def test_naf_arguments_rejected(lib):
    n = ctypes.c_size_t(0)
    assert lib.naf_compress_workspace_size(ctypes.byref(dp.make_opts(2, 0, 10, 20000, 0.5)),
                                           ctypes.byref(n)) == _lib.ERR_INVALID_ARG
    o = dp.make_opts(2, 0, 10, 20, 0.5)
    assert lib.naf_compress_workspace_size(ctypes.byref(o), ctypes.byref(n)) == _lib.OK and n.value > 0
    k = ctypes.c_int64(0)
    buf = ctypes.create_string_buffer(64)
    assert lib.naf_compress(ctypes.byref(o), buf, float("nan"), buf, buf, ctypes.byref(k), buf, n.value,
                            None) == _lib.ERR_INVALID_ARG
    assert lib.naf_compress(ctypes.byref(o), None, 0.0, buf, buf, ctypes.byref(k), buf, n.value,
                            None) == _lib.ERR_INVALID_ARG
    assert lib.naf_compress(ctypes.byref(o), buf, 0.0, buf, buf, ctypes.byref(k), buf, 0,
                            None) == _lib.ERR_WORKSPACE


def test_ladder_arguments_rejected(lib):
    n = ctypes.c_size_t(0)
    assert lib.pp_ladder_workspace_size(0, 10, 2, 0, ctypes.byref(n)) == _lib.ERR_INVALID_ARG
    assert lib.pp_ladder_workspace_size(10, 10, 0, 0, ctypes.byref(n)) == _lib.ERR_INVALID_ARG
    assert lib.pp_ladder_workspace_size(10, 10, 2, 11, ctypes.byref(n)) == _lib.ERR_INVALID_ARG
    assert lib.pp_ladder_workspace_size(4096, 10, 2, 0, ctypes.byref(n)) == _lib.ERR_INVALID_ARG
    assert lib.pp_ladder_workspace_size(10, 10, 2, 0, ctypes.byref(n)) == 0 and n.value > 0
    full = n.value
    assert lib.pp_ladder_workspace_size(10, 10, 2, 6, ctypes.byref(n)) == 0 and n.value > 0
    assert full > 0
    # without X, n_kept other than 0 or n_vir is refused before any device access
    fake = ctypes.c_void_p(0x1000)
    st = lib.pp_ladder(10, 10, 2, fake, fake, None, 0, 5, fake, fake, ctypes.c_size_t(1 << 30), None)
    assert st == _lib.ERR_INVALID_ARG
    st = lib.pp_ladder(10, 10, 2, None, fake, None, 0, 0, fake, fake, ctypes.c_size_t(1 << 30), None)
    assert st == _lib.ERR_INVALID_ARG
    st = lib.pp_ladder(10, 10, 2, fake, fake, None, 0, 0, fake, fake, ctypes.c_size_t(16), None)
    assert st == _lib.ERR_WORKSPACE
    # X with a leading dimension below n_kept
    st = lib.pp_ladder(10, 10, 2, fake, fake, fake, 4, 6, fake, fake, ctypes.c_size_t(1 << 30), None)
    assert st == _lib.ERR_INVALID_ARG


def test_active_particle_arguments_rejected(lib):
    o = dp.make_opts(4, 2, 30, 20, 0.5)
    n = ctypes.c_size_t(0)
    assert lib.dfpt2_active_particle_workspace_size(ctypes.byref(o), ctypes.byref(n)) == 0 and n.value > 0
    fake = ctypes.c_void_p(0x1000)
    st = lib.dfpt2_add_active_particle_density(ctypes.byref(o), fake, fake, fake, fake, None, fake, fake,
                                               ctypes.c_size_t(n.value), None)
    assert st == _lib.ERR_INVALID_ARG
    st = lib.dfpt2_add_active_particle_density(ctypes.byref(o), fake, fake, fake, fake, fake, fake, fake,
                                               ctypes.c_size_t(16), None)
    assert st == _lib.ERR_WORKSPACE
    bad = dp.make_opts(4, 2, 30, 20, -1.0)
    assert lib.dfpt2_active_particle_workspace_size(ctypes.byref(bad), ctypes.byref(n)) == _lib.ERR_INVALID_ARG
