"""The C-ABI library loads and exports every symbol include/apcloud.h declares
(CPU only: no compute call is made without a GPU)."""
import ctypes as ct
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "apcloud.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(apc2?_[a-z_0-9]+)\s*\(", src)))


@pytest.fixture(scope="module")
def apc():
    from paper_1603_04039_amd import apcloud
    if not os.path.exists(apcloud.LIB_PATH):
        from paper_1603_04039_amd.build import build_library
        build_library()
    apcloud.load_library()
    return apcloud


def test_exports_every_declared_symbol(apc):
    lib = apc.load_library()
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(apc.EXPORTS) == names


def test_error_strings_and_defaults(apc):
    lib = apc.load_library()
    assert lib.apc_strerror(apc.APC_EDOMAIN).decode() == "particle outside the domain"
    assert lib.apc_strerror(12345).decode() == "unknown error"
    p = apc.make_params(order=2, c=0.04, max_depth=10)
    assert (p.order, p.ring_min, p.ring_max, p.m_cap, p.precision) == (2, 2, 5, 40, 0)
    assert p.max_depth == 10 and p.c == 0.04 and p.L == 1.0


def test_struct_layouts_match_header(apc):
    # apc_params: lo[3], L, order (+pad), c, max_depth, ring_min, ring_max, m_cap, poisson_c,
    # precision, stage_cap, criterion_pow, ring_lds, ring_first_cap (+pad), tau_dom,
    # periodic, kernel, mask_level (+pad), mask
    assert ct.sizeof(apc.Params) == 3 * 8 + 8 + 8 + 8 + 4 * 4 + 8 + 8 + 8 + 8 + 8 + 8 + 8 + 8
    assert apc.Params.criterion_pow.offset == 80 and apc.Params.ring_lds.offset == 84
    assert apc.Params.ring_first_cap.offset == 88 and apc.Params.tau_dom.offset == 96
    assert apc.Params.periodic.offset == 104 and apc.Params.kernel.offset == 108
    assert apc.Params.mask_level.offset == 112 and apc.Params.mask.offset == 120
    assert ct.sizeof(apc.Stats) == 4 * 4 + 8 + 8 + 8 + 8 + 4 + 4 + 8 + 8 + 8


def test_binding_fails_loudly_without_library(apc, tmp_path):
    with pytest.raises(ImportError):
        apc.load_library.__wrapped__(str(tmp_path / "missing.so")) \
            if hasattr(apc.load_library, "__wrapped__") else _load_missing(apc, tmp_path)


def _load_missing(apc, tmp_path):
    saved = apc._lib
    apc._lib = None
    try:
        apc.load_library(str(tmp_path / "missing.so"))
    finally:
        apc._lib = saved
