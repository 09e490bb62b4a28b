"""Host-side checks of the C ABI: the library loads and exports every entry
point that include/gnk.h declares (no GPU work)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gnk.h")


def _declared():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^GNK_API\s+[\w\s\*]+?\b(gnk_\w+)\s*\(", src, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    from paper_1308_5351_amd import gnk
    if not os.path.exists(gnk.LIB_PATH):
        from paper_1308_5351_amd import build
        build.build()
    return gnk.load_library()


def test_header_declares_entry_points():
    names = _declared()
    for f in ("gnk_create", "gnk_destroy", "gnk_fbie", "gnk_fbie_ad", "gnk_apply", "gnk_cauchy_sum"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    for name in _declared():
        assert hasattr(lib, name), name


def test_binding_lists_match_header():
    from paper_1308_5351_amd import gnk
    assert sorted(gnk.EXPORTED) == _declared()


def test_version_string(lib):
    assert b"gnk" in lib.gnk_version()


def test_null_arguments_rejected(lib):
    # argument checks run before any device work
    assert lib.gnk_create(None, 0) == -1
    assert lib.gnk_destroy(None) == -1
    assert lib.gnk_set_stream(None, None) == -1
    assert lib.gnk_fbie(None, None, None, 1, None, None, None, None) == -1
