"""The C-ABI library loads, exports every symbol include/fr.h declares, and
rejects bad configurations before touching a device (runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fr.h")
LIB = os.path.join(ROOT, "paper_2402_13435_amd", "libfr.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fr_[a-z_]+)\s*\(", text)))


needs_lib = pytest.mark.skipif(not os.path.exists(LIB), reason="libfr.so not built")


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("fr_create", "fr_destroy", "fr_load_corpus", "fr_update_docs", "fr_search",
              "fr_last_error", "fr_debug_masks"):
        assert s in syms


@needs_lib
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for s in declared_symbols():
        assert hasattr(lib, s), s


@needs_lib
def test_binding_covers_every_symbol():
    from paper_2402_13435_amd import SYMBOLS
    assert set(declared_symbols()) == set(SYMBOLS)


@needs_lib
def test_bad_configs_rejected_without_a_device():
    from paper_2402_13435_amd import FrError, Index
    from paper_2402_13435_amd.binding import FR_EINVAL, FR_EUNSUPPORTED
    cases = [
        (dict(capacity=10, dim=0, vocab=16, k_max=10), FR_EUNSUPPORTED),
        (dict(capacity=10, dim=300, vocab=16, k_max=10), FR_EUNSUPPORTED),
        (dict(capacity=10, dim=8, vocab=0, k_max=10), FR_EINVAL),
        (dict(capacity=10, dim=8, vocab=16, k_max=0), FR_EINVAL),
        (dict(capacity=10, dim=8, vocab=16, k_max=5000), FR_EINVAL),
        (dict(capacity=0, dim=8, vocab=16, k_max=10), FR_EINVAL),
    ]
    for kw, status in cases:
        with pytest.raises(FrError) as e:
            Index(**kw)
        assert e.value.status == status, (kw, e.value)


@needs_lib
def test_null_handles_are_errors():
    from paper_2402_13435_amd import lib
    L = lib()
    assert L.fr_destroy(None) == 0
    assert L.fr_search(None, 0, None, None, None, None, None, None, None, None, 0) == -1
    assert L.fr_load_corpus(None, 0, None, None, None, None, 0) == -1
    assert b"null" in L.fr_last_error()
