"""The C-ABI library loads without a GPU and exports every entry point that
include/lob.h declares; the binding fails loudly when the library is absent."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lob.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lob_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2308_13289_amd import build
    if not os.path.exists(build.LIB):
        build.build()
    return build.LIB


def test_header_declares_the_boundary():
    names = declared()
    for n in ("lob_create", "lob_destroy", "lob_process_messages", "lob_step", "lob_read_l2",
              "lob_read_trades"):
        assert n in names


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_declares_every_export(libpath):
    from paper_2308_13289_amd import lob, serve
    assert sorted(lob.EXPORTS + serve.EXPORTS) == declared()
    lob.load(libpath)


def test_missing_library_fails_loudly(tmp_path):
    from paper_2308_13289_amd import lob
    with pytest.raises(lob.LobError):
        lob.load(str(tmp_path / "absent.so"))


def test_create_rejects_bad_config_without_gpu_work(libpath):
    """Argument checks happen before any device call: a NULL config or out-of-range
    values return LOB_EINVAL."""
    from paper_2308_13289_amd import lob
    L = lob.load(libpath)
    h = ctypes.c_void_p()
    assert L.lob_create(None, ctypes.byref(h)) == lob.EINVAL
    cfg = lob.Config()
    cfg.n_books = 0
    assert L.lob_create(ctypes.byref(cfg), ctypes.byref(h)) == lob.EINVAL
    assert b"n_books" in L.lob_last_error(None)
    assert L.lob_process_messages(None, None, 0, None, None, 0, None, None) == lob.EINVAL
    assert L.lob_destroy(None) is None


def test_binding_constants_match_the_header():
    """Status codes, modes, flags and limits the binding spells out are the header's."""
    from paper_2308_13289_amd import lob
    text = open(HEADER).read()
    defs = {m.group(1): int(m.group(2)) for m in re.finditer(r"#define\s+(LOB_[A-Z0-9_]+)\s+\(?(-?\d+)\)?", text)}
    for name in ("OK", "EINVAL", "ENOMEM", "EDEVICE", "ECAP", "L2_NONE", "L2_PER_MESSAGE", "L2_FINAL",
                 "MAX_CAPACITY", "MAX_LEVELS", "BOOK_SIDE_FULL", "BOOK_TIME_ORDER", "BOOK_TRADE_FULL",
                 "BOOK_FILLS_FULL", "BOOK_BAD_LOAD", "NOALLOC_MAX_BOOKS"):
        assert getattr(lob, name) == defs["LOB_" + name], name
