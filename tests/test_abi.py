"""The C-ABI library: it loads on a machine without a GPU, exports every
function the public headers declare, the Python binding covers exactly that
set, and the product path refuses to run when the library is missing."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
DECL = re.compile(r"^\s*(?:tt_status|int32_t|const\s+char\s*\*)\s*\**\s*(tt_[a-z0-9_]+)\s*\(", re.M)


def declared(header_glob="include/*.h"):
    names = set()
    for h in glob.glob(os.path.join(ROOT, header_glob)):
        with open(h) as f:
            names |= set(DECL.findall(f.read()))
    return names


def test_headers_declare_the_api():
    names = declared()
    for n in ("tt_channel_create", "tt_channel_set_taps", "tt_channel_apply_dl", "tt_channel_apply_ul",
              "tt_channel_apply_slot", "tt_server_create", "tt_server_run", "tt_serve", "tt_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    from paper_2601_08217_amd import binding as B
    if not os.path.exists(B.LIB_PATH):
        pytest.skip("library not built (python -m paper_2601_08217_amd.build)")
    lib = ctypes.CDLL(B.LIB_PATH)
    missing = [n for n in sorted(declared()) if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_the_channel_header():
    from paper_2601_08217_amd import binding as B
    assert set(B.EXPORTED) == declared()


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2601_08217_amd import binding as B
    monkeypatch.setattr(B, "LIB_PATH", str(tmp_path / "absent.so"))
    monkeypatch.setattr(B, "_lib", None)
    with pytest.raises(ImportError, match="no CPU fallback"):
        B.load()
