"""The C-ABI library loads and exports every entry point include/open.h declares; the
binding's signature table covers the same names.  No compute call is made here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "open.h")
LIB = os.path.join(ROOT, "paper_2508_07605_amd", "libopen.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(open_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared()
    for must in ["open_create", "open_destroy", "open_foldin", "open_fit", "open_predict", "open_mlp_foldin",
                 "open_mlp_train_step", "open_csr_to_csc", "open_objective", "open_residual"]:
        assert must in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libopen.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_covers_header():
    from paper_2508_07605_amd import native
    assert sorted(native.SIGNATURES) == declared()


@pytest.mark.skipif(not os.path.exists(LIB), reason="libopen.so not built")
def test_host_only_calls():
    from paper_2508_07605_amd import native
    L = native.lib()
    assert L.open_mlp_num_params(480, 32, 256) == 256 * 960 + 256 + 256 * 256 + 256 + 32 * 256 + 32
    # null context is rejected before any device work
    assert L.open_foldin(None, None, 0, 32, 0, None, None, None, 0.05, 1, None, None) == native.OPEN_E_INVALID
    assert L.open_last_error(None) == b"null context"
    assert L.open_perf_predict(None, None, 0, None, None, None, None, None, None, None, None,
                               None) == native.OPEN_E_INVALID
    assert L.open_phase_detect(None, None, 0, 0, 0, 60.0, 25, None) == native.OPEN_E_INVALID
