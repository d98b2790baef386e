"""CPU-side checks of the C-ABI library: it builds' artefact loads and exports
every entry point include/nxs.h declares; calls that fail argument checks
before touching the GPU return NXS_EINVAL."""
import ctypes
import re
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
HEADER = ROOT / "include" / "nxs.h"
LIB = ROOT / "paper_2603_02887_amd" / "libnxs.so"


def declared_symbols():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nxs_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ("nxs_create", "nxs_destroy", "nxs_render_forward", "nxs_last_error"):
        assert s in syms


@pytest.fixture(scope="module")
def lib():
    if not LIB.exists():
        pytest.fail(f"{LIB} missing: run python -m paper_2603_02887_amd.build")
    return ctypes.CDLL(str(LIB))


def test_library_exports_every_declared_symbol(lib):
    missing = [s for s in declared_symbols() if not hasattr(lib, s)]
    assert not missing, missing


def test_binding_symbol_list_matches_header():
    from paper_2603_02887_amd import nxs
    assert sorted(nxs.SYMBOLS) == declared_symbols()


def test_null_context_is_rejected_without_gpu(lib):
    lib.nxs_render_forward.restype = ctypes.c_int
    lib.nxs_render_forward.argtypes = [ctypes.c_void_p] * 7
    assert lib.nxs_render_forward(None, None, None, 1, None, None, None) == -1
    lib.nxs_last_error.restype = ctypes.c_char_p
    lib.nxs_last_error.argtypes = [ctypes.c_void_p]
    assert lib.nxs_last_error(None) == b""
    lib.nxs_create.restype = ctypes.c_int
    lib.nxs_create.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p,
                               ctypes.c_void_p]
    assert lib.nxs_create(None, 0, None, None, None) == -1
    # an allocator needs both callbacks
    out = ctypes.c_void_p()
    assert lib.nxs_create(ctypes.byref(out), 0, ctypes.c_void_p(1), None, None) == -1
    assert not out.value


def test_state_and_status_entry_points_reject_null_context(lib):
    for name, nargs in (("nxs_render_backward", 6), ("nxs_state_release", 3),
                        ("nxs_forward_status", 2), ("nxs_autotune", 10),
                        ("nxs_inspect_counts", 3), ("nxs_release_workspace", 1)):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p] * nargs
        assert f(*([None] * nargs)) == -1, name


def test_pipeline_entry_points_check_arguments_without_gpu(lib):
    create = lib.nxs_pipeline_create
    create.restype = ctypes.c_int
    create.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int32, ctypes.c_void_p,
                       ctypes.c_void_p, ctypes.c_void_p]
    out = ctypes.c_void_p()
    assert create(None, 0, 3, None, None, None) == -1
    for lanes in (0, -1, 9):                 # lanes in 1..8
        assert create(ctypes.byref(out), 0, lanes, None, None, None) == -1
        assert not out.value
    # an allocator needs both callbacks
    assert create(ctypes.byref(out), 0, 2, ctypes.c_void_p(1), None, None) == -1
    assert not out.value
    for name, nargs in (("nxs_pipeline_destroy", 1), ("nxs_pipeline_render", 7),
                        ("nxs_pipeline_join", 2), ("nxs_pipeline_status", 2)):
        f = getattr(lib, name)
        f.restype = ctypes.c_int
        f.argtypes = [ctypes.c_void_p] * nargs
        assert f(*([None] * nargs)) == -1, name
    lib.nxs_pipeline_last_error.restype = ctypes.c_char_p
    lib.nxs_pipeline_last_error.argtypes = [ctypes.c_void_p]
    assert lib.nxs_pipeline_last_error(None) == b"null pipeline"
