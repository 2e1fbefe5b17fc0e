"""The C-ABI library loads on a CPU-only host and exports every function that
include/bp.h declares; host-side argument checks fail cleanly without a GPU."""
import ctypes as C
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "bp.h")
LIB = os.path.join(ROOT, "paper_2510_20499_amd", "libbp.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b(bp_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("bp_load", "bp_propagate", "bp_propagate_batch", "bp_probe", "bp_free",
              "bp_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "run __graft_entry__.build() first"
    lib = C.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_side_errors_without_gpu():
    lib = C.CDLL(LIB)
    lib.bp_load.restype = C.c_int
    lib.bp_last_error.restype = C.c_char_p
    out = C.c_void_p()
    # null CSR: rejected before any device call
    rc = lib.bp_load(None, None, None, None, None, None, None, C.byref(out))
    assert rc == -1
    assert b"null" in lib.bp_last_error()
    lib.bp_propagate.restype = C.c_int
    assert lib.bp_propagate(None, None, None, None, C.c_int64(0), None, None) == -1


def test_binding_exports_match_header():
    from paper_2510_20499_amd import bp
    assert sorted(bp.EXPORTS) == declared_functions()


def test_failure_hook_and_server_queue_calls_check_arguments_without_gpu():
    from paper_2510_20499_amd import bp
    lib = bp.lib()
    assert lib.bp_debug_fail_alloc(-1) == bp.BP_EINVAL
    assert lib.bp_debug_fail_alloc(0) == bp.BP_OK
    assert lib.bp_server_cancel(None, 1) == bp.BP_EINVAL
    n = C.c_int32(7)
    assert lib.bp_server_expire(None, 1.0, C.byref(n)) == bp.BP_EINVAL
    assert n.value == 7  # untouched on error
