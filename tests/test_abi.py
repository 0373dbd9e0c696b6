"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/mw.h declares, and rejects invalid arguments before touching a device."""
import ctypes
import os
import re

import pytest

import paper_1110_6298_amd as mw

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "mw.h")


def declared_functions(header=HEADER):
    text = open(header).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(mw_\w+)\s*\(", text, re.M)))


def test_header_declares_the_abi():
    names = declared_functions()
    assert set(names) == set(mw.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = mw.library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    prof = declared_functions(HEADER.replace("mw.h", "mw_profile.h"))
    assert set(prof) == set(mw.PROFILE_EXPORTS)
    for name in prof:
        assert hasattr(lib, name), name


def test_version_and_status_strings():
    lib = mw.library()
    assert b"gfx950" in lib.mw_version()
    assert lib.mw_status_string(0) == b"success"
    assert lib.mw_status_string(-1) == b"invalid argument"


def _raw(name, Ls, spins, reals, batch=None, ptrs=True, prec=0):
    lib = mw.library()
    n = len(Ls) if batch is None else batch
    arr = lambda v: (ctypes.c_int32 * max(1, len(v)))(*v)
    p = (ctypes.c_void_p * (2 * max(1, len(Ls))))(*([ctypes.c_void_p(0x1000)] * (2 * max(1, len(Ls)))))
    pp = ctypes.cast(p, ctypes.POINTER(ctypes.c_void_p)) if ptrs else None
    return getattr(lib, name)(arr(Ls), arr(spins), arr(reals), n, pp, prec, None)


@pytest.mark.parametrize("name", ["mw_forward", "mw_forward_noalloc", "mw_inverse", "mw_forward_adjoint",
                                  "mw_forward_compact", "mw_inverse_compact", "mw_forward_adjoint_compact",
                                  "mw_inverse_adjoint_compact",
                                  "mw_inverse_adjoint"])
@pytest.mark.parametrize("Ls,spins,reals,batch,ptrs,prec", [
    ([0], [0], [0], None, True, 0),          # L < 1
    ([4097], [0], [0], None, True, 0),       # L > MW_LMAX = 4096
    ([8], [8], [0], None, True, 0),          # |s| >= L
    ([8], [-8], [0], None, True, 0),
    ([8], [2], [1], None, True, 0),          # reality needs s = 0
    ([8], [0], [2], None, True, 0),          # reality not in {0,1}
    ([8], [0], [0], 0, True, 0),             # batch < 1
    ([8], [0], [0], None, False, 0),         # NULL ptrs
    ([8], [0], [0], None, True, 7),          # unknown precision
])
def test_invalid_arguments_rejected(name, Ls, spins, reals, batch, ptrs, prec):
    assert _raw(name, Ls, spins, reals, batch, ptrs, prec) == -1
    assert mw.library().mw_last_error()


def test_null_device_pointer_rejected():
    lib = mw.library()
    arr = lambda v: (ctypes.c_int32 * len(v))(*v)
    p = (ctypes.c_void_p * 2)(ctypes.c_void_p(0x1000), None)
    rc = lib.mw_forward(arr([8]), arr([0]), arr([0]), 1, ctypes.cast(p, ctypes.POINTER(ctypes.c_void_p)), 0, None)
    assert rc == -1


def test_workspace_size_is_host_only():
    assert mw.workspace_size([64], [0]) >= 2 * 127 * 64 * 16
    # two chunks (different (L, spin)) run on two internal streams, each with a
    # workspace half sized for the largest map
    assert mw.workspace_size([64, 512], [0, 2]) == 2 * mw.workspace_size([512], [2])
    with pytest.raises(mw.MWError):
        mw.workspace_size([0], [0])


def test_tune_cache_parser(tmp_path):
    """The autotuner's cache file: valid lines are taken, malformed ones and other
    architectures or impossible values skipped (host only)."""
    p = tmp_path / "tune.txt"
    p.write_text("gfx950 300 0 12 2\n"
                 "gfx950 301 1 5 4\n"
                 "garbage line\n"
                 "gfx942 302 0 3 2\n"          # another architecture
                 "gfx950 303 0 3 3\n"          # G not a power of two
                 "gfx950 99999 0 3 2\n"        # L out of range
                 "gfx950 304 2 3 2\n"          # reality not 0/1
                 "gfx950 305 0 3 2 extra\n")   # trailing token
    assert mw.tune_cache_load(str(p)) == 2
    assert mw.tuned_group(300, 0, 12) == 2
    assert mw.tuned_group(301, 1, 5) == 4
    assert mw.tuned_group(302, 0, 3) == 0
    assert mw.tuned_group(303, 0, 3) == 0
    assert mw.tune_cache_load(str(tmp_path / "missing.txt")) == 0
