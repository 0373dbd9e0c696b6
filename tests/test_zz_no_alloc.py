"""mw_forward_noalloc (the forward transform whose intermediates live in the
library's static device scratch) against mw_forward, called through the C ABI:
two calls in a row, the second with a smaller input, in FP64 and FP32C, and the
error returns for an unprepared band-limit and for a call too large for the
scratch."""
import ctypes

import numpy as np
import pytest

import mwsynth

pytestmark = pytest.mark.gpu

MW_ENOMEM = -2
NOALLOC_BYTES = 64 << 20   # MW_NOALLOC_BYTES in include/mw.h


@pytest.fixture(scope="module")
def tc():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def mw(tc):
    import paper_1110_6298_amd as m
    m.library()
    return m


def _maps(tc, specs, seed):
    out = []
    for k, (L, s, real) in enumerate(specs):
        g = mwsynth.grid_gaussian(L, seed + k, real=bool(real))
        out.append(tc.from_numpy(np.ascontiguousarray(g)).cuda())
    return out


def _abi(mw, tc, name, specs, maps, precision):
    """Raw C-ABI call of `name` (mw_forward or mw_forward_noalloc); returns the
    status and the coefficient outputs."""
    lib = mw.library()
    n = len(specs)
    outs = [tc.full((L * L,), complex("nan"), dtype=tc.complex128, device="cuda") for L, _, _ in specs]
    ptrs = []
    for x, y in zip(maps, outs):
        ptrs += [x.data_ptr(), y.data_ptr()]
    arr = lambda v: (ctypes.c_int32 * n)(*v)
    parr = (ctypes.c_void_p * (2 * n))(*[ctypes.c_void_p(p) for p in ptrs])
    rc = getattr(lib, name)(arr([L for L, _, _ in specs]), arr([s for _, s, _ in specs]),
                            arr([r for _, _, r in specs]), n, ctypes.cast(parr, ctypes.POINTER(ctypes.c_void_p)),
                            precision, ctypes.c_void_p(tc.cuda.current_stream().cuda_stream))
    return rc, outs


def _prepare(mw, specs, precision):
    mw.prepare([L for L, _, _ in specs], [s for _, s, _ in specs], [r for _, _, r in specs], precision)


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32c"])
def test_noalloc_matches_forward_two_calls(tc, mw, precision):
    """Two chunks then one smaller map: each output of the allocation-free call
    equals mw_forward's bit for bit (same kernels, same arithmetic), hence within
    the 1e-12 (FP64) and 1e-6 (FP32C) bounds of the parity tests."""
    calls = [
        [(256, 2, 0), (256, 2, 0), (128, 0, 1)],   # two chunks, 12.6 MB of slots
        [(64, -1, 0)],                             # smaller input, reusing the scratch
    ]
    for i, specs in enumerate(calls):
        print("noalloc call %d precision %d specs %s" % (i, precision, specs), flush=True)
        _prepare(mw, specs, precision)
        maps = _maps(tc, specs, seed=41000 + 10 * i)
        rc_ref, ref = _abi(mw, tc, "mw_forward", specs, maps, precision)
        assert rc_ref == 0, mw.library().mw_last_error().decode()
        tc.cuda.synchronize()
        rc, got = _abi(mw, tc, "mw_forward_noalloc", specs, maps, precision)
        assert rc == 0, mw.library().mw_last_error().decode()
        tc.cuda.synchronize()
        for b, (r, g) in enumerate(zip(ref, got)):
            r, g = r.cpu().numpy(), g.cpu().numpy()
            assert np.isfinite(g).all(), "call %d map %d: unwritten output" % (i, b)
            err = float(np.abs(g - r).max() / max(np.abs(r).max(), 1e-300))
            assert err <= (1e-12 if precision == 0 else 1e-6), (i, b, err)
            assert np.array_equal(g, r), "call %d map %d differs from mw_forward (rel %.3e)" % (i, b, err)


def test_noalloc_rejects_unprepared_and_oversized(tc, mw):
    """A band-limit never prepared, and a call whose workspace exceeds
    MW_NOALLOC_BYTES, fail with MW_ENOMEM before anything is enqueued (the
    outputs stay untouched)."""
    lib = mw.library()
    specs = [(1237, 0, 1)]   # L = 1237 is prepared nowhere in the suite
    maps = _maps(tc, specs, seed=42000)
    rc, outs = _abi(mw, tc, "mw_forward_noalloc", specs, maps, 0)
    assert rc == MW_ENOMEM
    assert b"not prepared" in lib.mw_last_error()
    big = [(512, 2, 0)] * 3   # 3 x 25 MB of slots > 64 MiB
    _prepare(mw, big, 0)
    maps = _maps(tc, big, seed=42100)
    rc, outs = _abi(mw, tc, "mw_forward_noalloc", big, maps, 0)
    assert rc == MW_ENOMEM
    assert b"static scratch" in lib.mw_last_error()
    tc.cuda.synchronize()
    for y in outs:
        assert tc.isnan(y).all().item()
