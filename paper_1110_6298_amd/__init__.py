"""MI355X (gfx950) McEwen-Wiaux spin spherical-harmonic transforms.

Thin binding over the C ABI of ``libmw.so`` (declared in ``include/mw.h``).
This module only marshals arguments: every stage of every transform runs in
the library's HIP kernels.  Tensors are torch CUDA (ROCm) tensors used as
device memory; work is enqueued on the current torch stream.

    import paper_1110_6298_amd as mw
    flm = mw.forward(x, L=512, spin=2)          # x: (L, 2L-1) complex128 on cuda
    x2  = mw.inverse(flm, L=512, spin=2)        # flm: (L*L,) complex128 on cuda

If the library has not been built (``python -m paper_1110_6298_amd.build``) or
cannot be loaded, every entry point raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Sequence

__all__ = ["forward", "inverse", "spin_flip", "spin_flip_batch", "forward_compact", "inverse_compact", "compact_batch", "forward_noalloc", "forward_noalloc_batch", "quadrature_weights", "integrate",
           "integrate_batch", "forward_adjoint", "inverse_adjoint", "forward_batch",
           "inverse_batch", "forward_adjoint_batch", "inverse_adjoint_batch", "prepare", "release",
           "workspace_size", "set_workspace", "library", "MWError", "FP64", "FP32C", "EXPORTS", "LIB_PATH"]

FP64, FP32C = 0, 1
_PREC = {"fp64": FP64, "fp32c": FP32C, FP64: FP64, FP32C: FP32C}

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libmw.so")
EXPORTS = ("mw_forward", "mw_forward_noalloc", "mw_inverse", "mw_quadrature_weights", "mw_integrate", "mw_spin_flip",
           "mw_forward_compact", "mw_inverse_compact", "mw_forward_adjoint_compact", "mw_inverse_adjoint_compact", "mw_forward_adjoint", "mw_inverse_adjoint",
           "mw_workspace_size", "mw_set_workspace", "mw_prepare", "mw_release", "mw_status_string",
           "mw_last_error", "mw_version")
PROFILE_EXPORTS = ("mw_profile_enable", "mw_profile_read", "mw_profile_stage_name", "mw_profile_tuned_group",
                   "mw_profile_split_fft", "mw_profile_inverse_triangle", "mw_profile_tune_cache_load")
NSTAGE = 9

_lib = None


class MWError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str):
        super().__init__("%s failed: status %d (%s)" % (what, status, detail))
        self.status = status


def library():
    """The loaded ``libmw.so`` (ctypes.CDLL), loading it on first use."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmw.so is not built (%s); run `python -m paper_1110_6298_amd.build`"
                               % LIB_PATH)
        lib = ctypes.CDLL(LIB_PATH)
        i32p = ctypes.POINTER(ctypes.c_int32)
        vpp = ctypes.POINTER(ctypes.c_void_p)
        for name in ("mw_forward", "mw_forward_noalloc", "mw_inverse", "mw_forward_adjoint",
                     "mw_inverse_adjoint", "mw_forward_compact", "mw_inverse_compact",
                     "mw_forward_adjoint_compact", "mw_inverse_adjoint_compact"):
            fn = getattr(lib, name)
            fn.restype = ctypes.c_int
            fn.argtypes = [i32p, i32p, i32p, ctypes.c_int32, vpp, ctypes.c_int32, ctypes.c_void_p]
        lib.mw_spin_flip.restype = ctypes.c_int
        lib.mw_spin_flip.argtypes = [i32p, i32p, ctypes.c_int32, vpp, ctypes.c_void_p]
        lib.mw_quadrature_weights.restype = ctypes.c_int
        lib.mw_quadrature_weights.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p, ctypes.c_void_p]
        lib.mw_integrate.restype = ctypes.c_int
        lib.mw_integrate.argtypes = [i32p, i32p, i32p, ctypes.c_int32, vpp, ctypes.c_int32, ctypes.c_void_p]
        lib.mw_workspace_size.restype = ctypes.c_int
        lib.mw_workspace_size.argtypes = [i32p, i32p, i32p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_size_t)]
        lib.mw_set_workspace.restype = ctypes.c_int
        lib.mw_set_workspace.argtypes = [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        lib.mw_prepare.restype = ctypes.c_int
        lib.mw_prepare.argtypes = [i32p, i32p, i32p, ctypes.c_int32, ctypes.c_int32]
        lib.mw_release.restype = ctypes.c_int
        lib.mw_release.argtypes = []
        for name in ("mw_status_string",):
            getattr(lib, name).restype = ctypes.c_char_p
            getattr(lib, name).argtypes = [ctypes.c_int]
        for name in ("mw_last_error", "mw_version"):
            getattr(lib, name).restype = ctypes.c_char_p
            getattr(lib, name).argtypes = []
        lib.mw_profile_enable.restype = ctypes.c_int
        lib.mw_profile_enable.argtypes = [ctypes.c_int]
        lib.mw_profile_read.restype = ctypes.c_int
        lib.mw_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int)]
        lib.mw_profile_stage_name.restype = ctypes.c_char_p
        lib.mw_profile_stage_name.argtypes = [ctypes.c_int]
        lib.mw_profile_split_fft.restype = ctypes.c_int
        lib.mw_profile_split_fft.argtypes = [ctypes.c_int]
        lib.mw_profile_inverse_triangle.restype = ctypes.c_int
        lib.mw_profile_inverse_triangle.argtypes = [ctypes.c_int]
        lib.mw_profile_tune_cache_load.restype = ctypes.c_int
        lib.mw_profile_tune_cache_load.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_int)]
        lib.mw_profile_tuned_group.restype = ctypes.c_int
        lib.mw_profile_tuned_group.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                               ctypes.POINTER(ctypes.c_int)]
        _lib = lib
    return _lib


def _arr(vals):
    vals = [int(v) for v in vals]
    return (ctypes.c_int32 * len(vals))(*vals)


def _check(rc: int, what: str):
    if rc != 0:
        lib = library()
        raise MWError(rc, what, lib.mw_last_error().decode() or lib.mw_status_string(rc).decode())


def _stream_handle(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def call(name: str, Ls: Sequence[int], spins: Sequence[int], reals: Sequence[int], ptrs: Sequence[int],
         precision=FP64, stream=None) -> None:
    """Raw C-ABI call: ``ptrs`` are integer device addresses (2 per map)."""
    lib = library()
    n = len(Ls)
    parr = (ctypes.c_void_p * (2 * n))(*[ctypes.c_void_p(int(p)) for p in ptrs])
    rc = getattr(lib, name)(_arr(Ls), _arr(spins), _arr(reals), n,
                            ctypes.cast(parr, ctypes.POINTER(ctypes.c_void_p)),
                            _PREC[precision], _stream_handle(stream))
    _check(rc, name)


def _check_tensor(t, shape, dtypes, what):
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA tensor" % what)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s must have shape %s (got %s)" % (what, tuple(shape), tuple(t.shape)))
    if t.dtype not in dtypes:
        raise TypeError("%s has dtype %s, expected one of %s" % (what, t.dtype, dtypes))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % what)


def _map_shape(L):
    return (L, 2 * L - 1)


_MAP, _COEF, _CMAP = "map", "coeffs", "compact map"
_OPS = {  # name: (input kind, output kind)
    "mw_forward_compact": (_CMAP, _COEF),
    "mw_inverse_compact": (_COEF, _CMAP),
    "mw_forward_adjoint_compact": (_COEF, _CMAP),
    "mw_inverse_adjoint_compact": (_CMAP, _COEF),
    "mw_forward": (_MAP, _COEF),
    "mw_forward_noalloc": (_MAP, _COEF),
    "mw_inverse": (_COEF, _MAP),
    "mw_forward_adjoint": (_COEF, _MAP),
    "mw_inverse_adjoint": (_MAP, _COEF),
}


def _kind_spec(kind, L, real):
    import torch
    if kind == _MAP:
        return _map_shape(L), (torch.float64 if real else torch.complex128)
    if kind == _CMAP:
        return ((L - 1) * (2 * L - 1) + 1,), (torch.float64 if real else torch.complex128)
    return (L * L,), torch.complex128


def _batch(name, inputs, Ls, spins, realities, precision, outs, stream):
    n = len(inputs)
    if not (len(Ls) == len(spins) == n):
        raise ValueError("inputs, Ls and spins must have the same length")
    realities = [0] * n if realities is None else list(realities)
    outs = list(outs) if outs is not None else [None] * n
    kin, kout = _OPS[name]
    import torch
    ptrs = []
    for b in range(n):
        L = int(Ls[b])
        shp, dt = _kind_spec(kin, L, realities[b])
        _check_tensor(inputs[b], shp, (dt,), "%s %d" % (kin, b))
        shp, dt = _kind_spec(kout, L, realities[b])
        if outs[b] is None:
            outs[b] = torch.empty(shp, dtype=dt, device=inputs[b].device)
        _check_tensor(outs[b], shp, (dt,), "%s %d" % (kout, b))
        ptrs += [inputs[b].data_ptr(), outs[b].data_ptr()]
    call(name, Ls, spins, realities, ptrs, precision, stream)
    return outs


def forward_batch(maps, Ls, spins, realities=None, precision=FP64, outs=None, stream=None):
    """Forward transforms of a batch of maps in one library call (maps of
    reality 1 are float64, the others complex128)."""
    return _batch("mw_forward", maps, Ls, spins, realities, precision, outs, stream)


def forward_noalloc_batch(maps, Ls, spins, realities=None, precision=FP64, outs=None, stream=None):
    """mw_forward_noalloc: the forward transforms of a batch with the library's
    static device scratch as workspace (no allocation in the call; the plans
    must have been prepared, and the call's workspace must fit MW_NOALLOC_BYTES)."""
    return _batch("mw_forward_noalloc", maps, Ls, spins, realities, precision, outs, stream)


def inverse_batch(coeffs, Ls, spins, realities=None, precision=FP64, outs=None, stream=None):
    """Inverse transforms of a batch of coefficient vectors in one library call."""
    return _batch("mw_inverse", coeffs, Ls, spins, realities, precision, outs, stream)


def forward_adjoint_batch(coeffs, Ls, spins, realities=None, precision=FP64, outs=None, stream=None):
    """Adjoints of the forward map (coefficients -> grid) for a batch."""
    return _batch("mw_forward_adjoint", coeffs, Ls, spins, realities, precision, outs, stream)


def inverse_adjoint_batch(maps, Ls, spins, realities=None, precision=FP64, outs=None, stream=None):
    """Adjoints of the inverse map (grid -> coefficients) for a batch."""
    return _batch("mw_inverse_adjoint", maps, Ls, spins, realities, precision, outs, stream)


def compact_batch(name, inputs, Ls, spins, realities=None, precision=FP64, outs=None, stream=None):
    """The compact-storage transforms (Sec. IV-C): ``name`` is one of "forward",
    "inverse", "forward_adjoint", "inverse_adjoint"; maps are 1-D tensors of
    (L-1)(2L-1)+1 samples (the rings t < L-1, then the south-pole sample)."""
    return _batch("mw_%s_compact" % name, inputs, Ls, spins, realities, precision, outs, stream)


def forward_compact(x, L: int, spin: int = 0, reality: int = 0, precision=FP64, out=None, stream=None):
    """Forward transform of one map in compact storage ((L-1)(2L-1)+1 samples)."""
    return compact_batch("forward", [x], [L], [spin], [reality], precision, [out], stream)[0]


def inverse_compact(flm, L: int, spin: int = 0, reality: int = 0, precision=FP64, out=None, stream=None):
    """Inverse transform of one coefficient vector into compact storage."""
    return compact_batch("inverse", [flm], [L], [spin], [reality], precision, [out], stream)[0]


def forward(x, L: int, spin: int = 0, reality: int = 0, precision=FP64, out=None, stream=None):
    """Forward MW transform of one map (L, 2L-1) -> coefficients (L*L,)."""
    return forward_batch([x], [L], [spin], [reality], precision, [out], stream)[0]


def forward_noalloc(x, L: int, spin: int = 0, reality: int = 0, precision=FP64, out=None, stream=None):
    """Forward transform of one map without any allocation in the call (see
    forward_noalloc_batch)."""
    return forward_noalloc_batch([x], [L], [spin], [reality], precision, [out], stream)[0]


def inverse(flm, L: int, spin: int = 0, reality: int = 0, precision=FP64, out=None, stream=None):
    """Inverse MW transform of one coefficient vector (L*L,) -> map (L, 2L-1)."""
    return inverse_batch([flm], [L], [spin], [reality], precision, [out], stream)[0]


def forward_adjoint(y, L: int, spin: int = 0, reality: int = 0, precision=FP64, out=None, stream=None):
    """Conjugate transpose of the forward map: coefficients (L*L,) -> grid (L, 2L-1)
    (float64 Re(A^H y) when reality = 1)."""
    return forward_adjoint_batch([y], [L], [spin], [reality], precision, [out], stream)[0]


def inverse_adjoint(g, L: int, spin: int = 0, reality: int = 0, precision=FP64, out=None, stream=None):
    """Conjugate transpose of the inverse map: grid (L, 2L-1) -> coefficients (L*L,)."""
    return inverse_adjoint_batch([g], [L], [spin], [reality], precision, [out], stream)[0]


def spin_flip_batch(coeffs, Ls, spins, outs=None, stream=None):
    """Coefficients of the conjugate maps (spin -s) from spin-s coefficients:
    (-1)^{s+m} conj(f_{l,-m}) (Sec. IV-G).  ``outs`` may be the inputs (in place)."""
    import torch
    n = len(coeffs)
    outs = list(outs) if outs is not None else [None] * n
    ptrs = []
    for b in range(n):
        L = int(Ls[b])
        _check_tensor(coeffs[b], (L * L,), (torch.complex128,), "coeffs %d" % b)
        if outs[b] is None:
            outs[b] = torch.empty_like(coeffs[b])
        _check_tensor(outs[b], (L * L,), (torch.complex128,), "output %d" % b)
        ptrs += [coeffs[b].data_ptr(), outs[b].data_ptr()]
    parr = (ctypes.c_void_p * (2 * n))(*[ctypes.c_void_p(int(p)) for p in ptrs])
    _check(library().mw_spin_flip(_arr(Ls), _arr(spins), n, ctypes.cast(parr, ctypes.POINTER(ctypes.c_void_p)),
                                  _stream_handle(stream)), "mw_spin_flip")
    return outs


def spin_flip(flm, L: int, spin: int, out=None, stream=None):
    """Spin -s coefficients of the conjugate map of one coefficient vector."""
    return spin_flip_batch([flm], [L], [spin], [out], stream)[0]


GRID_QUADRATURE, GRID_TRANSFORM = 0, 1


def quadrature_weights(L: int, spin: int = 0, out=None, stream=None):
    """Weights q(theta_t), t < L, of the explicit quadrature (float64, on cuda)."""
    import torch
    if out is None:
        out = torch.empty(L, dtype=torch.float64, device="cuda")
    _check_tensor(out, (L,), (torch.float64,), "q")
    _check(library().mw_quadrature_weights(int(L), int(spin), ctypes.c_void_p(out.data_ptr()),
                                           _stream_handle(stream)), "mw_quadrature_weights")
    return out


def integrate_batch(maps, Ls, spins, realities=None, outs=None, stream=None):
    """Integrals over the sphere of a batch of maps by the explicit quadrature.
    Each map has shape (L, L) (the rule's grid) or (L, 2L-1) (the transforms'
    grid; all maps of one call on the same kind of grid); float64 when its
    reality is 1, else complex128.  Returns complex128 tensors of shape (1,)."""
    import torch
    n = len(maps)
    realities = [0] * n if realities is None else list(realities)
    if not (len(Ls) == len(spins) == len(realities) == n) or n == 0:
        raise ValueError("maps, Ls, spins and realities must have the same, nonzero length")
    grid = GRID_QUADRATURE if maps[0].dim() == 2 and maps[0].shape[1] == int(Ls[0]) else GRID_TRANSFORM
    outs = list(outs) if outs is not None else [None] * n
    ptrs = []
    for b in range(n):
        L = int(Ls[b])
        shp = (L, L) if grid == GRID_QUADRATURE else (L, 2 * L - 1)
        dt = torch.float64 if realities[b] else torch.complex128
        _check_tensor(maps[b], shp, (dt,), "map %d" % b)
        if outs[b] is None:
            outs[b] = torch.empty(1, dtype=torch.complex128, device=maps[b].device)
        _check_tensor(outs[b], (1,), (torch.complex128,), "integral %d" % b)
        ptrs += [maps[b].data_ptr(), outs[b].data_ptr()]
    lib = library()
    parr = (ctypes.c_void_p * (2 * n))(*[ctypes.c_void_p(int(p)) for p in ptrs])
    _check(lib.mw_integrate(_arr(Ls), _arr(spins), _arr(realities), n,
                            ctypes.cast(parr, ctypes.POINTER(ctypes.c_void_p)), grid, _stream_handle(stream)),
           "mw_integrate")
    return outs


def integrate(f, L: int, spin: int = 0, reality: int = 0, stream=None):
    """Integral over the sphere of one map (shape (L, L) or (L, 2L-1))."""
    return integrate_batch([f], [L], [spin], [reality], None, stream)[0]


def prepare(Ls, spins, realities=None, precision=FP64) -> None:
    """Build plans and workspace ahead of time (e.g. before stream capture)."""
    n = len(Ls)
    realities = [0] * n if realities is None else realities
    _check(library().mw_prepare(_arr(Ls), _arr(spins), _arr(realities), n, _PREC[precision]), "mw_prepare")


def workspace_size(Ls, spins, realities=None, precision=FP64) -> int:
    n = len(Ls)
    realities = [0] * n if realities is None else realities
    out = ctypes.c_size_t(0)
    _check(library().mw_workspace_size(_arr(Ls), _arr(spins), _arr(realities), n, _PREC[precision],
                                       ctypes.byref(out)), "mw_workspace_size")
    return int(out.value)


def set_workspace(buf, stream=None) -> None:
    """Bind a caller-owned device buffer (a CUDA tensor, or None to unbind) as the
    workspace of later calls on ``stream`` (default: the current torch stream).
    The caller keeps the tensor alive while those calls (or graph replays) run."""
    if buf is None:
        ptr, nbytes = None, 0
    else:
        import torch
        if not isinstance(buf, torch.Tensor) or not buf.is_cuda or not buf.is_contiguous():
            raise TypeError("the workspace must be a contiguous CUDA tensor")
        ptr, nbytes = ctypes.c_void_p(buf.data_ptr()), buf.numel() * buf.element_size()
    _check(library().mw_set_workspace(ptr, nbytes, _stream_handle(stream)), "mw_set_workspace")


def profile_enable(on: bool = True) -> None:
    """Bracket every kernel launch with HIP events on the launching stream."""
    _check(library().mw_profile_enable(1 if on else 0), "mw_profile_enable")


def profile_read() -> dict:
    """{stage name: (summed ms, launches)} of the kernels recorded since enabling."""
    lib = library()
    ms = (ctypes.c_double * NSTAGE)()
    cnt = (ctypes.c_int * NSTAGE)()
    _check(lib.mw_profile_read(ms, cnt), "mw_profile_read")
    return {lib.mw_profile_stage_name(i).decode(): (ms[i], cnt[i]) for i in range(NSTAGE) if cnt[i]}


def tuned_group(L: int, reality: int, nmaps: int) -> int:
    """Group size the autotuner chose for the groups that start at band-limit L in
    mixed-precision calls with ``nmaps`` maps of band-limit <= L and this
    reality (0 = not tuned)."""
    g = ctypes.c_int(0)
    _check(library().mw_profile_tuned_group(L, reality, nmaps, ctypes.byref(g)), "mw_profile_tuned_group")
    return int(g.value)


def tune_cache_load(path: str) -> int:
    """Load autotuner entries ("gfx950 L reality nmaps G" lines) from a file now;
    returns how many lines were taken (malformed ones are skipped)."""
    n = ctypes.c_int(0)
    _check(library().mw_profile_tune_cache_load(os.fsencode(path), ctypes.byref(n)), "mw_profile_tune_cache_load")
    return int(n.value)


def inverse_triangle(mode: int) -> None:
    """Test hook: mode 1 runs every later FP64 inverse (and forward adjoint) on
    the triangle contraction kernel, which by default runs real maps and complex
    maps from L = 1024; mode 0 restores the default."""
    _check(library().mw_profile_inverse_triangle(int(mode)), "mw_profile_inverse_triangle")


def split_fft(mode: int) -> None:
    """Test hook: mode 1 builds every later plan with N2 >= 2048 (L >= 257) with
    the split half-length Fourier kernels that L > 2048 needs; mode 0 restores
    the default."""
    _check(library().mw_profile_split_fft(int(mode)), "mw_profile_split_fft")


def release() -> None:
    _check(library().mw_release(), "mw_release")
