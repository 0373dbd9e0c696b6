"""Plain FP64 CPU oracle for the McEwen-Wiaux spin spherical-harmonic transforms.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py``; never by the product package.  It
shares no code with the GPU path.

``liboracle.so`` is built from ``mw_oracle.c`` with gcc + OpenMP (see ``build``).
Layouts follow the C file: map ``[t][p]`` (L x (2L-1)), coefficients at
``l*l + l + m``, planes ``[m + L-1][m' + L-1]``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mw_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``mw_oracle.c`` into ``liboracle.so`` (gcc, -O2, OpenMP, strict IEEE)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
               "-fno-fast-math", "-ffp-contract=off", _SRC, "-o", tmp, "-lm"]
        subprocess.check_call(cmd)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build(force=False)
        lib = ctypes.CDLL(_LIB_PATH)
        D = ctypes.POINTER(ctypes.c_double)
        I = ctypes.c_int
        IP = ctypes.POINTER(ctypes.c_int)
        sigs = {
            "orc_set_threads": (None, [I]),
            "orc_max_threads": (I, []),
            "orc_delta_plane": (I, [I, D]),
            "orc_weights": (None, [I, D]),
            "orc_forward": (I, [I, I, D, D]),
            "orc_forward_stages": (I, [I, I, D, D, D, D, D]),
            "orc_forward_orders": (I, [I, I, D, I, IP, D]),
            "orc_inverse": (I, [I, I, D, D]),
            "orc_inverse_orders": (I, [I, I, D, I, IP, D]),
            "orc_inverse_stages": (I, [I, I, D, D, D, D]),
            "orc_forward_adjoint": (I, [I, I, D, D]),
            "orc_inverse_adjoint": (I, [I, I, D, D]),
            "orc_row_plain": (I, [I, I, D]),
            "orc_quad_weights": (I, [I, I, D]),
            "orc_integrate": (I, [I, I, I, D, D]),
        }
        for name, (res, args) in sigs.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if a is not None else None


def _check(rc, what):
    if rc != 0:
        raise ValueError("oracle %s failed with code %d" % (what, rc))


def set_threads(n: int) -> None:
    _load().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def delta_plane(l: int) -> np.ndarray:
    """Delta^l_{m,n} = d^l_{mn}(pi/2) as a (2l+1)x(2l+1) array indexed [m+l, n+l]."""
    out = np.zeros((2 * l + 1, 2 * l + 1))
    _check(_load().orc_delta_plane(l, _dp(out)), "delta_plane")
    return out


def weights(L: int) -> np.ndarray:
    """w(k) for k = -2(L-1)..2(L-1) (weights of the theta convolution)."""
    out = np.zeros(4 * L - 3, dtype=np.complex128)
    _load().orc_weights(L, _dp(out.view(np.float64)))
    return out


def _grid(f, L):
    f = np.ascontiguousarray(f, dtype=np.complex128)
    if f.shape != (L, 2 * L - 1):
        raise ValueError("map must have shape (L, 2L-1)")
    return f


def _coeffs(flm, L):
    flm = np.ascontiguousarray(flm, dtype=np.complex128)
    if flm.shape != (L * L,):
        raise ValueError("coefficients must have shape (L*L,)")
    return flm


def forward(f, L: int, s: int) -> np.ndarray:
    """Forward MW transform (map -> f_lm) by the paper's algorithm, FP64."""
    f = _grid(f, L)
    out = np.zeros(L * L, dtype=np.complex128)
    _check(_load().orc_forward(L, s, _dp(f.view(np.float64)), _dp(out.view(np.float64))), "forward")
    return out


def forward_stages(f, L: int, s: int, contract: bool = True):
    """Intermediates of the forward: G[t][m], F[m][m'], Gmm[m][m'] and f_lm."""
    f = _grid(f, L)
    N1 = 2 * L - 1
    Gtm = np.zeros((L, N1), dtype=np.complex128)
    F = np.zeros((N1, N1), dtype=np.complex128)
    Gmm = np.zeros((N1, N1), dtype=np.complex128)
    flm = np.zeros(L * L, dtype=np.complex128) if contract else None
    rc = _load().orc_forward_stages(L, s, _dp(f.view(np.float64)), _dp(Gtm.view(np.float64)),
                                    _dp(F.view(np.float64)), _dp(Gmm.view(np.float64)),
                                    _dp(flm.view(np.float64)) if contract else None)
    _check(rc, "forward_stages")
    return Gtm, F, Gmm, flm


def forward_orders(f, L: int, s: int, ms) -> np.ndarray:
    """f_{l,m} for the listed orders m only: returns [len(ms)][L] (zero where |m|>l)."""
    f = _grid(f, L)
    ms = np.ascontiguousarray(ms, dtype=np.int32)
    out = np.zeros((ms.size, L), dtype=np.complex128)
    rc = _load().orc_forward_orders(L, s, _dp(f.view(np.float64)), int(ms.size),
                                    ms.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                    _dp(out.view(np.float64)))
    _check(rc, "forward_orders")
    return out


def inverse(flm, L: int, s: int) -> np.ndarray:
    """Inverse MW transform (f_lm -> map on the L x (2L-1) grid), FP64."""
    flm = _coeffs(flm, L)
    out = np.zeros((L, 2 * L - 1), dtype=np.complex128)
    _check(_load().orc_inverse(L, s, _dp(flm.view(np.float64)), _dp(out.view(np.float64))), "inverse")
    return out


def inverse_orders(flm, L: int, s: int, ms) -> np.ndarray:
    """F_m(theta_t) (the phi-Fourier coefficients of the inverse map's rings) for
    the listed orders: returns [len(ms)][L]."""
    flm = _coeffs(flm, L)
    ms = np.ascontiguousarray(ms, dtype=np.int32)
    out = np.zeros((ms.size, L), dtype=np.complex128)
    rc = _load().orc_inverse_orders(L, s, _dp(flm.view(np.float64)), int(ms.size),
                                    ms.ctypes.data_as(ctypes.POINTER(ctypes.c_int)),
                                    _dp(out.view(np.float64)))
    _check(rc, "inverse_orders")
    return out


def inverse_stages(flm, L: int, s: int):
    """Intermediates of the inverse: F[m][m'], F_m(theta_t) as [m][t], and the map."""
    flm = _coeffs(flm, L)
    N1 = 2 * L - 1
    F = np.zeros((N1, N1), dtype=np.complex128)
    Fmt = np.zeros((N1, L), dtype=np.complex128)
    f = np.zeros((L, N1), dtype=np.complex128)
    rc = _load().orc_inverse_stages(L, s, _dp(flm.view(np.float64)), _dp(F.view(np.float64)),
                                    _dp(Fmt.view(np.float64)), _dp(f.view(np.float64)))
    _check(rc, "inverse_stages")
    return F, Fmt, f


def forward_adjoint(y, L: int, s: int) -> np.ndarray:
    """Conjugate transpose of the forward map: coefficients -> grid."""
    y = _coeffs(y, L)
    out = np.zeros((L, 2 * L - 1), dtype=np.complex128)
    _check(_load().orc_forward_adjoint(L, s, _dp(y.view(np.float64)), _dp(out.view(np.float64))),
           "forward_adjoint")
    return out


def inverse_adjoint(g, L: int, s: int) -> np.ndarray:
    """Conjugate transpose of the inverse map: grid -> coefficients."""
    g = _grid(g, L)
    out = np.zeros(L * L, dtype=np.complex128)
    _check(_load().orc_inverse_adjoint(L, s, _dp(g.view(np.float64)), _dp(out.view(np.float64))),
           "inverse_adjoint")
    return out


def row_plain(l: int, m: int) -> np.ndarray:
    """Delta^l_{m,n}, n=0..l, by the plain-FP64 row recursion (stability study only)."""
    out = np.zeros(l + 1)
    _check(_load().orc_row_plain(l, m, _dp(out)), "row_plain")
    return out


def quad_weights(L: int, s: int) -> np.ndarray:
    """Weights q(theta_t), t < L, of the explicit quadrature Eq.(quadrature)
    (complex as evaluated; the imaginary part vanishes up to rounding)."""
    out = np.zeros(L, dtype=np.complex128)
    _check(_load().orc_quad_weights(L, s, _dp(out.view(np.float64))), "quad_weights")
    return out


def integrate(f, L: int, s: int) -> complex:
    """Integral of a map over the sphere by Eq.(quadrature): f of shape (L, L)
    (the rule's grid, phi'_p = 2 pi p/L) or (L, 2L-1) (the transform grid)."""
    f = np.ascontiguousarray(np.asarray(f, dtype=np.complex128))
    if f.ndim != 2 or f.shape[0] != L or f.shape[1] not in (L, 2 * L - 1):
        raise ValueError("map must have shape (L, L) or (L, 2L-1)")
    out = np.zeros(1, dtype=np.complex128)
    _check(_load().orc_integrate(L, s, f.shape[1], _dp(f.view(np.float64)), _dp(out.view(np.float64))),
           "integrate")
    return complex(out[0])


# --------------------------------------------------------------------------
# Compact storage (Sec. IV-C): N_MW = (L-1)(2L-1)+1 samples, the south pole once.
# The pole ring of a band-limited spin-s map is C e^{i s phi_p} with C = f(pi, 0)
# (at theta = pi only the order m = s survives; footnote on the poles, Sec. IV-B).
# --------------------------------------------------------------------------
def _pole_phase(L: int, s: int) -> np.ndarray:
    n1 = 2 * L - 1
    k = (s * np.arange(n1)) % n1
    return np.exp(2j * np.pi * k / n1)


def compact(f, L: int) -> np.ndarray:
    """Compact storage of a full-grid map: rings t < L-1, then f(pi, phi_0)."""
    f = np.asarray(f)
    return np.concatenate([f[:L - 1].reshape(-1), f[L - 1, :1]])


def expand_pole(fc, L: int, s: int) -> np.ndarray:
    """Full grid from compact storage, the pole ring C e^{i s phi_p}."""
    fc = np.asarray(fc, dtype=np.complex128)
    n1 = 2 * L - 1
    f = np.zeros((L, n1), dtype=np.complex128)
    f[:L - 1] = fc[:(L - 1) * n1].reshape(L - 1, n1)
    f[L - 1] = fc[(L - 1) * n1] * _pole_phase(L, s)
    return f


def forward_compact(fc, L: int, s: int) -> np.ndarray:
    return forward(expand_pole(fc, L, s), L, s)


def inverse_compact(flm, L: int, s: int) -> np.ndarray:
    return compact(inverse(flm, L, s), L)


def forward_adjoint_compact(y, L: int, s: int) -> np.ndarray:
    """Adjoint of forward_compact: the full adjoint's rings t < L-1 and, as the
    pole sample, sum_p e^{-i s phi_p} times its pole ring."""
    g = forward_adjoint(y, L, s)
    return np.concatenate([g[:L - 1].reshape(-1), [np.sum(np.conj(_pole_phase(L, s)) * g[L - 1])]])


def inverse_adjoint_compact(gc, L: int, s: int) -> np.ndarray:
    """Adjoint of inverse_compact: the full adjoint of the map whose pole ring
    holds the pole sample at p = 0 and zeros elsewhere."""
    gc = np.asarray(gc, dtype=np.complex128)
    n1 = 2 * L - 1
    g = np.zeros((L, n1), dtype=np.complex128)
    g[:L - 1] = gc[:(L - 1) * n1].reshape(L - 1, n1)
    g[L - 1, 0] = gc[(L - 1) * n1]
    return inverse_adjoint(g, L, s)
