"""Tiny-L brute force from the definitions (test infrastructure only).

* ``wigner_d`` -- d^l_{mn}(beta) from the Jacobi-polynomial closed form,
  Eq.(wignerd_b) (Sec. III-C), written for n >= |m| and extended to the whole
  plane with the symmetry Eq.(wignerd_sym1) and the transpose relation that
  follows from Eq.(wignerd_sym3).
* ``spin_harmonic`` -- sY_lm(theta, phi) = (-1)^s sqrt((2l+1)/4pi) D^{l*}_{m,-s}(phi, theta, 0),
  Eqs.(ssh_wigner) and (d_decomp).
* ``synthesis`` -- f(theta_t, phi_p) = sum_lm f_lm sY_lm on the MW grid of Eqs.(nodes_theta/phi).
* ``projection_gl`` -- f_lm = <f, sY_lm> by Gauss-Legendre quadrature in cos(theta)
  and a uniform rule in phi, exact for band-limited integrands (the exactness
  argument of the paper's Gauss-Legendre footnote in Sec. V).
Pure Python loops: only for L <= ~10.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import eval_jacobi


def wigner_d(l: int, m: int, n: int, beta: float) -> float:
    if abs(m) > l or abs(n) > l:
        return 0.0
    if n >= abs(m):
        pref = math.sqrt(math.factorial(l + n) * math.factorial(l - n) /
                         (math.factorial(l + m) * math.factorial(l - m)))
        return (pref * math.sin(beta / 2) ** (n - m) * math.cos(beta / 2) ** (n + m)
                * float(eval_jacobi(l - n, n - m, n + m, math.cos(beta))))
    if -n >= abs(m):
        # Eq.(wignerd_sym1): d_{mn} = (-1)^{m-n} d_{-m,-n}
        return (-1) ** (m - n) * wigner_d(l, -m, -n, beta)
    # |m| > |n|: d_{mn}(beta) = d_{nm}(-beta) = (-1)^{m-n} d_{nm}(beta)  (Eq.(wignerd_sym3))
    return (-1) ** (m - n) * wigner_d(l, n, m, beta)


def delta_plane(l: int) -> np.ndarray:
    out = np.zeros((2 * l + 1, 2 * l + 1))
    for m in range(-l, l + 1):
        for n in range(-l, l + 1):
            out[m + l, n + l] = wigner_d(l, m, n, math.pi / 2)
    return out


def spin_harmonic(l: int, m: int, s: int, theta, phi):
    theta = np.asarray(theta, dtype=np.float64)
    phi = np.asarray(phi, dtype=np.float64)
    d = np.vectorize(lambda th: wigner_d(l, m, -s, float(th)))(theta)
    return (-1) ** s * math.sqrt((2 * l + 1) / (4 * math.pi)) * np.exp(1j * m * phi) * d


def grid(L: int):
    t = np.arange(L)
    p = np.arange(2 * L - 1)
    return np.pi * (2 * t + 1) / (2 * L - 1), 2 * np.pi * p / (2 * L - 1)


def synthesis(flm, L: int, s: int) -> np.ndarray:
    theta, phi = grid(L)
    f = np.zeros((L, 2 * L - 1), dtype=np.complex128)
    TH, PH = np.meshgrid(theta, phi, indexing="ij")
    for l in range(abs(s), L):
        for m in range(-l, l + 1):
            c = flm[l * l + l + m]
            if c != 0:
                f += c * spin_harmonic(l, m, s, TH, PH)
    return f


def projection_gl(func, L: int, s: int) -> np.ndarray:
    """f_lm = int dOmega func(theta, phi) conj(sY_lm) for a band-limited func(theta, phi)."""
    x, wx = np.polynomial.legendre.leggauss(L + 1)
    theta = np.arccos(x)
    nphi = 2 * L + 1
    phi = 2 * np.pi * np.arange(nphi) / nphi
    TH, PH = np.meshgrid(theta, phi, indexing="ij")
    vals = func(TH, PH)
    out = np.zeros(L * L, dtype=np.complex128)
    for l in range(abs(s), L):
        for m in range(-l, l + 1):
            Y = spin_harmonic(l, m, s, TH, PH)
            out[l * l + l + m] = (2 * np.pi / nphi) * np.sum(wx[:, None] * vals * np.conj(Y))
    return out


def n_samples(L: int) -> dict:
    """Sample counts of the sampling theorems compared in Sec. II and Sec. V-A."""
    return {"MW": (L - 1) * (2 * L - 1) + 1, "GL": L * (2 * L - 1), "DH": 2 * L * (2 * L - 1),
            "S": (2 * L - 1) ** 2}
