"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's own formulas: each compares against an
independent route (Jacobi closed form, numerical integration, group
identities, brute-force synthesis, Gauss-Legendre projection, closed-form
harmonics, printed sample counts).  Run without a GPU.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy import integrate

import mwsynth
from oracle import brute

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rel_inf(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# --------------------------------------------------------------------------
# Delta^l = d^l(pi/2) from Risbo's recursion
# --------------------------------------------------------------------------
@pytest.mark.parametrize("l", list(range(0, 11)))
def test_delta_matches_jacobi_closed_form(orc, l):
    # Eq.(wignerd_b) (Jacobi polynomials) extended by Eq.(wignerd_sym1)/(wignerd_sym3)
    np.testing.assert_allclose(orc.delta_plane(l), brute.delta_plane(l), atol=2e-15, rtol=0)


@pytest.mark.parametrize("l", [1, 7, 40, 150])
def test_delta_orthogonal_and_squares_to_d_pi(orc, l):
    P = orc.delta_plane(l)
    n = 2 * l + 1
    # d(pi/2) is an orthogonal matrix (unitarity of the rotation representation)
    assert np.abs(P.T @ P - np.eye(n)).max() < 5e-14 * max(1, l / 10)
    # d(pi/2) d(pi/2) = d(pi) and d^l_{mn}(pi) = (-1)^{l-n} delta_{m,-n} (Eq.(wignerd_sym2) at beta=0)
    dpi = np.zeros((n, n))
    for k in range(-l, l + 1):
        dpi[-k + l, k + l] = (-1) ** (l - k)
    assert np.abs(P @ P - dpi).max() < 5e-14 * max(1, l / 10)


@pytest.mark.parametrize("l", [3, 8, 33])
def test_delta_symmetries(orc, l):
    P = orc.delta_plane(l)
    idx = np.arange(-l, l + 1)
    M, N = np.meshgrid(idx, idx, indexing="ij")
    # Eq.(wignerd_sym1): d_{mn} = (-1)^{m-n} d_{-m,-n}
    assert np.abs(P - (-1.0) ** (M - N) * P[::-1, ::-1]).max() < 1e-14
    # Eq.(wignerd_sym2) at beta = pi/2: Delta_{mn} = (-1)^{l-n} Delta_{-m,n}
    assert np.abs(P - (-1.0) ** (l - N) * P[::-1, :]).max() < 1e-14
    # Eq.(wignerd_sym3) at beta = pi/2 with d(-beta) = d(beta)^T: Delta_{mn} = (-1)^{m-n} Delta_{nm}
    assert np.abs(P - (-1.0) ** (M - N) * P.T).max() < 1e-14


@pytest.mark.parametrize("l", [5, 60, 200])
def test_delta_edge_closed_form(orc, l):
    # Eq.(wignerd_b) at n = l (Jacobi polynomial of degree 0):
    # d^l_{ml}(pi/2) = sqrt((2l)!/((l+m)!(l-m)!)) 2^{-l}
    P = orc.delta_plane(l)
    for m in range(-l, l + 1):
        ref = math.sqrt(float(math.comb(2 * l, l + m))) / 2.0 ** l   # exact integer binomial
        assert abs(P[m + l, 2 * l] - ref) <= 4e-16 * (2 * l + 1) * ref   # ~eps per half-step


@pytest.mark.parametrize("l", [2, 6, 10])
def test_fourier_factoring_of_d(orc, l):
    # Eq.(wigner_sum_reln): d^l_{mn}(b) = i^{n-m} sum_m' Delta_{m'm} Delta_{m'n} e^{i m' b}
    P = orc.delta_plane(l)
    rng = np.random.default_rng(7 + l)
    for beta in rng.uniform(0, np.pi, size=3):
        for m in range(-l, l + 1):
            for n in range(-l, l + 1):
                mp = np.arange(-l, l + 1)
                val = (1j) ** (n - m) * np.sum(P[mp + l, m + l] * P[mp + l, n + l] * np.exp(1j * mp * beta))
                assert abs(val.imag) < 1e-13
                assert abs(val.real - brute.wigner_d(l, m, n, beta)) < 2e-13


# --------------------------------------------------------------------------
# Weights of the theta convolution
# --------------------------------------------------------------------------
def test_weights_are_the_sine_integrals(orc):
    # w(k) is defined as int_0^pi sin(theta) e^{i k theta} d theta (Sec. IV-D)
    L = 9
    w = orc.weights(L)
    for k in range(-2 * (L - 1), 2 * (L - 1) + 1):
        re = integrate.quad(lambda t: math.sin(t) * math.cos(k * t), 0, math.pi, limit=200)[0]
        im = integrate.quad(lambda t: math.sin(t) * math.sin(k * t), 0, math.pi, limit=200)[0]
        assert abs(w[k + 2 * (L - 1)] - (re + 1j * im)) < 1e-12, k


# --------------------------------------------------------------------------
# Inverse transform
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L,s", [(1, 0), (2, 0), (4, 0), (5, 2), (6, -1), (6, 3), (7, 1)])
def test_inverse_equals_brute_synthesis(orc, L, s):
    flm = mwsynth.flm_gaussian(L, s, seed=100 + L + 10 * s)
    ref = brute.synthesis(flm, L, s)
    got = orc.inverse(flm, L, s)
    assert rel_inf(got, ref) < 1e-13


def test_inverse_low_l_closed_forms(orc):
    L = 6
    theta, phi = brute.grid(L)
    TH, PH = np.meshgrid(theta, phi, indexing="ij")

    def single(l, m, s):
        flm = np.zeros(L * L, dtype=np.complex128)
        flm[l * l + l + m] = 1.0
        return orc.inverse(flm, L, s)

    # scalar harmonics with the Condon-Shortley phase (Sec. III-A)
    assert np.abs(single(0, 0, 0) - 1 / math.sqrt(4 * math.pi)).max() < 1e-14
    assert np.abs(single(1, 0, 0) - math.sqrt(3 / (4 * math.pi)) * np.cos(TH)).max() < 1e-14
    assert np.abs(single(1, 1, 0) + math.sqrt(3 / (8 * math.pi)) * np.sin(TH) * np.exp(1j * PH)).max() < 1e-14
    assert np.abs(single(2, 0, 0) - math.sqrt(5 / (16 * math.pi)) * (3 * np.cos(TH) ** 2 - 1)).max() < 1e-14
    # spin-2 harmonics from Eq.(ssh_wigner) with textbook d^2 values:
    # d^2_{2,-2}(t) = sin^4(t/2), d^2_{0,-2}(t) = sqrt(3/8) sin^2 t
    assert np.abs(single(2, 2, 2) - math.sqrt(5 / (4 * math.pi)) * np.exp(2j * PH) * np.sin(TH / 2) ** 4).max() < 1e-14
    assert np.abs(single(2, 0, 2) - math.sqrt(5 / (4 * math.pi)) * math.sqrt(3 / 8) * np.sin(TH) ** 2).max() < 1e-14


@pytest.mark.parametrize("s", [0, 2, -3])
def test_inverse_south_pole_ring(orc, s):
    # At theta = pi only m = s survives (d^l_{m,-s}(pi) ~ delta_{m,s}), so the last ring
    # of any band-limited map is c * exp(i s phi_p) (pole footnote of Sec. IV-B).
    L = 10
    flm = mwsynth.flm_gaussian(L, s, seed=3)
    f = orc.inverse(flm, L, s)
    phi = 2 * np.pi * np.arange(2 * L - 1) / (2 * L - 1)
    ring = f[L - 1] * np.exp(-1j * s * phi)
    assert np.abs(ring - ring[0]).max() < 1e-13


# --------------------------------------------------------------------------
# Forward transform
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L,s", [(3, 0), (5, 2), (6, -1), (7, 3)])
def test_forward_equals_gauss_legendre_projection(orc, L, s):
    # f_lm = <f, sY_lm> evaluated by Gauss-Legendre quadrature, exact for band-limited f
    flm = mwsynth.flm_gaussian(L, s, seed=200 + L)

    def func(TH, PH):
        out = np.zeros(TH.shape, dtype=np.complex128)
        for l in range(abs(s), L):
            for m in range(-l, l + 1):
                out += flm[l * l + l + m] * brute.spin_harmonic(l, m, s, TH, PH)
        return out

    proj = brute.projection_gl(func, L, s)
    np.testing.assert_allclose(proj, flm, atol=1e-13)   # the quadrature itself is exact
    f = brute.synthesis(flm, L, s)
    got = orc.forward(f, L, s)
    assert rel_inf(got, proj) < 1e-13


@pytest.mark.parametrize("L,s", [(2, 0), (16, 0), (16, 2), (17, -2), (24, 5), (32, 1)])
def test_round_trip_exact(orc, L, s):
    # The sampling theorem (Sec. IV-E): forward(inverse(f_lm)) = f_lm for band-limited f_lm
    flm = mwsynth.flm_uniform(L, s, seed=300 + L)
    back = orc.forward(orc.inverse(flm, L, s), L, s)
    assert np.abs(back - flm).max() < 1e-14 * L + 1e-14


def test_round_trip_error_grows_slowly(orc):
    # paper Sec. V-D: max abs error of order machine precision, growing ~linearly with L
    errs = {}
    for L in (16, 64, 128):
        flm = mwsynth.flm_uniform(L, 0, seed=5)
        errs[L] = np.abs(orc.forward(orc.inverse(flm, L, 0), L, 0) - flm).max()
    assert errs[128] < 1e-12
    assert errs[128] < 40 * errs[16] + 1e-14


def test_forward_and_inverse_share_fmm(orc):
    # Both sides of Eq.(Gmt_Fmt): the F_{mm'} of the forward's theta-DFT equals Eq.(Fmm)
    L, s = 9, 2
    flm = mwsynth.flm_gaussian(L, s, seed=11)
    Finv, _, f = orc.inverse_stages(flm, L, s)
    _, Ffwd, _, _ = orc.forward_stages(f, L, s, contract=False)
    assert np.abs(Ffwd - Finv).max() < 1e-14


def test_fmm_symmetry(orc):
    # Eq.(Fmm_sym1): F_{m,-m'} = (-1)^{m+s} F_{m m'}
    L, s = 8, 3
    F, _, _ = orc.inverse_stages(mwsynth.flm_gaussian(L, s, seed=12), L, s)
    m = np.arange(-(L - 1), L)
    assert np.abs(F[:, ::-1] - ((-1.0) ** (m + s))[:, None] * F).max() < 1e-14


def test_forward_responds_to_pole_ring(orc):
    # reading of the grid: every sample of the south-pole ring is used as given
    L, s = 6, 0
    f = orc.inverse(mwsynth.flm_gaussian(L, s, seed=13), L, s)
    g = f.copy()
    phi = 2 * np.pi * np.arange(2 * L - 1) / (2 * L - 1)
    g[L - 1] += 1e-3 * np.exp(1j * (s + 1) * phi)
    assert np.abs(orc.forward(g, L, s) - orc.forward(f, L, s)).max() > 1e-6


def test_real_signal_symmetries(orc):
    # Sec. IV-G: real s=0 maps have f*_lm = (-1)^m f_{l,-m} and F_{-m,-m'} = conj(F_{mm'})
    L = 12
    rng = np.random.default_rng(14)
    f = rng.standard_normal((L, 2 * L - 1)).astype(np.complex128)
    flm = orc.forward(f, L, 0)
    l, m = mwsynth.lm_arrays(L)
    np.testing.assert_allclose(np.conj(flm), (-1.0) ** m * flm[l * l + l - m], atol=1e-14)
    F, _, _ = orc.inverse_stages(mwsynth.make_real_symmetric(mwsynth.flm_gaussian(L, 0, 15), L), L, 0)
    assert np.abs(F[::-1, ::-1] - np.conj(F)).max() < 1e-14


def test_spin_independent_accuracy(orc):
    # Sec. V-D: error is identical (to statistical noise) across s in {0, 2, 10}
    L = 48
    errs = []
    for s in (0, 2, 10):
        flm = mwsynth.flm_uniform(L, s, seed=21)
        errs.append(np.abs(orc.forward(orc.inverse(flm, L, s), L, s) - flm).max())
    assert max(errs) < 5 * min(errs) + 1e-15


def test_forward_orders_matches_full(orc):
    L, s = 20, 2
    f = orc.inverse(mwsynth.flm_gaussian(L, s, 16), L, s) + 0.1 * mwsynth.grid_gaussian(L, 17)
    full = orc.forward(f, L, s)
    ms = [-19, -3, 0, 2, 7, 19]
    part = orc.forward_orders(f, L, s, ms)
    for k, m in enumerate(ms):
        for l in range(L):
            ref = full[l * l + l + m] if abs(m) <= l else 0
            assert abs(part[k, l] - ref) < 1e-15


@pytest.mark.parametrize("L", [5, 9, 20])
@pytest.mark.parametrize("s", [0, 2, -3])
def test_inverse_orders_are_ring_fourier_coefficients(orc, L, s):
    # Eq.(f_pfft): F_m(theta_t) is the phi-Fourier coefficient of ring t of the
    # inverse map, (1/N1) sum_p f(theta_t, phi_p) e^{-i m phi_p}.  The map comes
    # from the full inverse (itself pinned by brute-force synthesis), the ring
    # DFT from numpy; negative m sit at residue m mod N1.
    if abs(s) >= L:
        pytest.skip("spin needs |s| < L")
    N1 = 2 * L - 1
    flm = mwsynth.flm_gaussian(L, s, seed=40 + L)
    ring_dft = np.fft.fft(orc.inverse(flm, L, s), axis=1) / N1    # [t][m mod N1]
    ms = sorted({-(L - 1), -2, -1, 0, 1, 3 % L, L - 1})
    got = orc.inverse_orders(flm, L, s, ms)
    scale = np.abs(ring_dft).max()
    for k, m in enumerate(ms):
        np.testing.assert_allclose(got[k], ring_dft[:, m % N1], atol=1e-14 * scale, rtol=0)


# --------------------------------------------------------------------------
# Adjoints (dot-product identity)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L,s", [(5, 0), (8, 2), (9, -1)])
def test_adjoint_dot_products(orc, L, s):
    rng = np.random.default_rng(30 + L)
    x = mwsynth.grid_gaussian(L, 31 + L)
    y = mwsynth.zero_below_spin(mwsynth.complex_normal(rng, L * L), L, s)
    lhs = np.vdot(y, orc.forward(x, L, s))
    rhs = np.vdot(orc.forward_adjoint(y, L, s), x)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    g = mwsynth.grid_gaussian(L, 32 + L)
    lhs = np.vdot(g, orc.inverse(y, L, s))
    rhs = np.vdot(orc.inverse_adjoint(g, L, s), y)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def test_forward_adjoint_is_not_inverse(orc):
    # the forward uses quadrature weights, so A^H != Y
    L, s = 5, 0
    y = mwsynth.flm_gaussian(L, s, 40)
    assert np.abs(orc.forward_adjoint(y, L, s) - orc.inverse(y, L, s)).max() > 0.1


# --------------------------------------------------------------------------
# Sample counts (Sec. II, IV-C, V-A, V-E)
# --------------------------------------------------------------------------
def test_sample_counts_golden():
    with open(os.path.join(GOLDEN, "sample_counts.json")) as fh:
        g = json.load(fh)
    for L in range(1, 12):
        n = brute.n_samples(L)
        assert (n["MW"] == L * L) == (L in g["bound_L"]["MW"])
        assert (n["GL"] == L * L) == (L in g["bound_L"]["GL"])
        assert n["GL"] - n["MW"] == 2 * (L - 1)
        assert n["MW"] >= L * L and n["DH"] > n["GL"]
    gl = sum(brute.n_samples(L)["GL"] for L in g["mri_shells"])
    mw = sum(brute.n_samples(L)["MW"] for L in g["mri_shells"])
    assert round(100 * (gl - mw) / gl) == g["mri_reduction_percent"]


# --------------------------------------------------------------------------
# Stability observation of Sec. V-D: a plain-FP64 row recursion started from
# the edge breaks down at large l (its 2^-l start underflows); at moderate l it
# agrees with Risbo.
# --------------------------------------------------------------------------
def test_plain_row_recursion_agrees_at_moderate_l(orc):
    l = 60
    P = orc.delta_plane(l)
    for m in (0, 13, 59, 60):
        np.testing.assert_allclose(orc.row_plain(l, m), P[m + l, l:], atol=1e-13)


def test_plain_row_recursion_fails_at_large_l(orc):
    l = 1200
    row = orc.row_plain(l, l)   # start 2^-1200 underflows in FP64
    norm = row[0] ** 2 + 2 * np.sum(row[1:] ** 2)
    assert abs(norm - 1.0) > 0.5
    row0 = orc.row_plain(l, 3)  # start ~ l^-1/4 is representable: row stays unitary
    norm0 = row0[0] ** 2 + 2 * np.sum(row0[1:] ** 2)
    assert abs(norm0 - 1.0) < 1e-12


# --------------------------------------------------------------------------
# Explicit quadrature (Sec. IV-F, Eq.(quadrature))
# --------------------------------------------------------------------------
def _synth_on(flm, L, s, theta, phi):
    """Brute-force synthesis sum_lm f_lm sY_lm on an arbitrary product grid."""
    TH, PH = np.meshgrid(theta, phi, indexing="ij")
    f = np.zeros(TH.shape, dtype=np.complex128)
    for l in range(abs(s), L):
        for m in range(-l, l + 1):
            c = flm[l * l + l + m]
            if c != 0:
                f += c * brute.spin_harmonic(l, m, s, TH, PH)
    return f


def _exact_integral(flm, L, s):
    """int dOmega sum_lm f_lm sY_lm: only m = 0 survives the phi integral (2 pi);
    the theta integral of sin(theta) sY_l0(theta, 0) by 120-point Gauss-Legendre
    in theta on [0, pi] (smooth integrand, converged to rounding)."""
    x, w = np.polynomial.legendre.leggauss(120)
    th = 0.5 * np.pi * (x + 1.0)
    wt = 0.5 * np.pi * w
    tot = 0.0
    for l in range(abs(s), L):
        y = brute.spin_harmonic(l, 0, s, th, np.zeros_like(th))
        tot += flm[l * l + l] * 2.0 * np.pi * np.sum(wt * np.sin(th) * y)
    return tot


@pytest.mark.parametrize("L", [1, 2, 3, 8, 33])
def test_quadrature_weights_integrate_one(orc, L):
    # f = 1: L rings of L samples, sum_t L q_t = 4 pi; the weights are real
    q = orc.quad_weights(L, 0)
    assert abs(L * q.real.sum() - 4 * np.pi) < 1e-13
    assert np.abs(q.imag).max() < 1e-15
    assert np.allclose(orc.integrate(np.ones((L, L)), L, 0), 4 * np.pi, rtol=1e-14, atol=0)
    assert np.allclose(orc.integrate(np.ones((L, 2 * L - 1)), L, 0), 4 * np.pi, rtol=1e-14, atol=0)


@pytest.mark.parametrize("L", [2, 3, 5, 8])
def test_quadrature_exact_for_band_limited_scalar(orc, L):
    # int Y_lm dOmega = sqrt(4 pi) delta_l0 delta_m0, so I = sqrt(4 pi) f_00
    flm = mwsynth.flm_gaussian(L, 0, seed=900 + L)
    theta = np.pi * (2 * np.arange(L) + 1) / (2 * L - 1)
    for nphi in (L, 2 * L - 1):
        f = _synth_on(flm, L, 0, theta, 2 * np.pi * np.arange(nphi) / nphi)
        got = orc.integrate(f, L, 0)
        assert abs(got - math.sqrt(4 * np.pi) * flm[0]) < 1e-13 * np.abs(flm).max(), nphi


@pytest.mark.parametrize("L,s", [(4, 1), (5, 2), (6, -3), (7, 2)])
def test_quadrature_exact_for_band_limited_spin(orc, L, s):
    # spin-s maps: the rule reproduces int dOmega f, computed independently
    flm = mwsynth.flm_gaussian(L, s, seed=950 + L)
    theta = np.pi * (2 * np.arange(L) + 1) / (2 * L - 1)
    ref = _exact_integral(flm, L, s)
    assert abs(ref) > 1e-3
    for nphi in (L, 2 * L - 1):
        f = _synth_on(flm, L, s, theta, 2 * np.pi * np.arange(nphi) / nphi)
        assert abs(orc.integrate(f, L, s) - ref) < 1e-13 * np.abs(flm).max(), nphi


# --------------------------------------------------------------------------
# Compact storage (Sec. IV-C): N_MW samples, the pole once
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L,s", [(2, 0), (5, 2), (7, -3), (9, 1)])
def test_compact_storage_is_exact(orc, L, s):
    flm = mwsynth.flm_gaussian(L, s, seed=970 + L)
    xc = orc.inverse_compact(flm, L, s)
    assert xc.size == brute.n_samples(L)["MW"]
    # the pole ring of the brute-force synthesis is C e^{i s phi_p} with the stored C
    x = brute.synthesis(flm, L, s)
    assert rel_inf(orc.expand_pole(xc, L, s), x) < 1e-13
    # the sampling theorem on N_MW samples: forward(inverse) = identity
    assert rel_inf(orc.forward_compact(xc, L, s), flm) < 1e-13


@pytest.mark.parametrize("L,s", [(4, 0), (6, 2), (8, -1)])
def test_compact_adjoint_dot_products(orc, L, s):
    rng = np.random.default_rng(990 + L)
    n = brute.n_samples(L)["MW"]
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    y = mwsynth.zero_below_spin(mwsynth.flm_gaussian(L, 0, seed=991 + L), L, s)
    lhs, rhs = np.vdot(y, orc.forward_compact(x, L, s)), np.vdot(orc.forward_adjoint_compact(y, L, s), x)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    lhs, rhs = np.vdot(x, orc.inverse_compact(y, L, s)), np.vdot(orc.inverse_adjoint_compact(x, L, s), y)
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)


# --------------------------------------------------------------------------
# Spin -s coefficients of the conjugate map (Sec. IV-G)
# --------------------------------------------------------------------------
@pytest.mark.parametrize("L,s", [(6, 0), (7, 2), (8, -3)])
def test_conjugate_map_has_flipped_coefficients(orc, L, s):
    # conj(sY_lm) = (-1)^{s+m} (-s)Y_{l,-m}, so conj(f) of spin -s has coefficients
    # (-1)^{s+m} conj(f_{l,-m}); checked on brute-force synthesis and on the
    # oracle's forward of a grid that is not band-limited (the algorithm commutes
    # with conjugation as well)
    flm = mwsynth.flm_gaussian(L, s, seed=1300 + L)
    l, m = mwsynth.lm_arrays(L)
    flip = (-1.0) ** (s + m) * np.conj(flm[l * l + l - m])
    assert rel_inf(np.conj(brute.synthesis(flm, L, s)), brute.synthesis(flip, L, -s)) < 1e-13
    x = mwsynth.grid_gaussian(L, seed=1310 + L)
    a, b = orc.forward(x, L, s), orc.forward(np.conj(x), L, -s)
    assert rel_inf(b, (-1.0) ** (s + m) * np.conj(a[l * l + l - m])) < 1e-13
