"""The explicit quadrature (Sec. IV-F) on the GPU against the oracle: the
weights, integrals of seeded maps on the rule's grid and on the transform grid,
batches, and exactness for band-limited maps at full size."""
import math

import numpy as np
import pytest

import mwsynth

pytestmark = pytest.mark.gpu

TOL = 1e-12


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


def dev(tc, x):
    return tc.from_numpy(np.ascontiguousarray(x)).cuda()


def host(tc, t):
    tc.cuda.synchronize()
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("L,s", [(1, 0), (2, 1), (7, -2), (64, 0), (301, 3), (4096, 2)])
def test_weights_match_oracle(orc, tc, mw, L, s):
    print("quadrature weights L=%d s=%d" % (L, s), flush=True)
    got = host(tc, mw.quadrature_weights(L, s))
    ref = orc.quad_weights(L, s).real
    assert np.abs(got - ref).max() <= TOL * np.abs(ref).max()


def _map(L, nphi, real, seed):
    rng = np.random.default_rng(seed)
    if real:
        return rng.standard_normal((L, nphi))
    z = rng.standard_normal((L, nphi, 2))
    return z[..., 0] + 1j * z[..., 1]


def _scale(orc, f, L, s):
    # sum_t |q_t| sum_p |f(t, p)| L/nphi: the size of the terms of the sum
    q = np.abs(orc.quad_weights(L, s))
    return float((q * np.abs(f).sum(axis=1)).sum() * L / f.shape[1])


@pytest.mark.parametrize("L,s,real", [(1, 0, 0), (5, 2, 0), (33, 0, 1), (128, -1, 0), (257, 0, 1)])
@pytest.mark.parametrize("grid", ["quadrature", "transform"])
def test_integrals_match_oracle(orc, tc, mw, L, s, real, grid):
    print("integrate L=%d s=%d real=%d %s grid" % (L, s, real, grid), flush=True)
    nphi = L if grid == "quadrature" else 2 * L - 1
    f = _map(L, nphi, real, seed=19000 + L)
    got = complex(host(tc, mw.integrate(dev(tc, f), L, s, reality=real))[0])
    ref = orc.integrate(f.astype(np.complex128), L, s)
    assert abs(got - ref) <= TOL * _scale(orc, f, L, s)


def test_batch_equals_single_calls(tc, mw):
    specs = [(16, 0, 0), (40, 2, 0), (33, 0, 1), (64, -1, 0), (40, 2, 0)]
    maps = [dev(tc, _map(L, 2 * L - 1, r, seed=19500 + i)) for i, (L, s, r) in enumerate(specs)]
    outs = mw.integrate_batch(maps, [a for a, _, _ in specs], [b for _, b, _ in specs], [c for _, _, c in specs])
    for i, (L, s, r) in enumerate(specs):
        single = host(tc, mw.integrate(maps[i], L, s, reality=r))
        assert np.array_equal(host(tc, outs[i]), single), i


@pytest.mark.parametrize("L,real", [(512, 0), (4096, 1)])
def test_exact_for_band_limited_maps(tc, mw, L, real):
    """A band-limited scalar map (the GPU inverse of seeded coefficients):
    int dOmega f = sqrt(4 pi) f_00 (int Y_lm dOmega = sqrt(4 pi) delta_l0 delta_m0)."""
    print("integrate band-limited L=%d real=%d" % (L, real), flush=True)
    flm = mwsynth.flm_cl_real(L, seed=19900 + L) if real else mwsynth.flm_gaussian(L, 0, seed=19900 + L)
    x = mw.inverse(dev(tc, flm), L, 0, reality=real)
    got = complex(host(tc, mw.integrate(x, L, 0, reality=real))[0])
    ref = math.sqrt(4 * math.pi) * flm[0]
    # the map carries the inverse's rounding (<= 1e-12 of its largest sample),
    # which integrates to at most 4 pi times that
    xmax = float(tc.abs(x).max().item())
    print("  I = %r, sqrt(4 pi) f_00 = %r, |diff| %.3e" % (got, ref, abs(got - ref)), flush=True)
    assert abs(got - ref) <= 1e-12 * 4 * math.pi * xmax
