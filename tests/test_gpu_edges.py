"""Edge cases of the HIP path: the smallest band-limits on every path, chunks
of more than 32 maps, maps of many classes in one call, extreme spins, and
errors raised before any launch."""
import numpy as np
import pytest

import mwsynth

pytestmark = pytest.mark.gpu


def rel(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


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


@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 1e-6)])
@pytest.mark.parametrize("L", [1, 2, 3])
def test_tiny_band_limits_all_paths(orc, tc, mw, L, precision, tol):
    for s in sorted({0, L - 1, -(L - 1)}):
        flm = mwsynth.flm_gaussian(L, s, seed=30000 + 10 * L + s)
        x = orc.inverse(flm, L, s)
        assert rel(host(tc, mw.inverse(dev(tc, flm), L, s, precision=precision)), x) < tol
        assert rel(host(tc, mw.forward(dev(tc, x), L, s, precision=precision)), orc.forward(x, L, s)) < tol
        y = mwsynth.flm_gaussian(L, 0, seed=30100 + L)
        assert rel(host(tc, mw.forward_adjoint(dev(tc, y), L, s, precision=precision)),
                   orc.forward_adjoint(y, L, s)) < tol
        assert rel(host(tc, mw.inverse_adjoint(dev(tc, x), L, s, precision=precision)),
                   orc.inverse_adjoint(x, L, s)) < tol
    # real scalar maps
    flm = mwsynth.make_real_symmetric(mwsynth.flm_gaussian(L, 0, seed=30200 + L), L)
    x = np.real(orc.inverse(flm, L, 0))
    assert rel(host(tc, mw.inverse(dev(tc, flm), L, 0, reality=1, precision=precision)), x) < tol
    assert rel(host(tc, mw.forward(dev(tc, x), L, 0, reality=1, precision=precision)),
               orc.forward(x.astype(np.complex128), L, 0)) < tol


@pytest.mark.parametrize("precision", [0, 1])
def test_more_maps_than_one_chunk(tc, mw, precision):
    """70 maps of one class run as three chunks (at most 32 maps per launch);
    every map equals its own single call (the result does not depend on the
    batch a map runs in)."""
    L, s, n = 24, 1, 70
    flms = [mwsynth.flm_gaussian(L, s, seed=31000 + i) for i in range(n)]
    outs = mw.inverse_batch([dev(tc, f) for f in flms], [L] * n, [s] * n, precision=precision)
    for i in (0, 31, 32, 63, 64, 69):
        single = host(tc, mw.inverse(dev(tc, flms[i]), L, s, precision=precision))
        assert np.array_equal(host(tc, outs[i]), single), i


def test_many_classes_in_one_call(orc, tc, mw):
    """Maps of 12 (L, spin, reality) classes interleaved in one call."""
    specs = []
    for i in range(24):
        L = (8, 13, 21)[i % 3]
        s = (0, 2, -1, 0)[i % 4]
        r = 1 if (s == 0 and i % 5 == 0) else 0
        specs.append((L, s, r))
    flms = []
    for i, (L, s, r) in enumerate(specs):
        f = mwsynth.flm_gaussian(L, s, seed=32000 + i)
        flms.append(mwsynth.make_real_symmetric(f, L) if r else f)
    Ls, ss, rs = zip(*specs)
    maps = mw.inverse_batch([dev(tc, f) for f in flms], Ls, ss, rs)
    for i, (L, s, r) in enumerate(specs):
        ref = orc.inverse(flms[i], L, s)
        assert rel(host(tc, maps[i]), np.real(ref) if r else ref) < 1e-12, i


def test_extreme_spin_at_moderate_l(orc, tc, mw):
    L = 40
    for s in (L - 1, -(L - 1), L // 2):
        flm = mwsynth.flm_gaussian(L, s, seed=33000 + s)
        x = orc.inverse(flm, L, s)
        assert rel(host(tc, mw.inverse(dev(tc, flm), L, s)), x) < 1e-12
        assert rel(host(tc, mw.forward(dev(tc, x), L, s)), flm) < 1e-12


def test_binding_rejects_bad_tensors(tc, mw):
    L = 8
    good = tc.zeros(L * L, dtype=tc.complex128, device="cuda")
    with pytest.raises(ValueError):
        mw.inverse(tc.zeros(L * L + 1, dtype=tc.complex128, device="cuda"), L)
    with pytest.raises(TypeError):
        mw.inverse(tc.zeros(L * L, dtype=tc.complex64, device="cuda"), L)
    with pytest.raises(TypeError):
        mw.inverse(tc.zeros(L * L, dtype=tc.complex128), L)           # host tensor
    with pytest.raises(TypeError):
        mw.forward(tc.zeros((L, 2 * L - 1), dtype=tc.complex128, device="cuda"), L, reality=1)
    with pytest.raises(mw.MWError):
        mw.inverse(good, L, 8)                                          # |s| >= L
    with pytest.raises(mw.MWError):
        mw.inverse(good, L, 2, reality=1)                               # reality needs s = 0
