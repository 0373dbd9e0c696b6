"""The spin -s coefficients of the conjugate map (Sec. IV-G) on the GPU:
mw_spin_flip against its definition, in place, and against a second transform."""
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


def _flip(f, L, s):
    l, m = mwsynth.lm_arrays(L)
    out = (-1.0) ** (s + m) * np.conj(f[l * l + l - m])
    out[l < abs(s)] = 0
    return out


@pytest.mark.parametrize("L,s", [(1, 0), (2, 1), (33, -2), (512, 2), (4096, 3)])
def test_spin_flip_is_exact(tc, mw, L, s):
    f = mwsynth.flm_gaussian(L, 0, seed=22000 + L)
    got = host(tc, mw.spin_flip(dev(tc, f), L, s))
    assert np.array_equal(got, _flip(f, L, s))
    t = dev(tc, f)
    mw.spin_flip(t, L, s, out=t)   # in place
    assert np.array_equal(host(tc, t), _flip(f, L, s))


@pytest.mark.parametrize("L,s", [(64, 2), (257, -1)])
def test_flip_equals_transform_of_conjugate(orc, tc, mw, L, s):
    """The spin -s forward of conj(x) equals the flip of the spin-s forward of x
    (to the FP64 tolerance), and the oracle agrees."""
    x = mwsynth.grid_gaussian(L, seed=22100 + L)
    a = mw.forward(dev(tc, x), L, s)
    b = host(tc, mw.forward(dev(tc, np.conj(x)), L, -s))
    fl = host(tc, mw.spin_flip(a, L, s))
    assert rel(fl, b) < 1e-12
    assert rel(fl, orc.forward(np.conj(x), L, -s)) < 1e-12
