"""Compact storage (Sec. IV-C: N_MW = (L-1)(2L-1)+1 samples, the south pole
once) on the GPU against the oracle's compact transforms, their adjoint
identities, and the round trip at L = 4096."""
import numpy as np
import pytest

import mwsynth

pytestmark = pytest.mark.gpu

TOL = 1e-12


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


def nmw(L):
    return (L - 1) * (2 * L - 1) + 1


@pytest.mark.parametrize("L,s", [(1, 0), (2, 1), (9, -2), (64, 0), (129, 3), (300, 2)])
@pytest.mark.parametrize("precision,tol", [("fp64", TOL), ("fp32c", 1e-6)])
def test_compact_transforms_match_oracle(orc, tc, mw, L, s, precision, tol):
    print("compact L=%d s=%d %s" % (L, s, precision), flush=True)
    flm = mwsynth.flm_gaussian(L, s, seed=20000 + L, decay=1.0)
    got = host(tc, mw.inverse_compact(dev(tc, flm), L, s, precision=precision))
    assert got.shape == (nmw(L),)
    assert rel(got, orc.inverse_compact(flm, L, s)) < tol
    rng = np.random.default_rng(20100 + L)
    xc = rng.standard_normal(nmw(L)) + 1j * rng.standard_normal(nmw(L))
    got = host(tc, mw.forward_compact(dev(tc, xc), L, s, precision=precision))
    assert rel(got, orc.forward_compact(xc, L, s)) < tol


@pytest.mark.parametrize("L,s", [(2, 1), (9, -2), (64, 0), (300, 2)])
def test_compact_adjoints_match_oracle(orc, tc, mw, L, s):
    print("compact adjoints L=%d s=%d" % (L, s), flush=True)
    y = mwsynth.flm_gaussian(L, 0, seed=20200 + L)
    got = host(tc, mw.compact_batch("forward_adjoint", [dev(tc, y)], [L], [s])[0])
    assert rel(got, orc.forward_adjoint_compact(y, L, s)) < TOL
    rng = np.random.default_rng(20300 + L)
    g = rng.standard_normal(nmw(L)) + 1j * rng.standard_normal(nmw(L))
    got = host(tc, mw.compact_batch("inverse_adjoint", [dev(tc, g)], [L], [s])[0])
    assert rel(got, orc.inverse_adjoint_compact(g, L, s)) < TOL


@pytest.mark.parametrize("L", [7, 130])
def test_compact_real_maps(orc, tc, mw, L):
    print("compact real L=%d" % L, flush=True)
    flm = mwsynth.make_real_symmetric(mwsynth.flm_gaussian(L, 0, seed=20400 + L), L)
    got = host(tc, mw.inverse_compact(dev(tc, flm), L, 0, reality=1))
    assert got.dtype == np.float64
    assert rel(got, orc.inverse_compact(flm, L, 0).real) < TOL
    xc = np.random.default_rng(20500 + L).standard_normal(nmw(L))
    got = host(tc, mw.forward_compact(dev(tc, xc), L, 0, reality=1))
    assert rel(got, orc.forward_compact(xc, L, 0)) < TOL
    y = mwsynth.flm_gaussian(L, 0, seed=20600 + L)
    got = host(tc, mw.compact_batch("forward_adjoint", [dev(tc, y)], [L], [0], [1])[0])
    assert rel(got, orc.forward_adjoint_compact(y, L, 0).real) < TOL


def test_compact_batch_of_mixed_maps(tc, mw):
    specs = [(16, 0, 0), (40, 2, 0), (33, 0, 1), (40, 2, 0)]
    flms = []
    for i, (L, s, r) in enumerate(specs):
        f = mwsynth.flm_gaussian(L, s, seed=20700 + i)
        flms.append(dev(tc, mwsynth.make_real_symmetric(f, L) if r else f))
    Ls, ss, rs = [a for a, _, _ in specs], [b for _, b, _ in specs], [c for _, _, c in specs]
    maps = mw.compact_batch("inverse", flms, Ls, ss, rs)
    back = mw.compact_batch("forward", maps, Ls, ss, rs)
    for i, (L, s, r) in enumerate(specs):
        assert np.array_equal(host(tc, maps[i]), host(tc, mw.inverse_compact(flms[i], L, s, r)))
        assert rel(host(tc, back[i]), host(tc, flms[i])) < TOL


@pytest.mark.parametrize("L,s,real", [(4096, 2, 0), (4096, 0, 1)])
def test_compact_round_trip_full_size(tc, mw, L, s, real):
    """The sampling theorem on N_MW samples at the largest band-limit."""
    print("compact round trip L=%d s=%d real=%d" % (L, s, real), flush=True)
    flm = mwsynth.flm_cl_real(L, seed=20800) if real else mwsynth.flm_gaussian(L, s, seed=20800, decay=1.0)
    xc = mw.inverse_compact(dev(tc, flm), L, s, reality=real)
    back = host(tc, mw.forward_compact(xc, L, s, reality=real))
    assert rel(back, flm) < TOL
