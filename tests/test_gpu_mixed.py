"""GPU mixed-precision path (MW_FP32C) against the FP64 CPU oracle.

The O(L^3) contraction rounds Delta*Delta and the Fourier data to FP32 and
accumulates on the matrix cores; everything else stays FP64.  Stated bound:
infinity-norm relative error <= 1e-6 against the oracle (FP32 rounding of the
two factors is 2^-24 each; the sums over up to L terms with random signs and
segment-wise FP32 accumulation stay two orders of magnitude below the bound
at L <= 512, measured ~1e-7).
"""
import numpy as np
import pytest

import mwsynth

pytestmark = pytest.mark.gpu

TOL = 1e-6
FP32C = 1


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


CASES = [(1, 0), (2, 1), (3, -2), (8, 0), (17, 3), (31, -3), (64, 2), (65, 0), (100, -1), (129, 7), (257, -2)]


@pytest.mark.parametrize("L,s", CASES)
def test_mixed_inverse_and_forward(orc, tc, mw, L, s):
    print("mixed L=%d s=%d" % (L, s), flush=True)
    flm = mwsynth.flm_gaussian(L, s, seed=11000 + L + s)
    xref = orc.inverse(flm, L, s)
    x = host(tc, mw.inverse(dev(tc, flm), L, s, precision=FP32C))
    assert rel(x, xref) < TOL
    g = xref + 0.5 * mwsynth.grid_gaussian(L, seed=11100 + L)
    fref = orc.forward(g, L, s)
    f = host(tc, mw.forward(dev(tc, g), L, s, precision=FP32C))
    assert rel(f, fref) < TOL


@pytest.mark.parametrize("L,s", [(8, 2), (65, -1), (128, 2)])
def test_mixed_adjoints(orc, tc, mw, L, s):
    print("mixed adjoints L=%d s=%d" % (L, s), flush=True)
    y = mwsynth.flm_gaussian(L, 0, seed=12000 + L)
    ref = orc.forward_adjoint(y, L, s)
    assert rel(host(tc, mw.forward_adjoint(dev(tc, y), L, s, precision=FP32C)), ref) < TOL
    g = mwsynth.grid_gaussian(L, seed=12100 + L)
    ref = orc.inverse_adjoint(g, L, s)
    assert rel(host(tc, mw.inverse_adjoint(dev(tc, g), L, s, precision=FP32C)), ref) < TOL


def test_mixed_config_spin2_l512(orc, tc, mw):
    """L = 512, s = 2, f_lm ~ (N + iN)/(l+1): the mixed path against the oracle,
    and the FP64 path's error stated beside it."""
    w = mwsynth.workload_spin2_l512()
    L, s, flm = w["L"], w["s"], w["flm"]
    xref = orc.inverse(flm, L, s)
    fref = orc.forward(xref, L, s)
    x32 = host(tc, mw.inverse(dev(tc, flm), L, s, precision=FP32C))
    f32 = host(tc, mw.forward(dev(tc, xref), L, s, precision=FP32C))
    e_inv, e_fwd = rel(x32, xref), rel(f32, fref)
    print("FP32C L=512 s=2: inverse %.3e forward %.3e" % (e_inv, e_fwd), flush=True)
    assert e_inv < TOL and e_fwd < TOL
    # a mixed round trip returns the coefficients to the same bound
    back = host(tc, mw.forward(mw.inverse(dev(tc, flm), L, s, precision=FP32C), L, s, precision=FP32C))
    assert rel(back, flm) < 2 * TOL


def test_mixed_real_maps(orc, tc, mw):
    L = 96
    flm = mwsynth.make_real_symmetric(mwsynth.flm_gaussian(L, 0, seed=13000), L)
    xref = np.real(orc.inverse(flm, L, 0))
    x = host(tc, mw.inverse(dev(tc, flm), L, 0, reality=1, precision=FP32C))
    assert x.dtype == np.float64 and rel(x, xref) < TOL
    # a lone real map's inverse contraction is the FP64 one in either precision
    assert np.array_equal(x, host(tc, mw.inverse(dev(tc, flm), L, 0, reality=1)))
    f = host(tc, mw.forward(dev(tc, xref), L, 0, reality=1, precision=FP32C))
    assert rel(f, orc.forward(xref.astype(np.complex128), L, 0)) < TOL
    # two real maps run the mixed inverse kernel (a group shares the chains)
    flm2 = mwsynth.make_real_symmetric(mwsynth.flm_gaussian(L, 0, seed=13001), L)
    xs = mw.inverse_batch([dev(tc, flm), dev(tc, flm2)], [L, L], [0, 0], [1, 1], precision=FP32C)
    assert rel(host(tc, xs[0]), xref) < TOL
    assert rel(host(tc, xs[1]), np.real(orc.inverse(flm2, L, 0))) < TOL


def test_mixed_batch_of_uneven_maps(orc, tc, mw):
    """Maps of several band-limits and spins in one call: maps of one spin share
    the chains in groups; each map matches the oracle and its own single call."""
    specs = [(64, 2, 0), (48, 2, 0), (33, 2, 0), (64, 0, 1), (40, 0, 0), (64, 0, 1), (17, -1, 0), (64, 2, 0),
             (50, 0, 1)]
    Ls = [a for a, _, _ in specs]
    ss = [b for _, b, _ in specs]
    rs = [c for _, _, c in specs]
    flms = []
    for i, (L, s, r) in enumerate(specs):
        f = mwsynth.flm_gaussian(L, s, seed=14000 + i)
        if r:
            f = mwsynth.make_real_symmetric(f, L)
        flms.append(f)
    mw.prepare(Ls, ss, rs, precision=FP32C)
    maps = mw.inverse_batch([dev(tc, f) for f in flms], Ls, ss, rs, precision=FP32C)
    maps_h = [host(tc, m) for m in maps]
    refs = []
    for i, (L, s, r) in enumerate(specs):
        ref = orc.inverse(flms[i], L, s)
        if r:
            ref = np.ascontiguousarray(np.real(ref))
        refs.append(ref)
        assert rel(maps_h[i], ref) < TOL, i
        single = host(tc, mw.inverse(dev(tc, flms[i]), L, s, r, precision=FP32C))
        assert rel(maps_h[i], single) < TOL, i
    # the forward of the oracle's maps (inputs independent of the GPU path)
    back = mw.forward_batch([dev(tc, m) for m in refs], Ls, ss, rs, precision=FP32C)
    for i, (L, s, r) in enumerate(specs):
        assert rel(host(tc, back[i]), orc.forward(refs[i].astype(np.complex128), L, s)) < TOL, i


def test_mixed_batch_equal_band_limits_is_exact(tc, mw):
    """Maps of one band-limit and spin are bitwise the same in any group size:
    each keeps its own accumulators over the same shared chains."""
    L, s, n = 80, 2, 5
    flms = [mwsynth.flm_gaussian(L, s, seed=15000 + i) for i in range(n)]
    outs = mw.inverse_batch([dev(tc, f) for f in flms], [L] * n, [s] * n, precision=FP32C)
    for i in range(n):
        single = mw.inverse(dev(tc, flms[i]), L, s, precision=FP32C)
        assert np.array_equal(host(tc, outs[i]), host(tc, single))


def test_mixed_large_l_sampled(orc, tc, mw):
    """L = 2048 real grid in mixed precision: sampled coefficients of the
    forward against the oracle's per-order forward."""
    L = 2048
    x = mwsynth.grid_gaussian(L, seed=17004, real=True)      # seeded input, not from the GPU path
    f = host(tc, mw.forward(dev(tc, x), L, 0, reality=1, precision=FP32C))
    orders = [0, 1, 700, 1500, 2047]
    ref = orc.forward_orders(x.astype(np.complex128), L, 0, orders)
    got, want = [], []
    for k, m in enumerate(orders):
        ls = np.arange(m, L)
        got.append(f[ls * ls + ls + m])
        want.append(ref[k, ls])
    got, want = np.concatenate(got), np.concatenate(want)
    print("FP32C L=2048 real, sampled orders: %.3e" % rel(got, want), flush=True)
    assert rel(got, want) < TOL


def _rows(f, L, orders):
    """[orders][L] rows of an L*L coefficient vector (0 where |m| > l)."""
    out = np.zeros((len(orders), L), dtype=np.complex128)
    for k, m in enumerate(orders):
        ls = np.arange(abs(m), L)
        out[k, ls] = f[ls * ls + ls + m]
    return out


def _ring_orders(x, L, orders):
    """phi-Fourier coefficients F_m(theta_t) of a map's rings: [orders][t]."""
    spec = np.fft.fft(np.asarray(x, dtype=np.complex128), axis=1) / (2 * L - 1)
    return spec[:, np.array(orders) % (2 * L - 1)].T


@pytest.mark.parametrize("L,s,real", [(512, 2, 0), (256, 2, 0), (256, 0, 1)])
def test_mixed_groups_at_batch_sizes(orc, tc, mw, L, s, real):
    """Four maps of one class in one call (one group of four sharing the chains,
    several chain segments restarted from checkpoint planes at these L): two of
    them against the oracle on sampled orders, all four bitwise against single
    calls (per-map arithmetic does not depend on the group; a real map's inverse
    goes in with a copy of itself, since alone it takes the FP64 contraction)."""
    print("mixed groups L=%d s=%d real=%d" % (L, s, real), flush=True)
    n = 4
    flm = []
    for i in range(n):
        f = mwsynth.flm_gaussian(L, s, seed=16000 + 10 * L + i, decay=1.0)
        flm.append(mwsynth.make_real_symmetric(f, L) if real else f)
    maps = mw.inverse_batch([dev(tc, f) for f in flm], [L] * n, [s] * n, [real] * n, precision=FP32C)
    maps_h = [host(tc, t) for t in maps]
    orders = [0, 1, 7, L // 2, L - 1] + ([] if real else [-1, -(L // 3), -(L - 1)])
    for i in range(n):
        if real:
            pair = mw.inverse_batch([dev(tc, flm[i])] * 2, [L] * 2, [s] * 2, [real] * 2, precision=FP32C)
            single = host(tc, pair[0])
        else:
            single = host(tc, mw.inverse(dev(tc, flm[i]), L, s, real, precision=FP32C))
        assert np.array_equal(maps_h[i], single), i
    for i in range(2):
        e = rel(_ring_orders(maps_h[i], L, orders), orc.inverse_orders(flm[i], L, s, orders))
        print("  FP32C inverse, map %d: %.3e" % (i, e), flush=True)
        assert e < TOL
    grids = [mwsynth.grid_gaussian(L, seed=16500 + i, real=bool(real)) for i in range(n)]
    fw = mw.forward_batch([dev(tc, g) for g in grids], [L] * n, [s] * n, [real] * n, precision=FP32C)
    fw_h = [host(tc, t) for t in fw]
    for i in range(n):
        single = host(tc, mw.forward(dev(tc, grids[i]), L, s, real, precision=FP32C))
        assert np.array_equal(fw_h[i], single), i
    for i in range(2):
        ref = orc.forward_orders(grids[i].astype(np.complex128), L, s, orders)
        e = rel(_rows(fw_h[i], L, orders), ref)
        print("  FP32C forward, map %d: %.3e" % (i, e), flush=True)
        assert e < TOL


def test_mixed_inverse_large_l_sampled(orc, tc, mw):
    """L = 2048 real scalar map (C_l = (l+1)^-2): the exponent-extended mixed
    inverse on sampled orders of its rings' phi-spectra against the oracle, and
    the per-degree error of the mixed round trip against the input. The map
    goes in twice in one call, so that the mixed inverse kernel runs (a lone
    real map takes the FP64 one)."""
    w = mwsynth.workload_real_l2048()
    L, flm = w["L"], w["flm"]
    xs = mw.inverse_batch([dev(tc, flm), dev(tc, flm)], [L, L], [0, 0], [1, 1], precision=FP32C)
    orders = [0, 1, 2, 700, 1024, 1500, 2046, 2047]
    ref = orc.inverse_orders(flm, L, 0, orders)
    for k in range(2):
        e = rel(_ring_orders(host(tc, xs[k]), L, orders), ref)
        print("FP32C L=2048 real inverse (map %d of a pair), sampled orders: %.3e" % (k, e), flush=True)
        assert e < TOL
    x = host(tc, xs[0])
    del xs
    back = host(tc, mw.forward(dev(tc, x), L, 0, reality=1, precision=FP32C))
    e_rt = rel(back, flm)
    e_deg = rel_per_degree(back, flm, L)
    print("FP32C L=2048 real round trip: %.3e, per degree %.3e" % (e_rt, e_deg), flush=True)
    assert e_rt < 2 * TOL
    assert e_deg < PER_DEGREE_TOL


def rel_per_degree(got, ref, L):
    """max over l of max_m |got - ref| / max_m |ref| (the per-degree relative error)."""
    worst = 0.0
    for l in range(L):
        sl = slice(l * l, (l + 1) * (l + 1))
        den = np.abs(ref[sl]).max()
        if den > 0:
            worst = max(worst, float(np.abs(got[sl] - ref[sl]).max() / den))
    return worst


# The per-degree error of the mixed path: FP32 rounding of both factors of each
# product (2^-24 relative each) over sums of up to L terms, relative to the
# largest coefficient of that degree; for spectra that fall by three orders of
# magnitude across l (C_l = (l+1)^-2 at L = 2048), the terms of a high degree
# are dominated by the low-degree content of the data, so the bound is wider
# than the global one.
PER_DEGREE_TOL = 1e-3


def test_mixed_groups_across_spins(orc, tc, mw):
    """One mixed-precision call with maps of several spins at one band-limit:
    groups of four share the order chains with two spin rows ({0, 1} and {2, 3}
    here).  Every map against the oracle; the forward also bitwise against
    single calls (its work list does not depend on the spin)."""
    L = 128
    spins = [0, 2, -2, 3, 0, 1, -1, 2]
    n = len(spins)
    flm = [mwsynth.flm_gaussian(L, s, seed=21000 + i, decay=1.0) for i, s in enumerate(spins)]
    mw.prepare([L] * n, spins, precision=FP32C)
    maps = [host(tc, t) for t in mw.inverse_batch([dev(tc, f) for f in flm], [L] * n, spins, precision=FP32C)]
    grids = [mwsynth.grid_gaussian(L, seed=21100 + i) for i in range(n)]
    fw = [host(tc, t) for t in mw.forward_batch([dev(tc, g) for g in grids], [L] * n, spins, precision=FP32C)]
    for i, s in enumerate(spins):
        print("  map %d spin %d" % (i, s), flush=True)
        assert rel(maps[i], orc.inverse(flm[i], L, s)) < TOL, i
        assert rel(fw[i], orc.forward(grids[i], L, s)) < TOL, i
        single = host(tc, mw.forward(dev(tc, grids[i]), L, s, precision=FP32C))
        assert np.array_equal(fw[i], single), i


def test_mixed_group_across_band_limits(orc, tc, mw):
    """Maps of L = 512, 256 and 128 (one spin) in one mixed-precision call form one
    group: its Wigner order chains run once, to L = 512, and each map masks the
    degrees l >= L_b (one contraction launch per direction).  Every map against
    the oracle (sampled orders at L = 512) and against its own single call."""
    specs = [(128, 2, 0), (512, 2, 0), (256, 2, 0)]
    Ls = [a for a, _, _ in specs]
    ss = [b for _, b, _ in specs]
    flm = [mwsynth.flm_gaussian(L, s, seed=22000 + L, decay=1.0) for L, s, _ in specs]
    grids = [mwsynth.grid_gaussian(L, seed=22100 + L) for L, _, _ in specs]
    # no mw_prepare: an untuned shape takes the largest group (four maps here)
    assert mw.tuned_group(512, 0, 3) in (0, 4)
    mw.profile_enable(True)
    maps = [host(tc, t) for t in mw.inverse_batch([dev(tc, f) for f in flm], Ls, ss, precision=FP32C)]
    fw = [host(tc, t) for t in mw.forward_batch([dev(tc, g) for g in grids], Ls, ss, precision=FP32C)]
    prof = mw.profile_read()
    mw.profile_enable(False)
    print("  launches: %s" % {k: v[1] for k, v in prof.items()}, flush=True)
    assert prof["contract_inverse"][1] == 1 and prof["contract_forward"][1] == 1
    for i, (L, s, _) in enumerate(specs):
        print("  map L=%d" % L, flush=True)
        if L == 512:
            orders = [0, 1, 2, 7, -1, -3, 255, -170, 510, 511, -511]
            e_inv = rel(_ring_orders(maps[i], L, orders), orc.inverse_orders(flm[i], L, s, orders))
            e_fwd = rel(_rows(fw[i], L, orders), orc.forward_orders(grids[i].astype(np.complex128), L, s, orders))
        else:
            e_inv = rel(maps[i], orc.inverse(flm[i], L, s))
            e_fwd = rel(fw[i], orc.forward(grids[i], L, s))
        print("    inverse %.3e forward %.3e" % (e_inv, e_fwd), flush=True)
        assert e_inv < TOL and e_fwd < TOL
        assert rel(maps[i], host(tc, mw.inverse(dev(tc, flm[i]), L, s, precision=FP32C))) < TOL
        assert rel(fw[i], host(tc, mw.forward(dev(tc, grids[i]), L, s, precision=FP32C))) < TOL
