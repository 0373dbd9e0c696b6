"""GPU adjoints and reverse-mode derivatives against the FP64 CPU oracle.

The adjoints are the conjugate transposes of the forward and inverse maps with
respect to the Euclidean inner products on the full grid and on the L^2
coefficients.  Checks: element-wise parity with the oracle's adjoints
(infinity-norm relative error <= 1e-12), the dot-product identity on the GPU,
the real-map variants, batching, and the gradient of the quadratic loss
sum_b ||forward(x_b) - y||^2 on 32 spin-2 maps at L = 256 against central
finite differences and against the oracle's adjoint.
"""
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


def real_fold(z, L):
    """Adjoint of the real-map coefficient expansion (m >= 0 read, negative m by
    f_{l,-m} = (-1)^m conj(f_lm)): y_{l,m} = z_{l,m} + (-1)^m conj(z_{l,-m}) for
    m > 0, y_{l,0} = z_{l,0}, y_{l,m<0} = 0."""
    y = np.zeros_like(z)
    for l in range(L):
        c = l * l + l
        y[c] = z[c]
        for m in range(1, l + 1):
            y[c + m] = z[c + m] + (-1) ** m * np.conj(z[c - m])
    return y


CASES = [(1, 0), (2, 1), (3, -2), (8, 0), (17, 3), (31, -3), (64, 2), (65, 0), (100, -1), (129, 7), (256, 2)]


@pytest.mark.parametrize("L,s", CASES)
def test_forward_adjoint_parity(orc, tc, mw, L, s):
    print("forward adjoint parity L=%d s=%d" % (L, s), flush=True)
    y = mwsynth.flm_gaussian(L, 0, seed=4000 + L + s)     # every entry, also l < |s|
    ref = orc.forward_adjoint(y, L, s)
    got = host(tc, mw.forward_adjoint(dev(tc, y), L, s))
    assert rel(got, ref) < TOL


@pytest.mark.parametrize("L,s", CASES)
def test_inverse_adjoint_parity(orc, tc, mw, L, s):
    print("inverse adjoint parity L=%d s=%d" % (L, s), flush=True)
    g = mwsynth.grid_gaussian(L, seed=5000 + L + s)
    ref = orc.inverse_adjoint(g, L, s)
    got = host(tc, mw.inverse_adjoint(dev(tc, g), L, s))
    assert rel(got, ref) < TOL


@pytest.mark.parametrize("L,s", [(64, 2), (257, -3)])
def test_dot_product_identities_on_gpu(tc, mw, L, s):
    print("dot products L=%d s=%d" % (L, s), flush=True)
    x = mwsynth.grid_gaussian(L, seed=6000 + L)
    y = mwsynth.zero_below_spin(mwsynth.flm_gaussian(L, 0, seed=6100 + L), L, s)
    Ax = host(tc, mw.forward(dev(tc, x), L, s))
    AHy = host(tc, mw.forward_adjoint(dev(tc, y), L, s))
    lhs, rhs = np.vdot(y, Ax), np.vdot(AHy, x)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(y) * np.linalg.norm(Ax)
    Yy = host(tc, mw.inverse(dev(tc, y), L, s))
    YHx = host(tc, mw.inverse_adjoint(dev(tc, x), L, s))
    lhs, rhs = np.vdot(x, Yy), np.vdot(YHx, y)
    assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(x) * np.linalg.norm(Yy)


@pytest.mark.parametrize("L", [1, 8, 65, 128])
def test_real_adjoints(orc, tc, mw, L):
    print("real adjoints L=%d" % L, flush=True)
    y = mwsynth.flm_gaussian(L, 0, seed=7000 + L)
    ref = np.real(orc.forward_adjoint(y, L, 0))
    got = host(tc, mw.forward_adjoint(dev(tc, y), L, 0, reality=1))
    assert got.dtype == np.float64
    assert rel(got, ref) < TOL
    g = mwsynth.grid_gaussian(L, seed=7100 + L, real=True)
    ref = real_fold(orc.inverse_adjoint(g.astype(np.complex128), L, 0), L)
    got = host(tc, mw.inverse_adjoint(dev(tc, g), L, 0, reality=1))
    assert rel(got, ref) < TOL
    # dot-product identity of the real inverse (reads m >= 0 only) and its adjoint
    f = mwsynth.flm_gaussian(L, 0, seed=7200 + L)
    Yf = host(tc, mw.inverse(dev(tc, f), L, 0, reality=1))
    assert abs(np.vdot(g, Yf).real - np.vdot(got, f).real) <= 1e-13 * np.linalg.norm(g) * np.linalg.norm(Yf)


@pytest.fixture(scope="module")
def grad_case(orc):
    w = mwsynth.workload_grad_l256()
    return w


def test_batched_adjoints_equal_single_calls(tc, mw, grad_case):
    L, s, x = grad_case["L"], grad_case["s"], grad_case["x"]
    n = x.shape[0]
    xs = [dev(tc, x[b]) for b in range(n)]
    outs = mw.inverse_adjoint_batch(xs, [L] * n, [s] * n)
    for b in (0, 7, n - 1):
        single = mw.inverse_adjoint(xs[b], L, s)
        assert np.array_equal(host(tc, outs[b]), host(tc, single))
    ys = [dev(tc, mwsynth.flm_gaussian(L, 0, seed=8000 + b)) for b in range(4)]
    outs = mw.forward_adjoint_batch(ys, [L] * 4, [s] * 4)
    for b in range(4):
        assert np.array_equal(host(tc, outs[b]), host(tc, mw.forward_adjoint(ys[b], L, s)))


def test_gradient_of_quadratic_loss(orc, tc, mw, grad_case):
    """32 spin-2 maps at L = 256, loss = sum_b ||forward(x_b) - y||^2.  The loss is
    quadratic in x, so a central difference with h = 1 is exact up to rounding
    (about eps |loss_b| / h); the gradient is checked on 64 random entries of Re
    and of Im per map against it (1e-7 of max |grad|), and in full against
    2 A^H (A x - y) from the oracle (1e-12)."""
    import paper_1110_6298_amd.autograd as ad
    L, s, x, y = grad_case["L"], grad_case["s"], grad_case["x"], grad_case["y"]
    n = x.shape[0]
    xt = dev(tc, x).requires_grad_(True)
    yt = dev(tc, y)
    loss = ((ad.forward(xt, L, s) - yt).abs() ** 2).sum()
    loss.backward()
    grad = host(tc, xt.grad)
    assert grad.shape == x.shape

    for b in (0, n - 1):
        ref = 2.0 * orc.forward_adjoint(orc.forward(x[b], L, s) - y, L, s)
        assert rel(grad[b], ref) < TOL

    rng = np.random.default_rng(9001)
    h = 1.0
    for b in range(n):
        xb = dev(tc, x[b])

        def loss_b(t):
            r = mw.forward(t, L, s) - yt
            return float((r.abs() ** 2).sum().item())

        gmax = np.abs(grad[b]).max()
        idx = rng.integers(0, L * (2 * L - 1), size=64)
        for part, unit in (("re", 1.0), ("im", 1j)):
            for k in idx:
                t, p = divmod(int(k), 2 * L - 1)
                xp = xb.clone()
                xp[t, p] += unit * h
                xm = xb.clone()
                xm[t, p] -= unit * h
                fd = (loss_b(xp) - loss_b(xm)) / (2 * h)
                an = grad[b, t, p].real if part == "re" else grad[b, t, p].imag
                assert abs(fd - an) <= 1e-7 * gmax, (b, part, t, p, fd, an)


def test_inverse_autograd_matches_adjoint(orc, tc, mw):
    import paper_1110_6298_amd.autograd as ad
    L, s = 48, -1
    f = mwsynth.flm_gaussian(L, s, seed=9100)
    g = mwsynth.grid_gaussian(L, seed=9200)
    ft = dev(tc, f).requires_grad_(True)
    loss = ((ad.inverse(ft, L, s) - dev(tc, g)).abs() ** 2).sum()
    loss.backward()
    ref = 2.0 * orc.inverse_adjoint(orc.inverse(f, L, s) - g, L, s)
    assert rel(host(tc, ft.grad), ref) < TOL
    # real scalar maps: gradient w.r.t. the m >= 0 coefficients the real inverse reads
    L = 33
    f = mwsynth.flm_gaussian(L, 0, seed=9300)
    g = mwsynth.grid_gaussian(L, seed=9400, real=True)
    ft = dev(tc, f).requires_grad_(True)
    loss = ((ad.inverse(ft, L, 0, reality=1) - dev(tc, g)) ** 2).sum()
    loss.backward()
    r = host(tc, mw.inverse(dev(tc, f), L, 0, reality=1)) - g
    ref = real_fold(2.0 * orc.inverse_adjoint(r.astype(np.complex128), L, 0), L)
    assert rel(host(tc, ft.grad), ref) < TOL
