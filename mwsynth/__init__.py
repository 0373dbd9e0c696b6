"""Seeded synthetic inputs for the MW transform workloads.

This module only draws random numbers and lays them out; it contains none of
the transform's arithmetic, so both the CPU oracle and the GPU path can be fed
from it.  Coefficients are stored at ``l*l + l + m`` (0 <= l < L, |m| <= l),
maps as ``[t][p]`` arrays of shape (L, 2L-1).

Draw order is fixed: index l*l+l+m ascending, real part before imaginary part
(numpy ``default_rng``).
"""
from __future__ import annotations

import numpy as np


def n_coeffs(L: int) -> int:
    return L * L


def lm_arrays(L: int):
    """(l, m) of every coefficient slot in index order."""
    l = np.repeat(np.arange(L), 2 * np.arange(L) + 1)
    m = np.arange(L * L) - l * l - l
    return l, m


def complex_normal(rng, n):
    z = rng.standard_normal((n, 2))
    return z[:, 0] + 1j * z[:, 1]


def zero_below_spin(flm: np.ndarray, L: int, s: int) -> np.ndarray:
    """Coefficients with l < |s| do not exist for spin s; they are set to 0."""
    l, _ = lm_arrays(L)
    out = flm.copy()
    out[l < abs(s)] = 0
    return out


def make_real_symmetric(flm: np.ndarray, L: int) -> np.ndarray:
    """Impose f_{l,-m} = (-1)^m conj(f_lm) (the reality condition of a scalar
    map, Sec. III-A): m > 0 entries are kept, m < 0 entries overwritten, m = 0
    made real."""
    l, m = lm_arrays(L)
    out = flm.copy()
    pos = m > 0
    out[l[pos] * l[pos] + l[pos] - m[pos]] = ((-1.0) ** m[pos]) * np.conj(flm[pos])
    zero = m == 0
    out[zero] = out[zero].real
    return out


def flm_gaussian(L: int, s: int, seed: int, decay: float = 0.0) -> np.ndarray:
    """Re, Im i.i.d. N(0,1), times (l+1)^-decay; zero for l < |s|."""
    rng = np.random.default_rng(seed)
    l, _ = lm_arrays(L)
    flm = complex_normal(rng, L * L) * (l + 1.0) ** (-decay)
    return zero_below_spin(flm, L, s)


def flm_uniform(L: int, s: int, seed: int) -> np.ndarray:
    """Re, Im i.i.d. uniform on [-1, 1] (the paper's test signals, Sec. V-D)."""
    rng = np.random.default_rng(seed)
    z = rng.uniform(-1.0, 1.0, size=(L * L, 2))
    return zero_below_spin(z[:, 0] + 1j * z[:, 1], L, s)


def flm_cl_real(L: int, seed: int, power: float = 2.0) -> np.ndarray:
    """Real scalar map with power spectrum C_l = (l+1)^-power:
    f_l0 = sqrt(C_l) N(0,1); f_lm = sqrt(C_l/2) (N + iN) for m > 0;
    f_{l,-m} = (-1)^m conj(f_lm)."""
    rng = np.random.default_rng(seed)
    l, m = lm_arrays(L)
    cl = (l + 1.0) ** (-power)
    z = rng.standard_normal((L * L, 2))
    flm = np.where(m == 0, np.sqrt(cl) * z[:, 0], np.sqrt(cl / 2) * (z[:, 0] + 1j * z[:, 1]))
    return make_real_symmetric(flm.astype(np.complex128), L)


def grid_gaussian(L: int, seed: int, real: bool = False) -> np.ndarray:
    """A map of i.i.d. N(0,1) samples (complex unless real) on the L x (2L-1) grid.
    Not band-limited."""
    rng = np.random.default_rng(seed)
    if real:
        return rng.standard_normal((L, 2 * L - 1))
    z = rng.standard_normal((L, 2 * L - 1, 2))
    return z[..., 0] + 1j * z[..., 1]


# ---------------------------------------------------------------------------
# The five workloads.  Each returns plain numpy data; synthesising maps from
# coefficients (where a workload asks for a band-limited map) is done by the
# caller with the transform under test or the oracle.
# ---------------------------------------------------------------------------
SEEDS = {"scalar_l64": 1001, "spin2_l512": 1002, "batch_mixed": 1003,
         "real_l2048": 1004, "grad_l256": 1005}


def workload_scalar_l64():
    """L=64, s=0, one complex map; f_lm Re/Im i.i.d. N(0,1)."""
    L, s = 64, 0
    return dict(L=L, s=s, flm=flm_gaussian(L, s, SEEDS["scalar_l64"]))


def workload_spin2_l512(L: int = 512):
    """L=512, s=2, one complex map; f_lm = (N + iN)/(l+1) for l >= 2."""
    s = 2
    return dict(L=L, s=s, flm=flm_gaussian(L, s, SEEDS["spin2_l512"], decay=1.0))


def workload_batch_mixed(n_maps: int = 256, Ls=(128, 256, 512), spins=(0, 2), seed=None):
    """n_maps maps; L uniform on Ls, spin uniform on spins; exactly half of them
    'real' by a seeded permutation: f_lm ~ N(0,1)/(l+1), with the conjugate
    symmetry f_{l,-m} = (-1)^m conj(f_lm) imposed on the 'real' ones."""
    rng = np.random.default_rng(SEEDS["batch_mixed"] if seed is None else seed)
    Lb = rng.choice(np.asarray(Ls), size=n_maps)
    sb = rng.choice(np.asarray(spins), size=n_maps)
    real = np.zeros(n_maps, dtype=bool)
    real[rng.permutation(n_maps)[: n_maps // 2]] = True
    maps = []
    for b in range(n_maps):
        L, s = int(Lb[b]), int(sb[b])
        l, _ = lm_arrays(L)
        flm = complex_normal(rng, L * L) / (l + 1.0)
        if real[b]:
            flm = make_real_symmetric(flm, L)
        maps.append(dict(L=L, s=s, real=bool(real[b]), flm=zero_below_spin(flm, L, s)))
    return maps


def workload_real_l2048(L: int = 2048):
    """L=2048, s=0, one real map with C_l = (l+1)^-2."""
    return dict(L=L, s=0, flm=flm_cl_real(L, SEEDS["real_l2048"]))


def workload_grad_l256(n_maps: int = 32, L: int = 256):
    """n_maps spin-2 maps at L=256: x complex N(0,1) on the grid (not band-limited),
    y_lm complex N(0,1) for l >= 2."""
    s = 2
    rng = np.random.default_rng(SEEDS["grad_l256"])
    x = rng.standard_normal((n_maps, L, 2 * L - 1, 2))
    x = x[..., 0] + 1j * x[..., 1]
    y = zero_below_spin(complex_normal(rng, L * L), L, s)
    return dict(L=L, s=s, x=x, y=y)
