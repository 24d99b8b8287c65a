"""Pins for the oracle's pattern DFT (Sec. 2.1, eqs. (Fouriermatrix)/(FourierTransform))."""
from fractions import Fraction

import numpy as np
import pytest

from oracle.dft import fourier_matrix, pattern_dft, pattern_idft
from oracle.lattice import Pattern

SMALL = [
    [[4, -2], [4, 14]],
    [[3, 1], [-2, 5]],
    [[8, 2, 0], [0, 8, 0], [0, 0, 4]],
    [[4, 1, 0], [0, 4, 0], [0, 0, 2]],
    [[3, 1, 0], [-1, 2, 1], [0, 1, 4]],
]


@pytest.mark.parametrize("M", SMALL)
def test_fast_dft_equals_fourier_matrix(M):
    """SNF-grid FFT == the Fourier matrix written out from its definition,
    rows and columns matched by exact coordinates (brute-force enumeration)."""
    P = Pattern(M)
    F, Hbf, Ybf = fourier_matrix(M)
    rng = np.random.default_rng(1)
    a = rng.standard_normal((P.m, 2)) + 1j * rng.standard_normal((P.m, 2))
    # a is indexed by the oracle's storage order; permute to the enumeration order
    Ynum = P.point_numerators()
    key = {tuple(Fraction(int(v), P.m) for v in row): i for i, row in enumerate(Ynum)}
    from oracle.lattice import brute_force_points
    order = [key[y] for y in brute_force_points(M)]
    ref = np.sqrt(P.m) * (F @ a[order])
    fast = pattern_dft(P, a)
    H, _ = P.frequencies()
    hkey = {tuple(h): i for i, h in enumerate(H.tolist())}
    horder = [hkey[tuple(h)] for h in Hbf.tolist()]
    np.testing.assert_allclose(fast[horder], ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("M", SMALL)
def test_fourier_matrix_unitary(M):
    F, _, _ = fourier_matrix(M)
    np.testing.assert_allclose(F.conj().T @ F, np.eye(F.shape[0]), atol=1e-12)


@pytest.mark.parametrize("M", SMALL)
def test_inverse_round_trip(M):
    P = Pattern(M)
    rng = np.random.default_rng(2)
    a = rng.standard_normal((P.m, 6))
    np.testing.assert_allclose(pattern_idft(P, pattern_dft(P, a)).real, a, atol=1e-13)


@pytest.mark.parametrize("M", SMALL)
def test_aliasing_lemma(M):
    """Lemma (Aliasing): sampling f = sum_k c_k e^{i k^T x} on 2 pi P(M) gives
    discrete coefficients c^M_h = sum_z c_{h + M^T z} (the bracket sum)."""
    P = Pattern(M)
    d = P.d
    rng = np.random.default_rng(3)
    K = np.array(np.meshgrid(*[np.arange(-9, 10)] * d, indexing="ij")).reshape(d, -1).T
    c = rng.standard_normal(len(K)) + 1j * rng.standard_normal(len(K))
    Y = P.points()
    samples = np.exp(1j * (2 * np.pi * Y) @ K.T) @ c          # f(2 pi y)
    disc = pattern_dft(P, samples) / P.m                          # c^M_h, h = h(b)
    H, _ = P.frequencies()
    # bracket sum: group k by its class mod M^T via the oracle's own reduction
    expect = np.zeros(P.m, dtype=complex)
    hkey = {tuple(h): i for i, h in enumerate(H.tolist())}
    for k, ck in zip(K.tolist(), c):
        hr, _ = P.reduce_frequency(k)
        expect[hkey[tuple(hr)]] += ck
    np.testing.assert_allclose(disc, expect, atol=1e-10)
