"""The discrete Fourier transform on the pattern P(M).

Test infrastructure (oracle); see the package docstring.

Sec. 2.1, eq. (Fouriermatrix): F(M) = m^{-1/2} (exp(-2 pi i h^T y)) with rows
h in G(M^T) and columns y in P(M); eq. (FourierTransform): a_hat = F(M) a.

Two forms are provided:

* ``fourier_matrix`` writes the definition out entry by entry over the
  brute-force enumerations of P(M) and G(M^T) (small m only);
* ``pattern_dft`` / ``pattern_idft`` evaluate the same sum in O(m log m):
  with the SNF orderings of ``lattice.Pattern`` the exponent h^T y equals
  sum_i a_i b_i / e_i mod 1, which is the multidimensional DFT over the SNF
  grid (``scipy.fft.fftn`` serves as that library step; it honours
  ``scipy.fft.set_workers`` for the number of host threads).

The fast form is unnormalised (no m^{-1/2}); the inverse carries 1/m, so the
pair is exact inverse to each other as the paper's unitary pair is.
"""
from __future__ import annotations

import numpy as np
import scipy.fft

from .lattice import Pattern, brute_force_generating_set, brute_force_points


def fourier_matrix(M):
    """F(M) by eq. (Fouriermatrix), with its row and column sets.

    Returns (F, H, Y): F complex (m, m), H int (m, d) the rows h in G(M^T),
    Y float (m, d) the columns y in P(M), both in sorted enumeration order.
    """
    Yf = brute_force_points(M)
    H = np.array(brute_force_generating_set(M), dtype=np.int64)
    Y = np.array([[float(v) for v in y] for y in Yf])
    m = len(Yf)
    F = np.exp(-2j * np.pi * (H @ Y.T)) / np.sqrt(m)
    return F, H, Y


def pattern_dft(P: Pattern, a):
    """Unnormalised pattern DFT of samples a (m, ...) in storage order.

    Output index is the frequency storage order b (SNF grid, last fastest);
    output[b] = sum_y a_y exp(-2 pi i h(b)^T y).
    """
    a = np.asarray(a)
    shape = tuple(P.e) + a.shape[1:]
    A = a.reshape(shape)
    return scipy.fft.fftn(A, axes=tuple(range(P.d))).reshape(a.shape[0:1] + a.shape[1:])


def pattern_idft(P: Pattern, ahat):
    """Inverse of pattern_dft: (1/m) sum_h ahat_h exp(+2 pi i h^T y)."""
    ahat = np.asarray(ahat)
    shape = tuple(P.e) + ahat.shape[1:]
    A = ahat.reshape(shape)
    return scipy.fft.ifftn(A, axes=tuple(range(P.d))).reshape(ahat.shape)
