"""CPU FP64 oracle for the Basic Scheme on the pattern P(M).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference that the
HIP path is checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import it; the product package
``paper_1701_04685_amd`` never does, and nothing here imports the product.

Modules
-------
lattice   integer Smith normal form, the pattern P(M), the generating set
          G(M^T) and the index maps onto the SNF grid (Sec. 2.1).
dft       the Fourier matrix F(M) by its definition and the fast form over the
          SNF grid (Sec. 2.1, eqs. (Fouriermatrix)/(FourierTransform)).
green     stiffness tensors, the Green operator of Def. (projection), the
          generating-function weights (Sec. 2.2) and the periodised Green
          operator of Def. (gamma_tilde_fourier).
scheme    the Basic Scheme fixed point for eq. (pde_coefficients) (Sec. 4),
          the effective stress and a dense direct solve of the same system.
plane     the same chain in two dimensions (2x2 patterns, plane strain,
          3-component Mandel fields), the setting of the numerics of Sec. 4.

Every function cites the passage it follows.  All floating point is float64.
The Box-spline alias sum truncation is the one fixed in Sec. 4.2 (a box of
terms around each frequency) with the normalisation over the truncated set.
"""
