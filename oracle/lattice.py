"""Pattern P(M), generating set G(M^T) and the Smith-normal-form index maps.

Test infrastructure (oracle); see the package docstring.

Paper, Sec. 2.1 ("The pattern and the generating set"): for a regular integer
matrix M the lattice is Lambda(M) = M^{-1} Z^d, the pattern P(M) is the set of
its points in the half-open cube [-1/2, 1/2)^d, the generating set is
G(M) = M P(M), and |P(M)| = |G(M)| = |det M| = m.

The Fourier matrix needs an ordering of P(M) and G(M^T).  With a Smith normal
form M = U D V (U, V unimodular, D = diag(e_1..e_d), e_i | e_{i+1}) the point
y(a) = M^{-1} U a  (a in Z_{e_1} x ... x Z_{e_d}) and the frequency
h(b) = V^T b satisfy h(b)^T y(a) = sum_i a_i b_i / e_i (mod 1), so the pattern
DFT is the plain multidimensional DFT over the SNF grid.  The SNF itself is
textbook integer linear algebra; the paper only cites an ordering-based FFT.

All arithmetic here is exact (Python integers).
"""
from __future__ import annotations

import itertools
from fractions import Fraction

import numpy as np


def _det(A):
    """Exact determinant of a small integer matrix (Laplace expansion)."""
    n = len(A)
    if n == 1:
        return A[0][0]
    if n == 2:
        return A[0][0] * A[1][1] - A[0][1] * A[1][0]
    s = 0
    for j in range(n):
        minor = [row[:j] + row[j + 1:] for row in A[1:]]
        s += (-1) ** j * A[0][j] * _det(minor)
    return s


def _adj(A):
    """Exact adjugate: adj(A) A = A adj(A) = det(A) I."""
    n = len(A)
    if n == 1:
        return [[1]]
    out = [[0] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            minor = [row[:j] + row[j + 1:] for k, row in enumerate(A) if k != i]
            out[j][i] = (-1) ** (i + j) * _det(minor)
    return out


def _matmul(A, B):
    return [[sum(A[i][k] * B[k][j] for k in range(len(B))) for j in range(len(B[0]))]
            for i in range(len(A))]


def _eye(n):
    return [[int(i == j) for j in range(n)] for i in range(n)]


def _as_int_matrix(M):
    A = [[int(v) for v in row] for row in np.asarray(M).tolist()]
    d = len(A)
    if d == 0 or any(len(r) != d for r in A):
        raise ValueError("M must be a square integer matrix")
    return A


def smith_normal_form(M):
    """Integer Smith normal form M = U D V.

    Returns (U, D, V) as Python int lists with U, V unimodular and
    D = diag(e_1, ..., e_d), e_i > 0, e_i | e_{i+1}.  Raises ValueError for a
    singular M (the pattern needs a regular M, Sec. 2.1).

    Method: row and column operations L A R on a working copy until it is
    diagonal with the divisibility chain; then U = L^{-1}, V = R^{-1}.
    """
    A = _as_int_matrix(M)
    d = len(A)
    if _det(A) == 0:
        raise ValueError("M is singular; the pattern needs det M != 0")
    L = _eye(d)  # row operations applied so far
    R = _eye(d)  # column operations applied so far

    def swap_rows(i, j):
        A[i], A[j] = A[j], A[i]
        L[i], L[j] = L[j], L[i]

    def swap_cols(i, j):
        for X in (A, R):
            for row in X:
                row[i], row[j] = row[j], row[i]

    def add_row(dst, src, q):  # row_dst += q * row_src
        for X in (A, L):
            X[dst] = [a + q * b for a, b in zip(X[dst], X[src])]

    def add_col(dst, src, q):  # col_dst += q * col_src
        for X in (A, R):
            for row in X:
                row[dst] += q * row[src]

    for t in range(d):
        while True:
            # pivot: the smallest non-zero magnitude in the trailing block
            best = None
            for i in range(t, d):
                for j in range(t, d):
                    if A[i][j] != 0 and (best is None or abs(A[i][j]) < abs(A[best[0]][best[1]])):
                        best = (i, j)
            if best is None:
                raise ValueError("M is singular")
            swap_rows(t, best[0])
            swap_cols(t, best[1])
            p = A[t][t]
            clean = True
            for i in range(t + 1, d):
                q = A[i][t] // p
                if q:
                    add_row(i, t, -q)
                if A[i][t] != 0:
                    clean = False
            for j in range(t + 1, d):
                q = A[t][j] // p
                if q:
                    add_col(j, t, -q)
                if A[t][j] != 0:
                    clean = False
            if not clean:
                continue
            # divisibility: every trailing entry must be a multiple of the pivot
            bad = None
            for i in range(t + 1, d):
                for j in range(t + 1, d):
                    if A[i][j] % p != 0:
                        bad = i
            if bad is not None:
                add_row(t, bad, 1)
                continue
            break
        if A[t][t] < 0:
            for X in (A, L):
                X[t] = [-v for v in X[t]]
    D = [A[i][i] for i in range(d)]
    detL = _det(L)
    detR = _det(R)
    assert abs(detL) == 1 and abs(detR) == 1
    U = [[v * detL for v in row] for row in _adj(L)]  # L^{-1}
    V = [[v * detR for v in row] for row in _adj(R)]  # R^{-1}
    return U, D, V


def _center_mod(v, m):
    """Representative of v mod m in [-m/2, m/2): the half-open cube rule."""
    h = m // 2
    return ((v + h) % m) - h


class Pattern:
    """P(M), G(M^T) and the SNF index maps for one regular integer matrix M.

    Attributes
    ----------
    M : (d, d) int list
    m : |det M|
    e : SNF diagonal (e_1 .. e_d), product m
    U, V : unimodular SNF factors, M = U diag(e) V
    """

    def __init__(self, M):
        self.M = _as_int_matrix(M)
        self.d = len(self.M)
        self.det = _det(self.M)
        if self.det == 0:
            raise ValueError("M is singular")
        self.m = abs(self.det)
        self.U, self.e, self.V = smith_normal_form(self.M)
        self.sign = 1 if self.det > 0 else -1
        self.adjM = _adj(self.M)
        self.MT = [list(r) for r in zip(*self.M)]
        self.adjMT = [list(r) for r in zip(*self.adjM)]

    # -- storage order ------------------------------------------------------
    def grid_indices(self):
        """All a in Z_{e_1} x ... x Z_{e_d} in storage (C, last index fastest) order."""
        return np.array(list(itertools.product(*[range(k) for k in self.e])), dtype=np.int64)

    # -- points -------------------------------------------------------------
    def point_numerators(self, a=None):
        """Integer numerators N with y = N / m in [-1/2, 1/2)^d, y = M^{-1} U a mod 1.

        Sec. 2.1: y in Lambda(M) = M^{-1} Z^d, represented in the half-open
        symmetric cube.  M^{-1} = adj(M) / det M, so m y is an integer vector.
        Vectorised int64 arithmetic, checked against overflow.
        """
        if a is None:
            a = self.grid_indices()
        a = np.asarray(a, dtype=np.int64)
        T = self.sign * np.array(_matmul(self.adjM, self.U), dtype=object)
        self._check_range(T, self.e)
        num = a @ np.array(T.T.tolist(), dtype=np.int64)
        return _center_mod_np(num, self.m)

    def points(self):
        """Pattern points y in storage order, float64 (exact rationals rounded once)."""
        return self.point_numerators().astype(np.float64) / self.m

    # -- frequencies ----------------------------------------------------------
    def reduce_frequency(self, h):
        """Representative of h mod M^T in G(M^T) = M^T P(M^T).

        Returns (h_rep, x_num) with x = M^{-T} h_rep = x_num / m in [-1/2, 1/2)^d.
        """
        h = [int(v) for v in h]
        xn = [self.sign * sum(self.adjMT[i][k] * h[k] for k in range(self.d)) for i in range(self.d)]
        xr = [_center_mod(v, self.m) for v in xn]
        z = [(a - b) // self.m for a, b in zip(xn, xr)]
        hr = [h[i] - sum(self.MT[i][k] * z[k] for k in range(self.d)) for i in range(self.d)]
        return hr, xr

    def frequencies(self, b=None):
        """h(b) = V^T b reduced into G(M^T), storage order.

        Returns (h int64 (n, d), x_num int64 (n, d)) with x = M^{-T} h = x_num / m
        in [-1/2, 1/2)^d.  Vectorised form of reduce_frequency.
        """
        if b is None:
            b = self.grid_indices()
        b = np.asarray(b, dtype=np.int64)
        VT = np.array(self.V, dtype=np.int64).T
        return self.reduce_frequencies(b @ VT.T)

    def reduce_frequencies(self, h):
        """Vectorised reduce_frequency for integer frequencies h (n, d)."""
        h = np.asarray(h, dtype=np.int64)
        A = self.sign * np.array(self.adjMT, dtype=object)
        bound = int(np.abs(h).max(initial=0)) * sum(abs(int(v)) for row in A.tolist() for v in row)
        if bound >= 2 ** 62:
            raise OverflowError("frequency too large for int64")
        xn = h @ np.array(A.tolist(), dtype=np.int64).T
        xr = _center_mod_np(xn, self.m)
        z = (xn - xr) // self.m
        hr = h - z @ np.array(self.MT, dtype=np.int64).T
        return hr, xr

    @staticmethod
    def _check_range(T, e):
        bound = sum(abs(int(v)) for row in np.asarray(T).tolist() for v in row) * max(e)
        if bound >= 2 ** 62:
            raise OverflowError("pattern too large for int64 index maps")


def _center_mod_np(v, m):
    h = m // 2
    return ((v + h) % m) - h


def brute_force_points(M):
    """P(M) by enumeration: every y = M^{-1} j in [-1/2, 1/2)^d (Sec. 2.1).

    Independent of the SNF: scans integer vectors j in a box large enough to
    hit every class of Z^d / M Z^d and keeps the distinct reduced points.
    Returns a sorted list of tuples of Fractions.
    """
    A = _as_int_matrix(M)
    d = len(A)
    det = _det(A)
    adj = _adj(A)
    m = abs(det)
    # every class of Z^d / M Z^d has a member in the parallelotope M [0,1)^d,
    # whose i-th coordinate lies between the sums of the negative and positive
    # entries of row i
    ranges = [range(sum(min(0, v) for v in row), sum(max(0, v) for v in row) + 1) for row in A]
    seen = set()
    for j in itertools.product(*ranges):
        y = []
        for i in range(d):
            f = Fraction(sum(adj[i][k] * j[k] for k in range(d)), det)
            f = f - (f + Fraction(1, 2)).__floor__()  # into [-1/2, 1/2)
            y.append(f)
        seen.add(tuple(y))
    pts = sorted(seen)
    if len(pts) != m:
        raise AssertionError(f"enumeration found {len(pts)} points, expected {m}")
    return pts


def brute_force_generating_set(M):
    """G(M^T) = M^T P(M^T) by enumeration (Sec. 2.1); list of int tuples."""
    A = _as_int_matrix(M)
    AT = [list(r) for r in zip(*A)]
    out = []
    for x in brute_force_points(AT):
        h = tuple(int(sum(AT[i][k] * x[k] for k in range(len(AT)))) for i in range(len(AT)))
        out.append(h)
    return sorted(out)
