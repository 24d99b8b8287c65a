"""Pins for the oracle's lattice code (Sec. 2.1): SNF, P(M), G(M^T), index maps."""
import itertools
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle.lattice import (Pattern, brute_force_generating_set, brute_force_points,
                            smith_normal_form)

HERE = os.path.dirname(__file__)
SMALL = [
    [[4, -2], [4, 14]],
    [[8, 0], [0, 8]],
    [[3, 1], [-2, 5]],
    [[8, 2, 0], [0, 8, 0], [0, 0, 4]],
    [[4, 1, 0], [0, 4, 0], [0, 0, 2]],
    [[3, 1, 0], [-1, 2, 1], [0, 1, 4]],
    [[2, 0, 0], [0, 3, 0], [0, 0, 4]],
    [[-2, 1, 1], [1, -3, 0], [0, 2, 5]],
]


def _minors_gcd(M, k):
    """k-th determinantal divisor: gcd of all k x k minors (textbook SNF invariant)."""
    A = np.array(M, dtype=object)
    d = A.shape[0]
    g = 0
    for rows in itertools.combinations(range(d), k):
        for cols in itertools.combinations(range(d), k):
            sub = A[np.ix_(rows, cols)].tolist()
            g = math.gcd(g, abs(int(round(_exact_det(sub)))))
    return g


def _exact_det(A):
    n = len(A)
    if n == 1:
        return A[0][0]
    return sum((-1) ** j * A[0][j] * _exact_det([r[:j] + r[j + 1:] for r in A[1:]]) for j in range(n))


def _random_matrices(n, d, seed):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < n:
        M = rng.integers(-9, 10, size=(d, d))
        if round(abs(np.linalg.det(M))) != 0 and abs(np.linalg.det(M)) < 600:
            out.append(M.tolist())
    return out


@pytest.mark.parametrize("M", SMALL + _random_matrices(12, 3, 7) + _random_matrices(8, 2, 8))
def test_snf_invariants(M):
    """U D V = M, U and V unimodular, e_i | e_{i+1}, prod e = |det M|, and the
    diagonal equals the determinantal-divisor quotients (independent of the
    algorithm that computed it)."""
    U, e, V = smith_normal_form(M)
    d = len(M)
    UDV = np.array(U, dtype=object) @ np.diag(e).astype(object) @ np.array(V, dtype=object)
    assert UDV.tolist() == [list(map(int, r)) for r in M]
    assert abs(_exact_det(U)) == 1 and abs(_exact_det(V)) == 1
    assert all(x > 0 for x in e)
    assert all(e[i + 1] % e[i] == 0 for i in range(d - 1))
    assert math.prod(e) == abs(_exact_det(M))
    prev = 1
    for k in range(1, d + 1):
        dk = _minors_gcd(M, k)
        assert e[k - 1] == dk // prev
        prev = dk


def test_paper_pattern_sizes():
    """|P(M)| = |det M| for the matrices printed in the paper (golden file)."""
    gold = json.load(open(os.path.join(HERE, "golden", "paper_patterns.json")))
    for item in gold["patterns"]:
        P = Pattern(item["M"])
        assert P.m == item["m"], item["cite"]
        assert math.prod(P.e) == item["m"]
        if item["m"] <= 64:
            assert len(brute_force_points(item["M"])) == item["m"]


@pytest.mark.parametrize("M", SMALL)
def test_points_match_enumeration(M):
    """The SNF point map is a bijection onto M^{-1} Z^d cap [-1/2,1/2)^d (Sec. 2.1)."""
    P = Pattern(M)
    N = P.point_numerators()
    got = sorted(tuple(Fraction(int(v), P.m) for v in row) for row in N)
    assert got == brute_force_points(M)
    assert np.all(N >= -(P.m // 2)) and np.all(N < P.m - P.m // 2)


@pytest.mark.parametrize("M", SMALL)
def test_frequencies_match_enumeration(M):
    """h(b) = V^T b reduced mod M^T is a bijection onto G(M^T) = M^T P(M^T)."""
    P = Pattern(M)
    H, Xn = P.frequencies()
    assert sorted(map(tuple, H.tolist())) == brute_force_generating_set(M)
    # x = M^{-T} h is the stored numerator over m, inside the half-open cube
    MinvT = np.linalg.inv(np.array(M, dtype=float)).T
    np.testing.assert_allclose(H @ MinvT.T, Xn / P.m, atol=1e-12)
    assert np.all(Xn / P.m >= -0.5) and np.all(Xn / P.m < 0.5)


@pytest.mark.parametrize("M", SMALL)
def test_exponent_identity(M):
    """h(b)^T y(a) = sum_i a_i b_i / e_i mod 1: the SNF grid DFT is the pattern DFT."""
    P = Pattern(M)
    a = P.grid_indices()
    Y = P.point_numerators()
    H, _ = P.frequencies()
    lhs = (H.astype(object) @ Y.T.astype(object))  # exact: m * h^T y
    rhs = np.zeros_like(lhs)
    for i, e in enumerate(P.e):
        rhs = rhs + np.outer(a[:, i], a[:, i]).astype(object) * (P.m // e)
    assert np.all(((lhs - rhs) % P.m) == 0)


def test_singular_rejected():
    with pytest.raises(ValueError):
        Pattern([[2, 4], [1, 2]])


def test_rank1_like_reduces_to_1d():
    """Rank-1 lattices reduce to a one-dimensional FFT (Sec. 2.1): SNF (1, ..., 1, m)."""
    P = Pattern([[1, 0, 0], [0, 1, 0], [3, 5, 17]])
    assert P.e == [1, 1, 17]
