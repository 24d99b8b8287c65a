"""GPU parity of the Box alias sums with their tail (lsh_set_kernel Box
parameter tail = 1) against the oracle (green.box_tail): the Green operator at
every half-spectrum bin to 1e-13, a lock-step solve, and the two-dimensional
path; plus the effect of the tail on the converged answer.
"""
import numpy as np
import pytest

import lsh_inputs as li
from helpers import PlaneProblem, Problem
from oracle import green, plane

pytestmark = pytest.mark.gpu
XI4 = np.array([[1, 0, 0, 1], [0, 1, 0, 1], [0, 0, 1, 0]], float)   # e3 a slow axis
CASES = [(np.diag([6, 8, 10]), {"Xi": XI4, "R": 10, "tail": True}),
         ([[4, 1, 0], [0, 4, 0], [0, 0, 2]], {"Xi": XI4, "R": 8, "tail": True}),
         (np.diag([6, 6, 6]), {"Xi": np.eye(3), "R": 6, "tail": True})]              # three slow axes


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def random_phase(seed):
    def f(Y):
        return np.random.default_rng(seed).integers(0, 2, size=len(Y))
    return f


@pytest.mark.parametrize("case", range(len(CASES)))
def test_gamma_probe_all_bins_with_tail(lib, case):
    M, params = CASES[case]
    pr = Problem(M, "box", params, random_phase(1))
    pr.bind("fp64")
    e = pr.G.e
    bins = np.array([(a, b, c) for a in range(e[0] // 2 + 1) for b in range(e[1]) for c in range(e[2])])
    got = pr.G.gamma_probe(bins)
    _, V = pr.G.snf()
    ref, den = green.gamma_symmetrised_at(pr.O, pr.C0, "box", params, bins @ V)
    no_tail, _ = green.gamma_symmetrised_at(pr.O, pr.C0, "box", dict(params, tail=False), bins @ V)
    iu = np.triu_indices(6)
    np.testing.assert_allclose(got, ref[:, iu[0], iu[1]], rtol=0, atol=1e-13)
    assert np.abs(ref - no_tail).max() > 1e-5          # the tail changes the operator


def test_lockstep_with_tail(lib):
    M, params = CASES[0]
    pr = Problem(M, "box", params, random_phase(4))
    pr.bind("fp64")
    eps0 = np.array([0.3, -0.2, 0.1, 0.4, -0.1, 0.25])
    ref = pr.oracle_solve(eps0, n_iter=7)
    res = pr.G.solve(eps0[None], tol=-1.0, max_iter=7, return_E=True)
    assert rel(res["sigma"][0], ref["sigma_voigt"]) < 1e-10
    assert rel(pr.gpu_E_to_oracle_mandel(res["E"].cpu().numpy()[0]), ref["E"]) < 1e-10


def test_plane_box_with_tail(lib):
    """d = 2, Xi = (e1, e2): both axes slow (the appended third axis carries none)."""
    params = {"Xi": np.array([[1, 0], [0, 1]], float), "R": 8, "tail": True}
    pr = PlaneProblem([[8, 8], [-8, 8]], "box", params, random_phase(2))
    pr.G.bind("fp64")
    eps0 = np.array([0.3, -0.2, 0.25])
    ref = pr.oracle_solve(eps0, n_iter=7)
    res = pr.G.solve(eps0[None], tol=-1.0, max_iter=7, return_E=True)
    assert rel(res["sigma"][0], ref["sigma_voigt"]) < 1e-10
    assert rel(pr.gpu_E_to_oracle_mandel(res["E"].cpu().numpy()[0]), ref["E"]) < 1e-10


def test_tail_makes_the_answer_converge_in_R(lib):
    """Converged sigma_bar for R = 4, 8, 16 against R = 32 (all with the tail):
    the differences fall much faster than without it."""
    from paper_1701_04685_amd import lsh
    M = np.diag([12, 12, 12])
    c, r = li.rsa_spheres(3, 1.0 / 12, 0.3, rmin=1.5, rmax=3.0)
    P = lsh.Pattern(M)
    ph = li.spheres_phase(P.points(), c, r)
    Cp = np.stack([li.isotropic_voigt(1.0, 0.3), li.isotropic_voigt(100.0, 0.3)])
    P.set_stiffness(Cp, li.mean_reference(Cp), ph)
    eps0 = np.array([[1.0, 0, 0, 0, 0, 0]])
    sig = {}
    for tail in (False, True):
        for R in (4, 8, 16, 32):
            P.set_kernel("box", {"Xi": XI4, "R": R, "tail": tail})
            P.bind("fp64")
            sig[(tail, R)] = P.solve(eps0, tol=1e-11, max_iter=20000)["sigma"][0]
    d_plain = [rel(sig[(False, R)], sig[(True, 32)]) for R in (4, 8, 16)]
    d_tail = [rel(sig[(True, R)], sig[(True, 32)]) for R in (4, 8, 16)]
    print("no tail", d_plain, "tail", d_tail, flush=True)
    assert d_tail[1] < d_plain[1] / 10 and d_tail[2] < d_plain[2] / 10
