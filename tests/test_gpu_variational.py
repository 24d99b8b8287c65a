"""GPU parity of the variational discretisation, eq. (pde_coefficients_variational),
against the FP64 oracle's strain-update iteration (lock-step: both run exactly
n iterations; FP64 1e-10, FP32 1e-5 relative on E and sigma_bar), and the
coincidence of the two discretisations for the Dirichlet kernel on the GPU."""
import numpy as np
import pytest

import lsh_inputs as li
from helpers import BOX_CFG3, Problem

pytestmark = pytest.mark.gpu
TOL = {"fp64": 1e-10, "fp32": 1e-5}
EPS0 = np.array([0.3, -0.2, 0.1, 0.4, -0.1, 0.25])
KERNELS = [("dirichlet", {}), ("dirichlet_modified", {}), ("dlvp", {"alpha": [0.75] * 3}),
           ("box", {"Xi": BOX_CFG3["Xi"], "R": 3})]


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def random_phase(seed, frac=0.4):
    rng = np.random.default_rng(seed)
    return lambda Y: (rng.random(len(Y)) < frac).astype(np.uint8)


CASES = [(np.diag([8, 8, 8]), random_phase(21)),
         ([[6, -3, 2], [1, 4, 0], [2, 0, 3]], random_phase(22)),
         (np.diag([24, 20, 18]), random_phase(23))]


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("kind,params", KERNELS)
def test_variational_lockstep(kind, params, case, prec):
    M, ph = CASES[case]
    pr = Problem(M, kind, params, ph)
    pr.G.set_scheme("ve")
    pr.bind(prec)
    n = 7
    res = pr.G.solve(EPS0[None], tol=-1.0, max_iter=n, return_E=True, history=True)
    ref = pr.oracle_solve_ve(EPS0, n_iter=n)
    np.testing.assert_allclose(res["history"][0], ref["history"], rtol=100 * TOL[prec], atol=1e-14)
    assert rel(res["sigma"][0], ref["sigma_voigt"]) < TOL[prec]
    assert rel(pr.gpu_E_to_oracle_mandel(res["E"].cpu().numpy()[0]), ref["E"]) < TOL[prec]


def test_dirichlet_variational_equals_ls_on_gpu():
    """Remark (constants): with the Dirichlet kernel the two discretisations have
    the same iterates (odd axes: no real-part projection on -1/2 faces)."""
    pr = Problem(np.diag([5, 5, 7]), "dirichlet", {}, random_phase(24))
    pr.bind("fp64")
    a = pr.G.solve(EPS0[None], tol=1e-12, max_iter=500, return_E=True)
    pr.G.set_scheme("ve")
    pr.bind("fp64")
    b = pr.G.solve(EPS0[None], tol=1e-12, max_iter=500, return_E=True)
    assert a["iterations"][0] == b["iterations"][0]
    assert rel(b["sigma"][0], a["sigma"][0]) < 1e-11


def test_variational_batch_matches_single():
    """A batch of variational tasks (several contrasts, one group) gives the
    single solves' results.  (The strain update converges slowly for non-Dirichlet
    kernels: the Green multiplier has small eigenvalues on its range.)"""
    from paper_1701_04685_amd import lsh
    pats, loads, singles = [], [], []
    for i, contrast in enumerate([3.0, 7.0, 20.0]):
        P = lsh.Pattern(np.diag([16, 16, 16]))
        P.set_kernel("dlvp", {"alpha": [0.75] * 3})
        Cp = np.stack([li.isotropic_voigt(1.0, 0.3), li.isotropic_voigt(contrast, 0.3)])
        ph = (np.random.default_rng(30 + i).random(P.m) < 0.3).astype(np.uint8)
        P.set_stiffness(Cp, li.mean_reference(Cp), ph)
        P.set_scheme("ve")
        P.bind("fp64")
        pats.append(P)
        loads.append(np.eye(6)[:2])
        singles.append(P.solve(np.eye(6)[:2], tol=1e-7, max_iter=40000))
    res = lsh.solve_batch(pats, loads, tol=1e-7, max_iter=40000, precision="fp64")
    for r, s in zip(res, singles):
        np.testing.assert_array_equal(r["iterations"], s["iterations"])
        assert rel(r["sigma"], s["sigma"]) < 1e-12
