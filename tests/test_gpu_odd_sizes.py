"""GPU parity on compile-time odd line lengths (125 = 5^3): the Basic Scheme
and conjugate gradients in lock step with the oracle, on patterns whose SNF
puts 125 on the axis-2 and axis-3 passes (diag(125, 125, 5) -> (5, 125, 125))
and on all three (diag(125, 125, 125)).  Tolerances as for the other
lock-step tests (FP64 1e-10, FP32 1e-5 relative).
"""
import numpy as np
import pytest

import lsh_inputs as li
from helpers import Problem
from oracle import scheme

pytestmark = pytest.mark.gpu
EPS0 = np.array([0.3, -0.2, 0.1, 0.4, -0.1, 0.25])


def rel(a, b):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def spheres(seed, rmin=2.0, rmax=4.0):
    def f(Y):
        c, r = li.rsa_spheres(seed, li.lattice_unit(len(Y)), 0.3, rmin=rmin, rmax=rmax)
        return li.spheres_phase(Y, c, r)
    return f


@pytest.fixture(scope="module")
def cube125(lib):
    """125^3, Dirichlet, contrast 50: one problem (and one oracle Green
    operator, the expensive part) for the Basic Scheme and CG tests."""
    Cp = np.stack([li.isotropic_voigt(1.0, 0.3), li.isotropic_voigt(50.0, 0.3)])
    # ~100 spheres of radius 8-14 grid steps (smaller ones would take thousands)
    pr = Problem(np.diag([125, 125, 125]), "dirichlet", {}, spheres(3, 8.0, 14.0), Cp, li.mean_reference(Cp))
    pr.gamma_oracle()
    return pr


@pytest.mark.parametrize("M,prec,kind", [(np.diag([125, 125, 5]), "fp64", "dlvp"),
                                         (np.diag([125, 125, 5]), "fp32", "dlvp"),
                                         (None, "fp64", "dirichlet")])
def test_basic_scheme_lockstep(lib, cube125, M, prec, kind):
    params = {"alpha": [0.75] * 3} if kind == "dlvp" else {}
    if M is None:
        pr = cube125
        pr.G.set_scheme("ls")
    else:
        pr = Problem(M, kind, params, spheres(2))
    assert 125 in pr.G.e
    print(f"odd-size lockstep e={pr.G.e} {kind} {prec}", flush=True)
    pr.bind(prec)
    n = 4
    ref = pr.oracle_solve(EPS0, n_iter=n)
    res = pr.G.solve(EPS0[None], tol=-1.0, max_iter=n, return_E=True)
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert rel(res["sigma"][0], ref["sigma_voigt"]) < tol
    assert rel(pr.gpu_E_to_oracle_mandel(res["E"].cpu().numpy()[0]), ref["E"]) < tol


@pytest.mark.parametrize("M", [np.diag([125, 125, 5]), None])
def test_cg_lockstep(lib, cube125, M):
    if M is None:
        pr = cube125
    else:
        Cp = np.stack([li.isotropic_voigt(1.0, 0.3), li.isotropic_voigt(50.0, 0.3)])
        pr = Problem(M, "dirichlet", {}, spheres(3), Cp, li.mean_reference(Cp))
    pr.G.set_scheme("cg")
    pr.bind("fp64")
    print(f"odd-size CG lockstep e={pr.G.e}", flush=True)
    n = 5
    ref = scheme.conjugate_gradient(pr.O, pr.gamma_oracle(), pr.Cp, pr.C0, pr.phase_o, EPS0, n_iter=n)
    res = pr.G.solve(EPS0[None], tol=-1.0, max_iter=n, return_E=True, history=True)
    assert rel(res["sigma"][0], ref["sigma_voigt"]) < 1e-10
    assert rel(pr.gpu_E_to_oracle_mandel(res["E"].cpu().numpy()[0]), ref["E"]) < 1e-10
    np.testing.assert_allclose(res["history"][0], ref["history"], rtol=1e-8, atol=1e-15)


def _anisotropic_C0():
    """An elliptic, cubic-anisotropic reference stiffness (not isotropic)."""
    C = li.isotropic_voigt(4.0, 0.25)
    C[0, 1] = C[1, 0] = C[0, 1] + 0.3
    C[3, 3] += 0.4
    C[5, 5] -= 0.2
    return C


@pytest.mark.parametrize("kind,params,aniso,prec", [
    ("dirichlet", {}, True, "fp64"),                                   # general form on the fly
    ("dlvp", {"alpha": [0.75] * 3}, True, "fp64"),                     # table, general alias sums
    ("box", {"Xi": np.array([[1, 0, 0, 1], [0, 1, 0, 1], [0, 0, 1, 0]], float), "R": 2}, False, "fp64"),
    ("box", {"Xi": np.array([[1, 0, 0, 1], [0, 1, 0, 1], [0, 0, 1, 0]], float), "R": 2}, False, "fp32"),
])
def test_odd_length_green_modes_lockstep(lib, kind, params, aniso, prec):
    """The odd-length Green pass in its table and general modes (the moment
    mode is covered above): diag(125, 5, 5) puts 125 on the axis-3 pass."""
    Cp = np.stack([li.isotropic_voigt(1.0, 0.3), li.isotropic_voigt(10.0, 0.3)])
    C0 = _anisotropic_C0() if aniso else li.mean_reference(Cp)
    pr = Problem(np.diag([125, 5, 5]), kind, params, spheres(5, 0.5, 1.0), Cp, C0)
    assert pr.G.e[2] == 125
    print(f"odd-length Green mode {kind} aniso={aniso} {prec} e={pr.G.e}", flush=True)
    pr.bind(prec)
    n = 4
    ref = pr.oracle_solve(EPS0, n_iter=n)
    res = pr.G.solve(EPS0[None], tol=-1.0, max_iter=n, return_E=True)
    tol = 1e-10 if prec == "fp64" else 1e-5
    assert rel(res["sigma"][0], ref["sigma_voigt"]) < tol
    assert rel(pr.gpu_E_to_oracle_mandel(res["E"].cpu().numpy()[0]), ref["E"]) < tol
