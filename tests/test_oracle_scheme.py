"""Pins for the oracle's Basic Scheme (Thm. (pde_discretization), Sec. 4)."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import green, scheme
from oracle.lattice import Pattern
import lsh_inputs as li

HERE = os.path.dirname(__file__)
BOX4 = {"Xi": np.array([[1, 0, 0, 1], [0, 1, 0, 1], [0, 0, 1, 0]], float), "R": 3}
KERNELS = [("dirichlet", {}), ("dirichlet_modified", {}), ("dlvp", {"alpha": [0.75] * 3}), ("box", BOX4)]


def two_phase(E1=1.0, E2=10.0, nu=0.3):
    Cp = np.stack([li.isotropic_voigt(E1, nu), li.isotropic_voigt(E2, nu)])
    return Cp, li.mean_reference(Cp)


@pytest.mark.parametrize("kind,params", KERNELS)
def test_homogeneous_material_one_iteration(kind, params):
    """C constant: the polarisation is constant, only h = 0 is excited, and
    Gamma^p_0 = 0, so E^1 = 0 exactly and sigma_bar = C eps0."""
    P = Pattern([[4, 1, 0], [0, 4, 0], [0, 0, 2]])
    Cp = np.stack([li.isotropic_voigt(3.0, 0.2)])
    C0 = li.isotropic_voigt(1.0, 0.3)
    G, _ = green.gamma_periodised(P, C0, kind, params)
    eps0 = np.array([0.3, -0.1, 0.2, 0.05, -0.4, 0.1])
    res = scheme.basic_scheme(P, G, Cp, C0, np.zeros(P.m, np.uint8), eps0, tol=1e-12)
    assert res["iterations"] == 1
    assert np.abs(res["E"]).max() < 1e-15
    np.testing.assert_allclose(res["sigma_voigt"], Cp[0] @ eps0, rtol=1e-14)


def _laminate_closed_form():
    gold = json.load(open(os.path.join(HERE, "golden", "laminate.json")))
    C = np.zeros((6, 6))
    names = {"C11": (0, 0), "C12": (0, 1), "C13": (0, 2), "C22": (1, 1), "C33": (2, 2),
             "C23": (1, 2), "C44": (3, 3), "C55": (4, 4), "C66": (5, 5)}
    for k, (i, j) in names.items():
        C[i, j] = C[j, i] = gold[k][0] / gold[k][1]
    return C, gold


def _laminate_formulas(E=(1.0, 10.0), nu=0.3):
    """Rank-one laminate, f = 1/2, normal e1 (textbook formulas, independent of the scheme)."""
    lam = np.array([li.lame(e, nu)[0] for e in E])
    mu = np.array([li.lame(e, nu)[1] for e in E])
    Pm = lam + 2 * mu
    av = lambda v: v.mean()
    C11 = 1 / av(1 / Pm)
    C12 = av(lam / Pm) * C11
    C22 = av(Pm - lam ** 2 / Pm) + av(lam / Pm) ** 2 * C11
    C23 = av(lam - lam ** 2 / Pm) + av(lam / Pm) ** 2 * C11
    return dict(C11=C11, C12=C12, C22=C22, C23=C23, C44=av(mu), C55=1 / av(1 / mu))


def test_laminate_golden_matches_formulas():
    C, _ = _laminate_closed_form()
    f = _laminate_formulas()
    for k, (i, j) in {"C11": (0, 0), "C12": (0, 1), "C22": (1, 1), "C23": (1, 2), "C44": (3, 3), "C55": (4, 4)}.items():
        assert abs(C[i, j] - f[k]) < 1e-14


@pytest.mark.parametrize("kind,params", KERNELS)
def test_laminate_closed_form(kind, params):
    """16^3 laminate (layers normal to x1, f = 1/2, E = 1/10, nu = 0.3, C0 = mean):
    the Basic Scheme reproduces the closed-form C^eff for every kernel and stops
    after 2 iterations (the first iterate is exact)."""
    C_ref, gold = _laminate_closed_form()
    P = Pattern(np.diag([16, 16, 16]))
    ph = li.laminate_phase(P.points(), 0)
    Cp, C0 = two_phase()
    G, _ = green.gamma_periodised(P, C0, kind, params)
    Ceff, its = scheme.effective_stiffness(P, G, Cp, C0, ph, tol=1e-10)
    np.testing.assert_allclose(Ceff, C_ref, rtol=0, atol=1e-12 * np.abs(C_ref).max())
    assert its[0] == gold["iterations_dirichlet_C0_mean"]


@pytest.mark.parametrize("M", [[[4, 1, 0], [0, 4, 0], [0, 0, 2]], [[3, 1, 0], [-1, 2, 1], [0, 1, 4]]])
@pytest.mark.parametrize("kind,params", KERNELS)
def test_fixed_point_equals_dense_solve(M, kind, params):
    """The Basic Scheme limit solves eq. (pde_coefficients): compare with a dense
    linear solve assembled from the Fourier matrix written out entry by entry."""
    P = Pattern(M)
    rng = np.random.default_rng(4)
    ph = rng.integers(0, 2, size=P.m).astype(np.uint8)
    Cp, C0 = two_phase(1.0, 5.0, 0.3)
    eps0 = np.array([0.2, -0.1, 0.05, 0.3, 0.1, -0.2])
    G, _ = green.gamma_periodised(P, C0, kind, params)
    res = scheme.basic_scheme(P, G, Cp, C0, ph, eps0, tol=1e-15, max_iter=5000)
    Ynum = P.point_numerators()
    by_point = {tuple(Fraction(int(v), P.m) for v in row): int(p) for row, p in zip(Ynum, ph)}
    Y, Ed = scheme.dense_fixed_point(M, C0, kind, params, Cp, by_point, eps0)
    key = {tuple(Fraction(int(v), P.m) for v in row): i for i, row in enumerate(Ynum)}
    from oracle.lattice import brute_force_points
    order = [key[y] for y in brute_force_points(M)]
    np.testing.assert_allclose(res["E"][order], Ed, atol=1e-11 * max(1, np.abs(Ed).max()))


@pytest.mark.parametrize("kind,params", [("dirichlet", {}), ("dlvp", {"alpha": [0.5] * 3}), ("box", BOX4)])
def test_effective_tensor_symmetric(kind, params):
    """C^eff is symmetric at the fixed point for every kernel (Gamma^p C0 is
    C0-self-adjoint, Sec. 3.2 adjointness theorem), up to the iteration error."""
    P = Pattern(np.diag([6, 6, 6]))
    rng = np.random.default_rng(6)
    ph = rng.integers(0, 2, size=P.m).astype(np.uint8)
    Cp, C0 = two_phase(1.0, 10.0, 0.3)
    G, _ = green.gamma_periodised(P, C0, kind, params)
    Ceff, _ = scheme.effective_stiffness(P, G, Cp, C0, ph, tol=1e-13, max_iter=3000)
    asym = np.linalg.norm(Ceff - Ceff.T) / np.linalg.norm(Ceff)
    assert asym < 1e-11


def test_dirichlet_between_reuss_and_voigt_bounds():
    """The Dirichlet discretisation is a Galerkin method on compatible fields,
    so C_Reuss <= C^eff <= C_Voigt in the Loewner order (Mandel form)."""
    P = Pattern(np.diag([6, 6, 6]))
    rng = np.random.default_rng(7)
    ph = rng.integers(0, 2, size=P.m).astype(np.uint8)
    Cp, C0 = two_phase(1.0, 10.0, 0.3)
    G, _ = green.gamma_periodised(P, C0, "dirichlet")
    Ceff, _ = scheme.effective_stiffness(P, G, Cp, C0, ph, tol=1e-13, max_iter=3000)
    Cm = green.voigt_stiffness_to_mandel(Cp)
    f = ph.mean()
    voigt = (1 - f) * Cm[0] + f * Cm[1]
    reuss = np.linalg.inv((1 - f) * np.linalg.inv(Cm[0]) + f * np.linalg.inv(Cm[1]))
    Ce = green.voigt_stiffness_to_mandel(0.5 * (Ceff + Ceff.T))
    assert np.linalg.eigvalsh(voigt - Ce).min() > -1e-10
    assert np.linalg.eigvalsh(Ce - reuss).min() > -1e-10


def test_ls_and_variational_differ_for_dlvp_only():
    """Remark (constants): eps_M - Gamma^p C0 eps_M = eps0 holds only for the
    Dirichlet space.  Check on the fixed point: the residual of the identity
    vanishes for Dirichlet and not for dlVP.  Odd axes: there the Dirichlet
    multiplier is even and no real-part projection is involved."""
    P = Pattern(np.diag([5, 5, 7]))
    rng = np.random.default_rng(8)
    ph = rng.integers(0, 2, size=P.m).astype(np.uint8)
    Cp, C0 = two_phase(1.0, 10.0, 0.3)
    C0m = green.voigt_stiffness_to_mandel(C0)
    from oracle import dft
    eps0 = np.array([1.0, 0, 0, 0, 0, 0])
    out = {}
    for kind, params in [("dirichlet", {}), ("dlvp", {"alpha": [0.75] * 3})]:
        G, _ = green.gamma_periodised(P, C0, kind, params)
        res = scheme.basic_scheme(P, G, Cp, C0, ph, eps0, tol=1e-14, max_iter=3000)
        eps = res["E"] + green.voigt_strain_to_mandel(eps0)
        GCe = dft.pattern_idft(P, np.einsum("bij,bj->bi", G @ C0m, dft.pattern_dft(P, eps))).real
        out[kind] = np.abs(eps - GCe - green.voigt_strain_to_mandel(eps0)).max()
    assert out["dirichlet"] < 1e-12
    assert out["dlvp"] > 1e-4


# ----------------------------------------------------- variational (VE) ---
def test_variational_iterates_equal_ls_for_dirichlet():
    """Remark (constants): for the Dirichlet space Gamma^p C0 fixes compatible
    fields, so the strain-update (variational) iterates equal the polarisation
    (Lippmann-Schwinger) iterates one by one.  Odd axes: no real-part projection."""
    P = Pattern(np.diag([5, 5, 7]))
    rng = np.random.default_rng(11)
    ph = rng.integers(0, 2, size=P.m).astype(np.uint8)
    Cp, C0 = two_phase(1.0, 10.0, 0.3)
    eps0 = np.array([0.3, -0.2, 0.1, 0.4, -0.1, 0.25])
    G, _ = green.gamma_periodised(P, C0, "dirichlet")
    a = scheme.basic_scheme(P, G, Cp, C0, ph, eps0, n_iter=12)
    b = scheme.variational_scheme(P, G, Cp, C0, ph, eps0, n_iter=12)
    np.testing.assert_allclose(b["history"], a["history"], rtol=1e-10)
    np.testing.assert_allclose(b["E"], a["E"], atol=1e-12)


@pytest.mark.parametrize("kind,params", [("dlvp", {"alpha": [0.75] * 3}), ("box", BOX4),
                                         ("dirichlet_modified", {})])
def test_variational_fixed_point_equals_dense_solve(kind, params):
    """The strain-update limit solves eq. (pde_coefficients_variational): compare
    with a dense solve in the range of the Green multiplier, assembled from the
    Fourier matrix written out entry by entry.  The Box multiplier has small
    eigenvalues on its range, where the strain update contracts slowly; there
    the comparison allows the iteration error r / (1 - rho), rho estimated from
    the last residuals."""
    M = [[4, 1, 0], [0, 4, 0], [0, 0, 2]]
    P = Pattern(M)
    rng = np.random.default_rng(12)
    ph = rng.integers(0, 2, size=P.m).astype(np.uint8)
    Cp, C0 = two_phase(1.0, 5.0, 0.3)
    eps0 = np.array([0.2, -0.1, 0.05, 0.3, 0.1, -0.2])
    G, _ = green.gamma_periodised(P, C0, kind, params)
    res = scheme.variational_scheme(P, G, Cp, C0, ph, eps0, tol=1e-15, max_iter=20000)
    Ynum = P.point_numerators()
    by_point = {tuple(Fraction(int(v), P.m) for v in row): int(p) for row, p in zip(Ynum, ph)}
    Y, Ed = scheme.dense_variational_point(M, C0, kind, params, Cp, by_point, eps0)
    key = {tuple(Fraction(int(v), P.m) for v in row): i for i, row in enumerate(Ynum)}
    from oracle.lattice import brute_force_points
    order = [key[y] for y in brute_force_points(M)]
    h = res["history"]
    rho = min(h[-1] / h[-2], 1 - 1e-12)
    bound = max(1e-10, 10 * h[-1] / (1 - rho)) * max(1, np.abs(Ed).max())
    assert bound < 1e-5
    np.testing.assert_allclose(res["E"][order], Ed, atol=bound)


@pytest.mark.parametrize("kind,params", KERNELS)
def test_variational_laminate_closed_form(kind, params):
    """The laminate's exact fields live on frequencies (h1, 0, 0), where every
    kernel's Gamma^p equals Gamma0, so the variational fixed point is the same
    closed form as the Lippmann-Schwinger one."""
    C, _ = _laminate_closed_form()
    P = Pattern(np.diag([16, 16, 16]))
    ph = (P.points()[:, 0] >= 0).astype(np.uint8)
    Cp, C0 = two_phase(1.0, 10.0, 0.3)
    G, _ = green.gamma_periodised(P, C0, kind, params)
    res = scheme.variational_scheme(P, G, Cp, C0, ph, np.array([1.0, 0, 0, 0, 0, 0]), tol=1e-12, max_iter=200)
    np.testing.assert_allclose(res["sigma_voigt"], C[:, 0], rtol=1e-10, atol=1e-12)


def test_variational_differs_from_ls_for_dlvp():
    """The two discretisations coincide only on the Dirichlet space: their
    effective stresses differ for dlVP and agree for Dirichlet (odd axes)."""
    P = Pattern(np.diag([5, 5, 7]))
    rng = np.random.default_rng(13)
    ph = rng.integers(0, 2, size=P.m).astype(np.uint8)
    Cp, C0 = two_phase(1.0, 10.0, 0.3)
    eps0 = np.array([1.0, 0, 0, 0, 0, 0])
    d = {}
    for kind, params in [("dirichlet", {}), ("dlvp", {"alpha": [0.75] * 3})]:
        G, _ = green.gamma_periodised(P, C0, kind, params)
        a = scheme.basic_scheme(P, G, Cp, C0, ph, eps0, tol=1e-14, max_iter=5000)["sigma_voigt"]
        b = scheme.variational_scheme(P, G, Cp, C0, ph, eps0, tol=1e-14, max_iter=5000)["sigma_voigt"]
        d[kind] = np.abs(a - b).max() / np.abs(a).max()
    assert d["dirichlet"] < 1e-11
    assert d["dlvp"] > 1e-4


# ---------------------------------------------------------------------------
# conjugate gradients for the Dirichlet kernel (scheme.conjugate_gradient)
# ---------------------------------------------------------------------------
def _cg_problem(M, kind, params, contrast=20.0, seed=11):
    P = Pattern(M)
    rng = np.random.default_rng(seed)
    ph = rng.integers(0, 2, size=P.m).astype(np.uint8)
    Cp, C0 = two_phase(1.0, contrast, 0.3)
    G, _ = green.gamma_periodised(P, C0, kind, params)
    return P, ph, Cp, C0, G


@pytest.mark.parametrize("M", [[[5, 1, 0], [0, 3, 0], [0, 0, 1]], [[3, 1, 0], [-1, 2, 1], [0, 1, 4]]])
def test_cg_limit_equals_dense_solve(M):
    """CG converges to the solution of eq. (pde_coefficients) assembled densely
    from the Fourier matrix written out entry by entry (Dirichlet, m odd)."""
    kind, params = "dirichlet", {}
    P, ph, Cp, C0, G = _cg_problem(M, kind, params, 20.0, 4)
    assert P.m % 2 == 1
    eps0 = np.array([0.2, -0.1, 0.05, 0.3, 0.1, -0.2])
    res = scheme.conjugate_gradient(P, G, Cp, C0, ph, eps0, tol=1e-14, max_iter=500)
    Ynum = P.point_numerators()
    by_point = {tuple(Fraction(int(v), P.m) for v in row): int(p) for row, p in zip(Ynum, ph)}
    _, Ed = scheme.dense_fixed_point(M, C0, kind, params, Cp, by_point, eps0)
    key = {tuple(Fraction(int(v), P.m) for v in row): i for i, row in enumerate(Ynum)}
    from oracle.lattice import brute_force_points
    order = [key[y] for y in brute_force_points(M)]
    np.testing.assert_allclose(res["E"][order], Ed, atol=1e-11 * max(1, np.abs(Ed).max()))


@pytest.mark.parametrize("M", [np.diag([5, 5, 7]), [[3, 1, 0], [-1, 2, 1], [0, 1, 4]]])
def test_cg_limit_equals_basic_scheme_for_dirichlet(M):
    """Without Nyquist faces (odd m) the Dirichlet operator G C0 is a projection
    and the variational and Lippmann-Schwinger solutions coincide
    (Remark (constants)); CG gets there with far fewer applications."""
    P, ph, Cp, C0, G = _cg_problem(M, "dirichlet", {}, 100.0)
    assert P.m % 2 == 1
    eps0 = np.array([1.0, 0.0, 0.0, 0.0, 0.5, 0.0])
    a = scheme.basic_scheme(P, G, Cp, C0, ph, eps0, tol=1e-13, max_iter=20000)
    b = scheme.conjugate_gradient(P, G, Cp, C0, ph, eps0, tol=1e-13, max_iter=2000)
    np.testing.assert_allclose(b["sigma_voigt"], a["sigma_voigt"], rtol=1e-10)
    np.testing.assert_allclose(b["E"], a["E"], atol=1e-9)
    assert b["iterations"] * 3 < a["iterations"]


def test_cg_directions_conjugate_and_residuals_orthogonal():
    """The defining properties of CG: directions conjugate in C, <p_i, C p_j> = 0,
    and residuals C0-orthogonal, <z_i, C0 z_j> = 0 (equivalently <R_i, z_j> = 0),
    for i != j (a wrong alpha or beta breaks both)."""
    P, ph, Cp, C0, G = _cg_problem(np.diag([5, 5, 7]), "dirichlet", {}, 10.0)
    res = scheme.conjugate_gradient(P, G, Cp, C0, ph, np.array([1.0, 0, 0, 0, 0, 0]), n_iter=7, trace=True)
    C = scheme.stiffness_field(Cp, ph)
    ps, Rs, zs = res["trace"]["p"], res["trace"]["R"], res["trace"]["z"]
    assert len(ps) == 6
    Cps = [np.einsum("yij,yj->yi", C, p) for p in ps]
    for i in range(6):
        for j in range(i):
            pij = abs(np.sum(ps[i] * Cps[j])) / np.sqrt(np.sum(ps[i] * Cps[i]) * np.sum(ps[j] * Cps[j]))
            rij = abs(np.sum(Rs[i] * zs[j])) / np.sqrt(abs(np.sum(Rs[i] * zs[i]) * np.sum(Rs[j] * zs[j])))
            assert pij < 1e-8 and rij < 1e-8, (i, j, pij, rij)


def test_cg_energy_error_decreases_and_finite_termination():
    """CG minimises the C-energy of the error over growing Krylov spaces: the
    energy error never grows, and on a tiny pattern (18 unknowns) the solution
    is reached to rounding within 19 applications."""
    P, ph, Cp, C0, G = _cg_problem(np.diag([5, 5, 5]), "dirichlet", {}, 10.0)
    eps0 = np.array([0.3, 0.1, -0.2, 0.0, 0.4, 0.1])
    ref = scheme.conjugate_gradient(P, G, Cp, C0, ph, eps0, tol=1e-15, max_iter=3000)
    C = scheme.stiffness_field(Cp, ph)
    errs = []
    for n in range(1, 25):
        Ek = scheme.conjugate_gradient(P, G, Cp, C0, ph, eps0, n_iter=n)["E"]
        d = Ek - ref["E"]
        errs.append(np.sum(d * np.einsum("yij,yj->yi", C, d)))
    assert all(b <= a * (1 + 1e-9) + 1e-28 for a, b in zip(errs, errs[1:]))
    Pt, pht, Cpt, C0t, Gt = _cg_problem([[3, 1, 0], [0, 1, 0], [0, 0, 1]], "dirichlet", {}, 50.0)
    assert Pt.m == 3
    r = scheme.conjugate_gradient(Pt, Gt, Cpt, C0t, pht, eps0, tol=1e-13, max_iter=100)
    assert r["iterations"] <= 19 and r["history"][-1] <= 1e-13
