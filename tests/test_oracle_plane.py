"""Pins for the two-dimensional oracle (oracle/plane.py): the d = 2 form of
Def. (projection), Def. (gamma_tilde_fourier) and the Basic Scheme of Sec. 4.

Each pin is fixed by something other than the 2-D code itself: the textbook
laminate formulas, the projection property of the Dirichlet operator, the
exactness for homogeneous material, and the three-dimensional oracle (pinned
on its own) run on the embedded pattern blockdiag(M, 1), whose frequencies all
have k3 = 0, so that in-plane loads give plane strain.
"""
import numpy as np
import pytest

import lsh_inputs as li
from oracle import green, plane, scheme
from oracle.lattice import Pattern

BOX2 = {"Xi": np.array([[1, 0, 1, 1], [0, 1, 1, -1]], float), "R": 4}
KERNELS = [("dirichlet", {}), ("dirichlet_modified", {}), ("dlvp", {"alpha": [0.4, 0.7]}), ("box", BOX2)]


def two_phase(E1=1.0, E2=10.0, nu=0.3):
    Cp = np.stack([li.isotropic_voigt_plane(E1, nu), li.isotropic_voigt_plane(E2, nu)])
    return Cp, li.mean_reference(Cp)


def test_plane_strain_stiffness_is_in_plane_block():
    C3 = li.isotropic_voigt(2.0, 0.25)
    C2 = li.isotropic_voigt_plane(2.0, 0.25)
    lam, mu = li.lame(2.0, 0.25)
    np.testing.assert_allclose(C2, [[lam + 2 * mu, lam, 0], [lam, lam + 2 * mu, 0], [0, 0, mu]], rtol=1e-15)
    np.testing.assert_array_equal(C2, C3[np.ix_([0, 1, 5], [0, 1, 5])])


@pytest.mark.parametrize("M", [[[8, 8], [-8, 8]], [[5, 2], [1, 4]]])
def test_dirichlet_gamma_is_c0_projection(M):
    """Dirichlet: Gamma^p_h = Gamma0_h at the representative, and Gamma0 C0 is a
    projection (Def. (projection)): G C0 G = G at every bin, G = 0 at h = 0."""
    P = Pattern(M)
    _, C0 = two_phase()
    G, den = plane.gamma_periodised(P, C0, "dirichlet")
    C0m = plane.voigt_stiffness_to_mandel(C0)
    assert np.all(den > 0)
    GCG = np.einsum("bij,jk,bkl->bil", G, C0m, G)
    np.testing.assert_allclose(GCG, G, atol=1e-14)
    # rank 2 (the compatible strains of a plane wave) at every nonzero bin
    H, _ = P.frequencies()
    nz = np.any(H != 0, axis=1)
    ranks = [np.linalg.matrix_rank(g, tol=1e-10) for g in G[nz]]
    assert set(ranks) == {2}
    assert np.all(G[~nz] == 0)


def test_dlvp_gamma_is_not_a_projection():
    """The weighted alias average of projections is no projection: catches a
    weight that collapses to a single alias."""
    P = Pattern([[8, 8], [-8, 8]])
    _, C0 = two_phase()
    G, _ = plane.gamma_periodised(P, C0, "dlvp", {"alpha": [0.8, 0.8]})
    C0m = plane.voigt_stiffness_to_mandel(C0)
    GCG = np.einsum("bij,jk,bkl->bil", G, C0m, G)
    assert np.abs(GCG - G).max() > 1e-3


@pytest.mark.parametrize("kind,params", KERNELS)
def test_homogeneous_material_one_iteration(kind, params):
    P = Pattern([[6, 2], [0, 5]])
    Cp = np.stack([li.isotropic_voigt_plane(3.0, 0.2)])
    C0 = li.isotropic_voigt_plane(1.0, 0.3)
    G, _ = plane.gamma_periodised(P, C0, kind, params)
    eps0 = np.array([0.3, -0.1, 0.2])
    res = plane.basic_scheme(P, G, Cp, C0, np.zeros(P.m, np.uint8), eps0, tol=1e-12)
    assert res["iterations"] == 1
    assert np.abs(res["E"]).max() < 1e-15
    np.testing.assert_allclose(res["sigma_voigt"], Cp[0] @ eps0, rtol=1e-14)


def _laminate_plane(E=(1.0, 10.0), nu=0.3):
    """Rank-one laminate, f = 1/2, normal e1, in plane strain: the in-plane
    entries of the textbook laminate formulas (the normal stress and shear
    tractions are continuous, the tangential strain is uniform)."""
    lam = np.array([li.lame(e, nu)[0] for e in E])
    mu = np.array([li.lame(e, nu)[1] for e in E])
    Pm = lam + 2 * mu
    av = lambda v: v.mean()
    C11 = 1 / av(1 / Pm)
    C12 = av(lam / Pm) * C11
    C22 = av(Pm - lam ** 2 / Pm) + av(lam / Pm) ** 2 * C11
    return np.array([[C11, C12, 0], [C12, C22, 0], [0, 0, 1 / av(1 / mu)]])


@pytest.mark.parametrize("kind,params", KERNELS)
def test_laminate_closed_form(kind, params):
    P = Pattern(np.diag([16, 16]))
    ph = li.laminate_phase(P.points(), 0)
    Cp, C0 = two_phase()
    G, _ = plane.gamma_periodised(P, C0, kind, params)
    Ceff, its = plane.effective_stiffness(P, G, Cp, C0, ph, tol=1e-12)
    ref = _laminate_plane()
    np.testing.assert_allclose(Ceff, ref, rtol=0, atol=1e-11 * np.abs(ref).max())


def _embed_params(kind, params):
    if kind == "dlvp":
        return {"alpha": list(params["alpha"]) + [0.5]}
    if kind == "box":
        Xi = np.asarray(params["Xi"], float)
        Xi3 = np.zeros((3, Xi.shape[1] + 1))
        Xi3[:2, :Xi.shape[1]] = Xi
        Xi3[2, -1] = 1.0
        return {"Xi": Xi3, "R": params["R"]}
    return params


@pytest.mark.parametrize("M", [[[4, 1], [0, 4]], [[3, 1], [-1, 4]]])
@pytest.mark.parametrize("kind,params", KERNELS)
def test_matches_three_dimensional_oracle_on_embedded_pattern(M, kind, params):
    """d = 2 against d = 3 on blockdiag(M, 1): all frequencies have k3 = 0, so the
    3-D Green operator acts as the plane-strain one; in-plane loads on
    isotropic phases then leave E33 = E13 = E23 = 0.  E, sigma_bar and the
    residual history agree (a dropped term, a wrong sqrt2 or a transposed k
    anywhere in the 2-D code fails here)."""
    P2 = Pattern(M)
    M3 = np.zeros((3, 3), dtype=np.int64)
    M3[:2, :2] = M
    M3[2, 2] = 1
    P3 = Pattern(M3)
    rng = np.random.default_rng(7)
    ph2 = rng.integers(0, 2, size=P2.m).astype(np.uint8)
    # map the 2-D points onto the 3-D storage order (y3 = 0 for every point)
    y2 = {tuple(r): i for i, r in enumerate(P2.point_numerators().tolist())}
    y3 = P3.point_numerators()
    assert np.all(y3[:, 2] == 0)
    q = np.array([y2[(r[0], r[1])] for r in y3.tolist()])
    ph3 = ph2[q]
    E = (1.0, 10.0)
    Cp2 = np.stack([li.isotropic_voigt_plane(e, 0.3) for e in E])
    Cp3 = np.stack([li.isotropic_voigt(e, 0.3) for e in E])
    C02, C03 = li.mean_reference(Cp2), li.mean_reference(Cp3)
    eps2 = np.array([0.2, -0.3, 0.5])
    eps3 = np.array([0.2, -0.3, 0.0, 0.0, 0.0, 0.5])
    G2, _ = plane.gamma_periodised(P2, C02, kind, params)
    G3, _ = green.gamma_periodised(P3, C03, kind, _embed_params(kind, params))
    r2 = plane.basic_scheme(P2, G2, Cp2, C02, ph2, eps2, n_iter=12)
    r3 = scheme.basic_scheme(P3, G3, Cp3, C03, ph3, eps3, n_iter=12)
    np.testing.assert_allclose(r2["history"], r3["history"], rtol=1e-11)
    np.testing.assert_allclose(r2["sigma_voigt"], r3["sigma_voigt"][[0, 1, 5]], rtol=1e-12, atol=1e-14)
    E3 = r3["E"]
    assert np.abs(E3[:, 2:5]).max() < 1e-13
    np.testing.assert_allclose(r2["E"][q], E3[:, [0, 1, 5]], atol=1e-13)


def test_effective_tensor_symmetric():
    P = Pattern([[8, 8], [-8, 8]])
    rng = np.random.default_rng(3)
    ph = rng.integers(0, 2, size=P.m).astype(np.uint8)
    Cp, C0 = two_phase(1.0, 5.0)
    G, _ = plane.gamma_periodised(P, C0, "dlvp", {"alpha": [0.5, 0.5]})
    Ceff, _ = plane.effective_stiffness(P, G, Cp, C0, ph, tol=1e-13, max_iter=3000)
    assert np.abs(Ceff - Ceff.T).max() < 1e-9 * np.abs(Ceff).max()
