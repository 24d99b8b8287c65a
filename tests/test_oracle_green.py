"""Pins for the oracle's Green operators and generating functions (Secs. 2.2, 3.1, 3.2)."""
import numpy as np
import pytest

from oracle import green
from oracle.lattice import Pattern
import lsh_inputs as li

RNG = np.random.default_rng(11)


def random_stiffness(rng):
    """A random elliptic C0 in SSym_3 (Voigt form): SPD in Mandel form."""
    A = rng.standard_normal((6, 6))
    Cm = A @ A.T + 3 * np.eye(6)
    return green.mandel_stiffness_to_voigt(Cm)


def mandel_sqrt(Cv):
    Cm = green.voigt_stiffness_to_mandel(Cv)
    w, Q = np.linalg.eigh(Cm)
    return Q @ np.diag(np.sqrt(w)) @ Q.T, Cm


# ---------------------------------------------------------------- Gamma0 ---
def test_isotropic_closed_form_equals_general():
    lam, mu = li.lame(3.7, 0.27)
    C0 = li.isotropic_voigt(3.7, 0.27)
    k = RNG.standard_normal((50, 3))
    np.testing.assert_allclose(green.gamma0(C0, k), green.gamma0_isotropic(lam, mu, k), atol=1e-13)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_gamma0_projection_properties(seed):
    """Gamma0_k C0 is a projection (the property quoted from Vondrejc et al. in
    the proof of the projection theorem, Sec. 3.2), fixes compatible strains
    sym(k (x) u) and annihilates equilibrated stresses (sigma k = 0)."""
    rng = np.random.default_rng(seed)
    C0 = random_stiffness(rng)
    C0m = green.voigt_stiffness_to_mandel(C0)
    for _ in range(20):
        k = rng.standard_normal(3)
        G = green.gamma0(C0, k[None])[0]
        GC = G @ C0m
        np.testing.assert_allclose(GC @ GC, GC, atol=1e-13)
        u = rng.standard_normal(3)
        eps = green.tensor_to_mandel(0.5 * (np.outer(k, u) + np.outer(u, k)))
        np.testing.assert_allclose(GC @ eps, eps, atol=1e-13)
        # equilibrated: sigma with sigma k = 0
        n = k / np.linalg.norm(k)
        t1 = np.cross(n, rng.standard_normal(3))
        t1 /= np.linalg.norm(t1)
        t2 = np.cross(n, t1)
        s = rng.standard_normal(3)
        sig = s[0] * np.outer(t1, t1) + s[1] * np.outer(t2, t2) + s[2] * (np.outer(t1, t2) + np.outer(t2, t1))
        np.testing.assert_allclose(G @ green.tensor_to_mandel(sig), 0, atol=1e-13)
        # even, homogeneous of degree 0, symmetric
        np.testing.assert_allclose(green.gamma0(C0, -k[None])[0], G, atol=1e-14)
        np.testing.assert_allclose(green.gamma0(C0, 7.3 * k[None])[0], G, atol=1e-13)
        np.testing.assert_allclose(G, G.T, atol=1e-14)


def test_gamma0_zero_frequency():
    C0 = li.isotropic_voigt(1.0, 0.3)
    assert np.all(green.gamma0(C0, np.zeros((1, 3))) == 0)


# ---------------------------------------------------- generating functions ---
def test_sinc_convention_against_quadrature():
    """Box spline weights: the Fourier transform of the centred box spline of
    Sec. 2.2 at 2 pi x is prod sinc(pi xi^T x) with sinc t = sin t / t.  Check
    by quadrature of the hat function B_{(1,1)} (1-D) and the unit box."""
    t = np.linspace(-1, 1, 200001)
    hat = 1 - np.abs(t)
    box = (np.abs(t) < 0.5).astype(float)
    for x in [0.0, 0.13, 0.5, 0.77, 1.9]:
        ft_hat = np.trapezoid(hat * np.cos(2 * np.pi * x * t), t)
        ft_box = np.trapezoid(box * np.cos(2 * np.pi * x * t), t)
        assert abs(green.g_box(np.array([[x, 0, 0]]), np.array([[1.0, 1.0], [0, 0], [0, 0]]))[0] - ft_hat) < 1e-6
        assert abs(green.g_box(np.array([[x, 0, 0]]), np.array([[1.0], [0], [0]]))[0] - ft_box) < 2e-5


def test_trapezoid_is_the_box_spline_of_sec22():
    """g_alpha = B_Xi with Xi = (diag alpha, I): Fourier transform at 2 pi y is
    sinc(pi alpha y) sinc(pi y); checked by quadrature of the trapezoid."""
    t = np.linspace(-1.5, 1.5, 300001)
    for a in [0.1, 0.5, 0.75, 1.0]:
        g = green.g_dlvp(np.stack([t, 0 * t, 0 * t], -1), [a, 0.3, 0.3])
        for y in [0.0, 0.31, 1.2]:
            ft = np.trapezoid(g * np.cos(2 * np.pi * y * t), t)
            assert abs(ft - np.sinc(a * y) * np.sinc(y)) < 1e-6


@pytest.mark.parametrize("alpha", [[0.0, 0.0, 0.0], [0.1, 0.2, 0.3], [0.75, 0.75, 0.75], [1.0, 0.5, 0.0]])
def test_dlvp_weights_admissible(alpha):
    """Admissibility (Sec. 2.2): g >= 0, g > 0 on the cube, sum_z g(x + z) = 1."""
    x = RNG.uniform(-0.5, 0.5, size=(400, 3))
    tot = sum(green.g_dlvp(x + np.array(z), alpha) for z in green.alias_offsets("dlvp", {}))
    np.testing.assert_allclose(tot, 1.0, atol=1e-14)
    assert np.all(green.g_dlvp(x, alpha) > 0)


def test_modified_dirichlet_is_dlvp_limit():
    x = RNG.uniform(-0.5, 0.5, size=(200, 3))
    x[:20, 0] = -0.5
    a = 1e-9
    np.testing.assert_allclose(green.g_dlvp(x, [a] * 3), green.weight_fn("dirichlet_modified", {})(x), atol=1e-8)


def test_box_order_zero_bracket_sum_closed_form():
    """sum_n sinc^2(pi (x + n)) = 1 (Xi = I, Brisard-Dormieux constant
    elements, Sec. 3.2): the truncated sum converges to 1 as R grows."""
    x = RNG.uniform(-0.5, 0.5, size=(50, 3))
    Xi = np.eye(3)
    errs = []
    for R in [2, 4, 8, 16]:
        Z = green.alias_offsets("box", {"R": R})
        s = sum(green.g_box(x + z, Xi) ** 2 for z in Z)
        errs.append(np.max(np.abs(s - 1)))
    assert all(b < a for a, b in zip(errs, errs[1:]))
    # 1-D tail bound: sum_{|n|>R} sinc^2 <= 2/(pi^2 (R - 1/2)); product of 3 axes
    assert errs[-1] < 3 * 2 / (np.pi ** 2 * 15.5)


# ------------------------------------------------------- periodised Gamma ---
@pytest.mark.parametrize("M", [np.diag([6, 6, 6]), [[4, 1, 0], [0, 4, 0], [0, 0, 2]], [[3, 1, 0], [-1, 2, 1], [0, 1, 4]]])
def test_dirichlet_coincides_with_gamma0_and_is_projection(M):
    """Thm. (CoincidenceGamma0GammaP) and the projection theorem: for the
    Dirichlet kernel Gamma^p_h = Gamma0_h and Gamma^p C0 is idempotent."""
    P = Pattern(M)
    C0 = random_stiffness(np.random.default_rng(5))
    C0m = green.voigt_stiffness_to_mandel(C0)
    G, den = green.gamma_periodised(P, C0, "dirichlet")
    H, _ = P.frequencies()
    np.testing.assert_allclose(G, green.gamma0(C0, H), atol=1e-13)
    GC = G @ C0m
    np.testing.assert_allclose(GC @ GC, GC, atol=1e-12)
    assert np.all(den == 1)


def test_dlvp_not_projection_but_exact_on_flat_top():
    """Projection theorem (Sec. 3.2): for a non-Dirichlet space Gamma^p C0 is
    not idempotent wherever aliases with different Gamma0 carry weight, while
    on the flat top |x_i| <= (1-alpha)/2 only z = 0 has weight and Gamma^p = Gamma0."""
    P = Pattern(np.diag([8, 8, 8]))
    C0 = li.isotropic_voigt(1.0, 0.3)
    C0m = green.voigt_stiffness_to_mandel(C0)
    alpha = [0.75] * 3
    G, _ = green.gamma_periodised(P, C0, "dlvp", {"alpha": alpha})
    H, Xn = P.frequencies()
    X = Xn / P.m
    flat = np.all(np.abs(X) <= 0.125, axis=1)
    np.testing.assert_allclose(G[flat], green.gamma0(C0, H[flat]), atol=1e-14)
    GC = G @ C0m
    defect = np.linalg.norm(GC @ GC - GC, axis=(1, 2))
    assert defect[~flat & np.any(H != 0, axis=1)].max() > 1e-3


@pytest.mark.parametrize("kind,params", [
    ("dirichlet", {}), ("dirichlet_modified", {}), ("dlvp", {"alpha": [0.3, 0.6, 0.9]}),
    ("box", {"Xi": np.array([[1, 0, 0, 1], [0, 1, 0, 1], [0, 0, 1, 0]], float), "R": 4}),
])
def test_spectral_bounds(kind, params):
    """Adjointness and boundedness theorems (Sec. 3.2): C0^{1/2} Gamma^p_h C0^{1/2}
    is symmetric with eigenvalues in [0, 1] (a weighted mean of orthogonal
    projections); for Dirichlet they are exactly 0 or 1."""
    P = Pattern([[4, 1, 0], [0, 4, 0], [0, 0, 3]])
    C0 = random_stiffness(np.random.default_rng(9))
    S, C0m = mandel_sqrt(C0)
    G, den = green.gamma_periodised(P, C0, kind, params)
    assert np.all(den > 0)
    A = S @ G @ S
    np.testing.assert_allclose(A, np.swapaxes(A, 1, 2), atol=1e-13)
    ev = np.linalg.eigvalsh(A)
    assert ev.min() > -1e-13 and ev.max() < 1 + 1e-13
    if kind == "dirichlet":
        assert np.all((np.abs(ev) < 1e-12) | (np.abs(ev - 1) < 1e-12))


@pytest.mark.parametrize("kind,params", [
    ("dirichlet_modified", {}), ("dlvp", {"alpha": [0.75] * 3}),
    ("box", {"Xi": np.array([[1, 0, 0, 1], [0, 1, 0, 1], [0, 0, 1, 0]], float), "R": 3}),
])
def test_even_kernels_are_hermitian(kind, params):
    """For even generating functions Gamma^p_{-h} = Gamma^p_h (real fields stay
    real).  The truncated Box sum is even only off the -1/2 faces: there the
    representative of -h is shifted and its alias box is not the mirror image."""
    P = Pattern([[4, 1, 0], [0, 4, 0], [0, 0, 2]])
    C0 = li.isotropic_voigt(2.0, 0.25)
    G, _ = green.gamma_periodised(P, C0, kind, params)
    Gs, _ = green.gamma_symmetrised(P, C0, kind, params)
    _, Xn = P.frequencies()
    face = np.any(2 * Xn == -P.m, axis=1)
    sel = ~face if kind == "box" else np.ones(P.m, bool)
    np.testing.assert_allclose(G[sel], Gs[sel], atol=1e-14)
    if kind == "box":
        assert np.abs(G - Gs).max() < 0.05


def test_dirichlet_even_axis_faces_not_hermitian():
    """The half-open cube makes the literal Dirichlet multiplier lose evenness
    on the -1/2 faces of even axes; the symmetrised table differs there only."""
    P = Pattern(np.diag([4, 4, 4]))
    C0 = li.isotropic_voigt(2.0, 0.25)
    G, _ = green.gamma_periodised(P, C0, "dirichlet")
    Gs, _ = green.gamma_symmetrised(P, C0, "dirichlet")
    _, Xn = P.frequencies()
    face = np.any(2 * Xn == -P.m, axis=1)
    diff = np.linalg.norm(G - Gs, axis=(1, 2))
    assert np.all(diff[~face] < 1e-15)
    assert diff[face].max() > 1e-2


def test_box_truncation_converges():
    """Gamma^p for the Box spline converges as the alias box grows (Sec. 4.2
    precomputes the bracket sums with a finite number of terms)."""
    P = Pattern([[4, 1, 0], [0, 4, 0], [0, 0, 2]])
    C0 = li.isotropic_voigt(1.0, 0.3)
    Xi = np.array([[1, 0, 0, 1], [0, 1, 0, 1], [0, 0, 1, 0]], float)
    prev = None
    deltas = []
    for R in [2, 4, 8, 16]:
        G, _ = green.gamma_periodised(P, C0, "box", {"Xi": Xi, "R": R})
        if prev is not None:
            deltas.append(np.abs(G - prev).max())
        prev = G
    # the weight tail beyond R decays like 1/R, so each doubling of R should
    # shrink the change by about half
    assert all(b < 0.75 * a for a, b in zip(deltas, deltas[1:]))


# ---------------------------------------------------------------------------
# tail of the Box alias sums (green.box_tail)
# ---------------------------------------------------------------------------
def _box_sum_by_moments(P, lam, mu, Xi, R, h):
    """Truncated Box alias sum at one frequency, evaluated independently of the
    oracle's loop: all aliases of [-R, R]^3 at once, isotropic C0 through the
    weighted moments of the alias directions (Gamma0 = S(n)/mu - r Q(n))."""
    M = np.array(P.M, float)
    hr, xn = P.reduce_frequencies(np.array([h]))
    hr = hr[0].astype(float)
    x = xn[0].astype(float) / P.m
    r1 = np.arange(-R, R + 1)
    A = np.zeros((3, 3))
    Q = np.zeros((3, 3, 3, 3))
    W = 0.0
    for z0 in r1:
        Z = np.array(np.meshgrid([z0], r1, r1, indexing="ij")).reshape(3, -1).T.astype(float)
        y = x[None] + Z
        w = np.ones(len(Z))
        for s in range(Xi.shape[1]):
            w *= np.sinc(y @ Xi[:, s]) ** 2
        k = hr[None] + Z @ M
        nk = np.linalg.norm(k, axis=1)
        ok = (w > 0) & (nk > 0)
        W += w.sum()
        n = k[ok] / nk[ok, None]
        A += np.einsum("p,pi,pj->ij", w[ok], n, n)
        Q += np.einsum("p,pi,pj,pk,pl->ijkl", w[ok], n, n, n, n)
    A /= W
    Q /= W
    rr = (lam + mu) / (mu * (lam + 2 * mu))
    G = np.zeros((6, 6))
    for J in range(6):
        e = np.zeros(6)
        e[J] = 1
        t = green.mandel_to_tensor(e)
        G[:, J] = green.tensor_to_mandel((0.5 / mu) * (A @ t + t @ A) - rr * np.einsum("ijkl,kl->ij", Q, t))
    return G


def test_box_slow_axes():
    assert green.box_slow_axes(np.array([[1, 0, 0, 1], [0, 1, 0, 1], [0, 0, 1, 0]])) == [(2, 2)]
    assert green.box_slow_axes(np.eye(3)) == [(0, 0), (1, 1), (2, 2)]
    assert green.box_slow_axes(np.array([[1, 0, 1, 0], [0, 1, 0, 1]])) == []
    assert green.box_slow_axes(np.array([[2, 0, 1], [0, 1, 1], [0, 0, 0]])) == []   # |xi_i| = 2: no closed form


def test_box_tail_restores_the_order_zero_denominator():
    """Xi = I: the weights are separable and their full sum is 1 (the closed form
    sum_n sinc^2(pi (x + n)) = 1); the corrected denominator misses only the
    corner tails, second order in the truncated mass."""
    P = Pattern(np.diag([6, 6, 6]))
    C0 = li.isotropic_voigt(2.0, 0.3)
    H = np.array([[3, 1, -2], [-3, -3, 2], [1, 2, 3]])
    for R in (2, 4, 8):
        _, d0 = green.gamma_at_frequencies(P, C0, "box", {"Xi": np.eye(3), "R": R}, H)
        _, d1 = green.gamma_at_frequencies(P, C0, "box", {"Xi": np.eye(3), "R": R, "tail": True}, H)
        e0, e1 = np.abs(1 - d0).max(), np.abs(1 - d1).max()
        assert e0 > 1e-3 / R and e1 < 5 * e0 ** 2, (R, e0, e1)


def test_box_tail_correction_converges_cubically():
    """Xi = {e1, e2, e3, e1+e2} (the 3-D workload's set; e3 is a slow axis):
    against the infinite sum (Richardson extrapolation of independently
    evaluated truncated sums at R = 16, 32, 64), plain truncation errs like
    1/R, the tail-corrected sum like R^-3."""
    P = Pattern(np.diag([8, 8, 8]))
    lam, mu = li.lame(5.5, 0.3)
    C0 = li.isotropic_voigt(5.5, 0.3)
    Xi = np.array([[1, 0, 0, 1], [0, 1, 0, 1], [0, 0, 1, 0]], float)
    H = [[3, 1, 4], [1, -3, 2]]
    T = {R: np.array([_box_sum_by_moments(P, lam, mu, Xi, R, h) for h in H]) for R in (16, 32, 64)}
    trunc16, _ = green.gamma_at_frequencies(P, C0, "box", {"Xi": Xi, "R": 16}, np.array(H))
    np.testing.assert_allclose(trunc16, T[16], atol=1e-13)        # the two evaluations agree
    S = (8 * T[64] - 6 * T[32] + T[16]) / 3
    err_t, err_c = [], []
    for R in (4, 8, 16):
        Tr, _ = green.gamma_at_frequencies(P, C0, "box", {"Xi": Xi, "R": R}, np.array(H))
        Co, _ = green.gamma_at_frequencies(P, C0, "box", {"Xi": Xi, "R": R, "tail": True}, np.array(H))
        err_t.append(np.abs(Tr - S).max())
        err_c.append(np.abs(Co - S).max())
    assert 1.6 < err_t[0] / err_t[1] < 2.5 and 1.6 < err_t[1] / err_t[2] < 2.5, err_t   # ~ 1/R
    assert err_c[0] / err_c[1] > 5 and err_c[1] / err_c[2] > 5, err_c                   # ~ R^-3
    assert err_c[2] < err_t[2] / 100
