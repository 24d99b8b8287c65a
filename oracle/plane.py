"""The two-dimensional problem: patterns P(M) of 2x2 integer matrices M.

Test infrastructure (oracle); see the package docstring.

The paper states its theory for d = 2 and 3 (Sec. 2.1, Sec. 3) and runs its
numerical study in two dimensions (Sec. 4).  In d = 2 strains and stresses are
symmetric 2x2 tensors, written here as Mandel 3-vectors (t11, t22, sqrt2 t12),
so the Frobenius product of Sec. 3.1 is the Euclidean one.  Stiffness tensors
with minor and major symmetry are 3x3 symmetric Mandel matrices.  At the
library boundary they are Voigt (11, 22, 12): strains with engineering shear
(gamma12 = 2 eps12), stresses and stiffness matrices with tensor components.

Green operator in d = 2, Def. (projection), eq. (gamma):
    Gamma0_k tau = sym(k (x) K^{-1} tau k),   K_im = sum_jl C0_ijlm k_j k_l,
the same derivation as in three dimensions with 2-vectors k and a 2x2
acoustic tensor; Gamma0_0 = 0.

The periodised operator of Def. (gamma_tilde_fourier) with orthonormalised
translates, the Basic Scheme of Sec. 4 and the effective stress follow the
three-dimensional modules (green.py, scheme.py) with d = 2; the generating
function weights g and their alias offsets are the d-general ones of green.py.
"""
from __future__ import annotations

import numpy as np

from . import dft
from . import green
from .lattice import Pattern

SQ2 = np.sqrt(2.0)
# Mandel / Voigt component order in d = 2: (11, 22, 12)
PAIRS2 = [(0, 0), (1, 1), (0, 1)]
MANDEL_W2 = np.array([1.0, 1.0, SQ2])


# ---------------------------------------------------------------------------
# Voigt <-> Mandel <-> tensor, d = 2
# ---------------------------------------------------------------------------
def voigt_stiffness_to_mandel(Cv):
    """C_mandel = W C_voigt W, W = diag(1, 1, sqrt2)."""
    Cv = np.asarray(Cv, dtype=np.float64)
    return Cv * MANDEL_W2[..., :, None] * MANDEL_W2[..., None, :]


def voigt_strain_to_mandel(e):
    """Engineering shear gamma12 = 2 eps12  ->  Mandel sqrt2 eps12 = gamma12 / sqrt2."""
    e = np.asarray(e, dtype=np.float64)
    return e * np.array([1.0, 1.0, 1.0 / SQ2])


def mandel_strain_to_voigt(e):
    e = np.asarray(e, dtype=np.float64)
    return e * np.array([1.0, 1.0, SQ2])


def mandel_stress_to_voigt(s):
    """Mandel sqrt2 s12 -> tensor component s12."""
    s = np.asarray(s, dtype=np.float64)
    return s * np.array([1.0, 1.0, 1.0 / SQ2])


def mandel_to_tensor(v):
    """Mandel 3-vectors (..., 3) -> symmetric tensors (..., 2, 2)."""
    v = np.asarray(v, dtype=np.float64)
    t = np.zeros(v.shape[:-1] + (2, 2))
    t[..., 0, 0] = v[..., 0]
    t[..., 1, 1] = v[..., 1]
    t[..., 0, 1] = t[..., 1, 0] = v[..., 2] / SQ2
    return t


def tensor_to_mandel(t):
    t = np.asarray(t, dtype=np.float64)
    return np.stack([t[..., 0, 0], t[..., 1, 1], SQ2 * 0.5 * (t[..., 0, 1] + t[..., 1, 0])], axis=-1)


def voigt_stiffness_to_tensor(Cv):
    """C_ijkl (2,2,2,2) from a 3x3 Voigt matrix (tensor components)."""
    Cv = np.asarray(Cv, dtype=np.float64)
    idx = np.zeros((2, 2), dtype=np.int64)
    for I, (i, j) in enumerate(PAIRS2):
        idx[i, j] = idx[j, i] = I
    C4 = np.zeros((2, 2, 2, 2))
    for i in range(2):
        for j in range(2):
            for k in range(2):
                for l in range(2):
                    C4[i, j, k, l] = Cv[idx[i, j], idx[k, l]]
    return C4


# ---------------------------------------------------------------------------
# Green operator, Def. (projection), d = 2
# ---------------------------------------------------------------------------
def gamma0(C0_voigt, k):
    """Gamma0_k as 3x3 Mandel matrices for frequencies k (..., 2); 0 at k = 0.

    Column J is the action tau -> sym(k (x) K^{-1} tau k) on Mandel basis
    vector J (eq. (gamma) with the 2x2 acoustic tensor).
    """
    C4 = voigt_stiffness_to_tensor(C0_voigt)
    k = np.asarray(k, dtype=np.float64)
    flat = k.reshape(-1, 2)
    out = np.zeros((flat.shape[0], 3, 3))
    nz = np.any(flat != 0, axis=1)
    kk = flat[nz]
    if len(kk):
        K = np.einsum("ijlm,nj,nl->nim", C4, kk, kk)
        N = np.linalg.inv(K)
        for J in range(3):
            e = np.zeros(3)
            e[J] = 1.0
            tau = mandel_to_tensor(e)
            tk = np.einsum("ab,nb->na", tau, kk)
            w = np.einsum("nab,nb->na", N, tk)
            res = 0.5 * (kk[:, :, None] * w[:, None, :] + w[:, :, None] * kk[:, None, :])
            out[nz, :, J] = tensor_to_mandel(res)
    return out.reshape(k.shape[:-1] + (3, 3))


def gamma_at_frequencies(P: Pattern, C0_voigt, kind, params, H, chunk=4096):
    """Gamma^p at integer frequencies H (n, 2), Def. (gamma_tilde_fourier) with
    orthonormalised translates: sum_z w(x+z) Gamma0_{h+M^T z} / sum_z w(x+z),
    w = g^2, x = M^{-T} h, h first reduced into G(M^T).  Returns (Gamma, bracket sums)."""
    if P.d != 2:
        raise ValueError("two-dimensional patterns only")
    params = params or {}
    H, Xn = P.reduce_frequencies(H)
    X = Xn.astype(np.float64) / P.m
    Z = green.alias_offsets(kind, params, 2)
    MT = np.array(P.MT, dtype=np.int64)
    g = green.weight_fn(kind, params)
    n = len(H)
    out = np.zeros((n, 3, 3))
    den_all = np.zeros(n)
    for s in range(0, n, chunk):
        h = H[s:s + chunk]
        x = X[s:s + chunk]
        num = np.zeros((len(h), 3, 3))
        den = np.zeros(len(h))
        for z in Z:
            w = g(x + z) ** 2
            sel = w > 0
            if not np.any(sel):
                continue
            k = h[sel] + (MT @ z)[None, :]
            num[sel] += w[sel, None, None] * gamma0(C0_voigt, k)
            den[sel] += w[sel]
        if kind == green.BOX and params.get("tail"):
            tn, td = green.box_tail(P, C0_voigt, params, h, x, gamma_fn=gamma0)
            num += tn
            den += td
        ok = den > 0
        out[s:s + chunk][ok] = num[ok] / den[ok, None, None]
        den_all[s:s + chunk] = den
    out[np.all(H == 0, axis=1)] = 0.0   # Gamma0_0 = 0: zero-mean fields
    return out, den_all


def gamma_periodised(P: Pattern, C0_voigt, kind, params=None):
    """Gamma^p_h over all frequencies h(b), b in storage order."""
    H, _ = P.frequencies()
    return gamma_at_frequencies(P, C0_voigt, kind, params, H)


def gamma_symmetrised_at(P: Pattern, C0_voigt, kind, params, H):
    """(Gamma^p_h + Gamma^p_{-h}) / 2: the multiplier that keeps real fields real."""
    Gp, d1 = gamma_at_frequencies(P, C0_voigt, kind, params, H)
    Gm, d2 = gamma_at_frequencies(P, C0_voigt, kind, params, -np.asarray(H))
    return 0.5 * (Gp + Gm), np.minimum(d1, d2)


# ---------------------------------------------------------------------------
# Basic Scheme, Sec. 4, d = 2
# ---------------------------------------------------------------------------
def basic_scheme(P: Pattern, Gamma, C_phases_voigt, C0_voigt, phase, eps0_voigt,
                 tol=1e-10, max_iter=1000, E_init=None, n_iter=None):
    """Fixed point of eq. (pde_coefficients) in d = 2, polarisation form
    E^{k+1} = -Re F^{-1}[Gamma^p_h F[(C - C0):(E^k + eps0)]_h], with the Cauchy
    residual ||E^{k+1} - E^k|| / ||E^{k+1} + eps0|| and
    sigma_bar = (1/m) sum_y C(y):(E_y + eps0) (same readings as scheme.basic_scheme).

    Gamma : (m, 3, 3) Gamma^p in frequency storage order.
    Returns dict(E (m, 3) Mandel, sigma_voigt (3,), iterations, history).
    """
    m = P.m
    C = voigt_stiffness_to_mandel(np.asarray(C_phases_voigt, dtype=np.float64))[np.asarray(phase, np.int64)]
    Delta = C - voigt_stiffness_to_mandel(C0_voigt)[None]
    eps0 = voigt_strain_to_mandel(eps0_voigt)
    if E_init is None:
        E = np.zeros((m, 3))
    else:
        E = np.array(E_init, dtype=np.float64).reshape(m, 3)
        E = E - E.mean(axis=0, keepdims=True)
    history = []
    it = 0
    limit = n_iter if n_iter is not None else max_iter
    while it < limit:
        tau = np.einsum("yij,yj->yi", Delta, E + eps0)
        E_hat = -np.einsum("bij,bj->bi", Gamma, dft.pattern_dft(P, tau))
        E_new = dft.pattern_idft(P, E_hat).real
        r = np.sqrt(np.sum((E_new - E) ** 2)) / np.sqrt(np.sum((E_new + eps0) ** 2))
        E = E_new
        it += 1
        history.append(r)
        if n_iter is None and r <= tol:
            break
    sigma = np.einsum("yij,yj->i", C, E + eps0) / m
    return dict(E=E, sigma_voigt=mandel_stress_to_voigt(sigma), iterations=it, history=np.array(history))


def effective_stiffness(P: Pattern, Gamma, C_phases_voigt, C0_voigt, phase, tol=1e-10, max_iter=1000):
    """C^eff (3x3 Voigt): column j is sigma_bar for the unit Voigt load e_j (Sec. 3.1)."""
    Ceff = np.zeros((3, 3))
    its = []
    for j in range(3):
        e = np.zeros(3)
        e[j] = 1.0
        res = basic_scheme(P, Gamma, C_phases_voigt, C0_voigt, phase, e, tol=tol, max_iter=max_iter)
        Ceff[:, j] = res["sigma_voigt"]
        its.append(res["iterations"])
    return Ceff, its
