"""Stiffness tensors, the Green operator and the periodised Green operator.

Test infrastructure (oracle); see the package docstring.

Conventions
-----------
Strains and stresses are 6-vectors in Mandel form
(t11, t22, t33, sqrt2 t23, sqrt2 t13, sqrt2 t12), so the Frobenius product of
Sec. 3.1 is the Euclidean product.  Fourth-order tensors with minor and major
symmetry (SSym_3, Sec. 3.1) are 6x6 symmetric Mandel matrices.  At the library
boundary strains are Voigt with engineering shear (2 t23 ...) and stresses and
stiffness matrices are Voigt (tensor components); conversions are below.

Green operator, Def. (projection), eq. (gamma):
    Gamma0_k tau = GradSym_k (conj(GradSym_k)^T C0 GradSym_k)^{-1} conj(GradSym_k)^T tau,
with GradSym_k u = (i/2)(k u^T + u k^T).  Writing it out:
conj(GradSym_k)^T tau = -i tau k, the bracket is the acoustic tensor
K_im = sum_jl C0_ijlm k_j k_l, hence Gamma0_k tau = sym(k (x) K^{-1} tau k).
Gamma0_0 = 0 (zero-mean compatible fields, Sec. 3.1).

Periodised Green operator, Def. (gamma_tilde_fourier):
    Gamma^p_h = m [ {Gamma0_k |c_k(f)|^2}_k ]^M_h     (bracket sum, eq. (bracketsum))
for orthonormal translates (the theorems of Sec. 3.2-3.3 assume them).  The
generating functions are given by a weight g on R^d with c_k(f) ~ g(M^{-T} k):
Def. (dlVP) for de la Vallee Poussin means and the Dirichlet kernel, and the
periodised pattern Box spline of Sec. 2.2 with c_k ~ prod_xi sinc(pi xi^T M^{-T} k).
Orthonormalising the translates (Lemma (FI:Props) c) divides |c_k|^2 by
m [|c|^2]_h, so with x = M^{-T} h and k = h + M^T z:
    Gamma^p_h = sum_z g(x+z)^2 Gamma0_{h+M^T z} / sum_z g(x+z)^2.
"""
from __future__ import annotations

import itertools

import numpy as np

from .lattice import Pattern

SQ2 = np.sqrt(2.0)
# Mandel / Voigt component order (11, 22, 33, 23, 13, 12)
PAIRS = [(0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1)]
MANDEL_W = np.array([1.0, 1.0, 1.0, SQ2, SQ2, SQ2])


# ---------------------------------------------------------------------------
# Voigt <-> Mandel <-> tensor
# ---------------------------------------------------------------------------
def voigt_stiffness_to_mandel(Cv):
    """C_mandel = W C_voigt W, W = diag(1,1,1,sqrt2,sqrt2,sqrt2)."""
    Cv = np.asarray(Cv, dtype=np.float64)
    return Cv * MANDEL_W[..., :, None] * MANDEL_W[..., None, :]


def mandel_stiffness_to_voigt(Cm):
    Cm = np.asarray(Cm, dtype=np.float64)
    return Cm / MANDEL_W[:, None] / MANDEL_W[None, :]


def voigt_strain_to_mandel(e):
    """Engineering shear gamma = 2 eps  ->  Mandel sqrt2 eps = gamma / sqrt2."""
    return np.asarray(e, dtype=np.float64) * np.array([1, 1, 1, 1 / SQ2, 1 / SQ2, 1 / SQ2])


def mandel_strain_to_voigt(e):
    return np.asarray(e, dtype=np.float64) * np.array([1, 1, 1, SQ2, SQ2, SQ2])


def mandel_stress_to_voigt(s):
    return np.asarray(s, dtype=np.float64) * np.array([1, 1, 1, 1 / SQ2, 1 / SQ2, 1 / SQ2])


def mandel_to_tensor(v):
    """6-vector(s) (..., 6) -> symmetric 3x3 tensor(s) (..., 3, 3)."""
    v = np.asarray(v)
    t = np.zeros(v.shape[:-1] + (3, 3), dtype=v.dtype)
    for I, (a, b) in enumerate(PAIRS):
        val = v[..., I] / (1.0 if a == b else SQ2)
        t[..., a, b] = val
        t[..., b, a] = val
    return t


def tensor_to_mandel(t):
    t = np.asarray(t)
    v = np.zeros(t.shape[:-2] + (6,), dtype=t.dtype)
    for I, (a, b) in enumerate(PAIRS):
        v[..., I] = t[..., a, b] * (1.0 if a == b else SQ2)
    return v


def voigt_stiffness_to_tensor(Cv):
    """C_ijkl from a Voigt stiffness matrix (whose entries are tensor components)."""
    Cv = np.asarray(Cv, dtype=np.float64)
    idx = np.zeros((3, 3), dtype=int)
    for I, (a, b) in enumerate(PAIRS):
        idx[a, b] = idx[b, a] = I
    C4 = np.empty((3, 3, 3, 3))
    for i, j, k, l in itertools.product(range(3), repeat=4):
        C4[i, j, k, l] = Cv[idx[i, j], idx[k, l]]
    return C4


# ---------------------------------------------------------------------------
# Green operator, Def. (projection)
# ---------------------------------------------------------------------------
def acoustic_tensor(C4, k):
    """K_im(k) = sum_jl C_ijlm k_j k_l, for k of shape (..., 3)."""
    k = np.asarray(k, dtype=np.float64)
    return np.einsum("ijlm,...j,...l->...im", C4, k, k)


def gamma0(C0_voigt, k):
    """Gamma0_k as 6x6 Mandel matrices for frequencies k (..., 3); 0 at k = 0.

    Built column by column from its action tau -> sym(k (x) K^{-1} tau k) on
    the Mandel basis (Def. (projection), eq. (gamma)).
    """
    C4 = voigt_stiffness_to_tensor(C0_voigt)
    k = np.asarray(k, dtype=np.float64)
    flat = k.reshape(-1, 3)
    out = np.zeros((flat.shape[0], 6, 6))
    nz = np.any(flat != 0, axis=1)
    kk = flat[nz]
    if len(kk):
        N = np.linalg.inv(acoustic_tensor(C4, kk))
        for J in range(6):
            e = np.zeros(6)
            e[J] = 1.0
            tau = mandel_to_tensor(e)
            tk = np.einsum("ab,nb->na", tau, kk)          # tau k
            w = np.einsum("nab,nb->na", N, tk)             # K^{-1} tau k
            res = 0.5 * (kk[:, :, None] * w[:, None, :] + w[:, :, None] * kk[:, None, :])
            out[nz, :, J] = tensor_to_mandel(res)
    return out.reshape(k.shape[:-1] + (6, 6))


def gamma0_isotropic(lam, mu, k):
    """Closed form of Gamma0_k for an isotropic C0 (Lame lam, mu).

    Gamma0_k tau = (1/mu) sym(n (x) tau n) - (lam+mu)/(mu(lam+2mu)) (n.tau n) n (x) n,
    n = k/|k|: the Sherman-Morrison inverse of K = mu|k|^2 I + (lam+mu) k k^T
    inserted into eq. (gamma).
    """
    k = np.asarray(k, dtype=np.float64)
    flat = k.reshape(-1, 3)
    out = np.zeros((flat.shape[0], 6, 6))
    nz = np.any(flat != 0, axis=1)
    n = flat[nz] / np.linalg.norm(flat[nz], axis=1, keepdims=True)
    c = (lam + mu) / (mu * (lam + 2 * mu))
    for J in range(6):
        e = np.zeros(6)
        e[J] = 1.0
        tau = mandel_to_tensor(e)
        tn = np.einsum("ab,nb->na", tau, n)
        ntn = np.einsum("na,na->n", n, tn)
        res = (0.5 / mu) * (n[:, :, None] * tn[:, None, :] + tn[:, :, None] * n[:, None, :]) \
            - c * ntn[:, None, None] * n[:, :, None] * n[:, None, :]
        out[nz, :, J] = tensor_to_mandel(res)
    return out.reshape(k.shape[:-1] + (6, 6))


# ---------------------------------------------------------------------------
# Generating functions (Sec. 2.2) as weights g(x), x = M^{-T} k
# ---------------------------------------------------------------------------
DIRICHLET = "dirichlet"
DIRICHLET_MODIFIED = "dirichlet_modified"
DLVP = "dlvp"
BOX = "box"


def g_dirichlet(x):
    """Dirichlet kernel D_M: g = indicator of the half-open cube [-1/2, 1/2)^d."""
    x = np.asarray(x)
    return np.all((x >= -0.5) & (x < 0.5), axis=-1).astype(np.float64)


def _trapezoid(t, a):
    """One axis of g_alpha = B_Xi, Xi = (diag(alpha), I): the centred box of
    width a convolved with the unit box; flat 1 for |t| <= (1-a)/2, linear to
    0 at (1+a)/2.  a = 0 is the limit: 1 inside, 1/2 on |t| = 1/2."""
    t = np.abs(np.asarray(t, dtype=np.float64))
    if a == 0.0:
        return np.where(t < 0.5, 1.0, np.where(t == 0.5, 0.5, 0.0))
    return np.clip(((1.0 + a) / 2.0 - t) / a, 0.0, 1.0)


def g_dlvp(x, alpha):
    """Admissible g_alpha of Sec. 2.2 (tensor trapezoid), alpha in [0,1]^d as in
    the definition; alpha = 0 gives the modified Dirichlet kernel f_{M,0}."""
    x = np.asarray(x, dtype=np.float64)
    out = np.ones(x.shape[:-1])
    for i, a in enumerate(alpha):
        out = out * _trapezoid(x[..., i], float(a))
    return out


def g_box(x, Xi):
    """Pattern Box spline weights: prod over the columns xi of sinc(pi xi^T x),
    sinc(t) = sin t / t (Sec. 2.2, c_k(B_Xi) with k -> M^{-T} k)."""
    x = np.asarray(x, dtype=np.float64)
    Xi = np.asarray(Xi, dtype=np.float64)
    out = np.ones(x.shape[:-1])
    for s in range(Xi.shape[1]):
        out = out * np.sinc(x @ Xi[:, s])  # numpy sinc(u) = sin(pi u)/(pi u)
    return out


def weight_fn(kind, params):
    if kind == DIRICHLET:
        return g_dirichlet
    if kind == DIRICHLET_MODIFIED:
        return lambda x: g_dlvp(x, [0.0] * x.shape[-1])
    if kind == DLVP:
        return lambda x: g_dlvp(x, params["alpha"])
    if kind == BOX:
        return lambda x: g_box(x, params["Xi"])
    raise ValueError(f"unknown kernel {kind}")


def alias_offsets(kind, params, d=3):
    """The finite set of z over which the bracket sum is taken.

    Dirichlet: z = 0 (x already in the cube).  Modified Dirichlet and dlVP
    (alpha <= 1): support |x_i + z_i| < 1, so z in {-1,0,1}^d (Sec. 3.2: the
    sum is finite and evaluated exactly).  Box: the truncation box
    [-R, R]^d (Sec. 4.2 precomputes 33^2 terms in 2-D, i.e. R = 16).
    """
    if kind == DIRICHLET:
        return np.zeros((1, d), dtype=np.int64)
    if kind in (DIRICHLET_MODIFIED, DLVP):
        return np.array(list(itertools.product((-1, 0, 1), repeat=d)), dtype=np.int64)
    if kind == BOX:
        R = int(params.get("R", 16))
        return np.array(list(itertools.product(range(-R, R + 1), repeat=d)), dtype=np.int64)
    raise ValueError(kind)


def gamma_periodised(P: Pattern, C0_voigt, kind, params=None, b=None, chunk=4096):
    """Gamma^p_h for the frequencies h(b), b in storage order (default: all).

    Def. (gamma_tilde_fourier) with orthonormalised translates:
    sum_z w(x+z) Gamma0_{h+M^T z} / sum_z w(x+z), w = g^2, x = M^{-T} h.
    Also returns the bracket sum of the weights (Lemma (FI:Props) b: it must be
    positive for linearly independent translates).
    """
    H, _ = P.frequencies(b)
    return gamma_at_frequencies(P, C0_voigt, kind, params, H, chunk)


def gamma_at_frequencies(P: Pattern, C0_voigt, kind, params, H, chunk=4096):
    """Gamma^p at integer frequencies H (n, d); each h is first reduced into G(M^T)."""
    params = params or {}
    H, Xn = P.reduce_frequencies(H)
    X = Xn.astype(np.float64) / P.m
    Z = alias_offsets(kind, params, P.d)
    MT = np.array(P.MT, dtype=np.int64)
    g = weight_fn(kind, params)
    n = len(H)
    out = np.zeros((n, 6, 6))
    den_all = np.zeros(n)
    for s in range(0, n, chunk):
        h = H[s:s + chunk]
        x = X[s:s + chunk]
        num = np.zeros((len(h), 6, 6))
        den = np.zeros(len(h))
        for z in Z:
            w = g(x + z) ** 2
            sel = w > 0
            if not np.any(sel):
                continue
            k = h[sel] + (MT @ z)[None, :]
            num[sel] += w[sel, None, None] * gamma0(C0_voigt, k)
            den[sel] += w[sel]
        if kind == BOX and params.get("tail"):
            tn, td = box_tail(P, C0_voigt, params, h, x)
            num += tn
            den += td
        ok = den > 0
        out[s:s + chunk][ok] = num[ok] / den[ok, None, None]
        den_all[s:s + chunk] = den
    # h = 0: zero-mean compatible fields (Gamma0_0 = 0); its aliases carry no
    # weight for the kernels above, set it exactly.
    zero = np.all(H == 0, axis=1)
    out[zero] = 0.0
    return out, den_all


def box_slow_axes(Xi):
    """Axes i of the alias lattice along which the Box weight decays only like
    1/t^2: exactly one column xi has xi_i != 0, and |xi_i| = 1.  Returns
    [(i, s)] with s the index of that column."""
    Xi = np.asarray(Xi, dtype=np.float64)
    out = []
    for i in range(Xi.shape[0]):
        nz = [s for s in range(Xi.shape[1]) if Xi[i, s] != 0.0]
        if len(nz) == 1 and abs(Xi[i, nz[0]]) == 1.0:
            out.append((i, nz[0]))
    return out


def box_tail(P: Pattern, C0_voigt, params, H, X, gamma_fn=None):
    """Leading term of the Box alias sum beyond the truncation box [-R, R]^d.

    For integer directions xi the factor sin^2(pi xi^T (x+z)) of each weight
    does not depend on z, so a weight is a rational function of z.  Along a
    slow axis i (box_slow_axes) only the column xi* involves z_i: the line of
    aliases z_perp + z_i e_i carries the weight w_perp(z_perp) sinc^2(pi (c + z_i))
    with c = xi*^T (x + z_perp) (xi*_i = +-1), and the part beyond |z_i| > R is
    exactly w_perp (1 - sum_{|n| <= R} sinc^2(pi (c + n))) by the identity
    sum_n sinc^2(pi (c + n)) = 1.  On those aliases k = h + M^T z turns towards
    +-M^T e_i, so Gamma0_k tends to Gamma0_{M^T e_i} (even, degree 0); the term
    odd in 1/z_i cancels between the two half-lines.  The neglected parts
    (the next order along the line, aliases beyond R on the fast axes) are
    O(R^-3) against O(R^-1) for plain truncation.
    gamma_fn(C0_voigt, k) gives the Green operator (default: gamma0 of this
    module, d = 3).  Returns (num (n, q, q), den (n,)) to add to the truncated
    sums."""
    gamma_fn = gamma_fn or gamma0
    Xi = np.asarray(params["Xi"], dtype=np.float64)
    R = int(params.get("R", 16))
    d = P.d
    MT = np.array(P.MT, dtype=np.float64)
    n = len(H)
    q = 6 if d == 3 else 3
    num = np.zeros((n, q, q))
    den = np.zeros(n)
    rng = np.arange(-R, R + 1)
    for i, s in box_slow_axes(Xi):
        G_inf = gamma_fn(C0_voigt, (MT @ np.eye(d)[i])[None])[0]
        others = [j for j in range(d) if j != i]
        for zp in itertools.product(rng, repeat=d - 1):
            z = np.zeros(d)
            z[others] = zp
            y = X + z[None, :]                      # z_i = 0: xi*_i (x_i + 0) enters c
            w_perp = np.ones(n)
            for t in range(Xi.shape[1]):
                if t != s:
                    w_perp *= np.sinc(y @ Xi[:, t]) ** 2
            c = y @ Xi[:, s]
            line = np.zeros(n)
            for m_ in rng:
                line += np.sinc(c + m_) ** 2
            add = w_perp * (1.0 - line)
            num += add[:, None, None] * G_inf[None]
            den += add
    return num, den


def gamma_symmetrised_at(P: Pattern, C0_voigt, kind, params, H):
    """(Gamma^p_h + Gamma^p_{-h}) / 2 at integer frequencies H (see gamma_symmetrised)."""
    Gp, d1 = gamma_at_frequencies(P, C0_voigt, kind, params, H)
    Gm, d2 = gamma_at_frequencies(P, C0_voigt, kind, params, -np.asarray(H))
    return 0.5 * (Gp + Gm), np.minimum(d1, d2)


def gamma_symmetrised(P: Pattern, C0_voigt, kind, params=None):
    """(Gamma^p_b + Gamma^p_{-b}) / 2 over the full spectrum (storage order).

    Real strain fields stay real only under a multiplier with
    Gamma_{-h} = Gamma_h.  The literal Dirichlet table breaks this on the -1/2
    faces of the cube; taking the real part of the inverse transform (what
    ``scheme.basic_scheme`` does) is the same as using this average.
    """
    G, den = gamma_periodised(P, C0_voigt, kind, params)
    e = P.e
    idx = P.grid_indices()
    neg = (-idx) % np.array(e)
    flat = np.ravel_multi_index(tuple(neg.T), tuple(e))
    return 0.5 * (G + G[flat]), den
