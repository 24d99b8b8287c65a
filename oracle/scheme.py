"""The Basic Scheme for the discretised Lippmann-Schwinger equation.

Test infrastructure (oracle); see the package docstring.

Thm. (pde_discretization), eq. (pde_coefficients): the sample values E_y of the
strain fluctuation satisfy
    E_y + Gamma^p_y (C(y) - C0) : (E_y + eps0) = 0,   y in P(M),
where Gamma^p acts as a Fourier multiplier on the pattern (the proof shows the
condition is an inverse pattern DFT of Gamma^p_h B_hat_h, B_y the polarisation).
Sec. 4 solves it by the fixed-point iteration of Moulinec and Suquet on E_y,
stopped by a relative Cauchy criterion.  Readings used here:

* polarisation form  E^{k+1} = -Re F^{-1}[ Gamma^p_h F[(C - C0):(E^k + eps0)]_h ],
  E^0 = 0 (or a given start with its mean removed);
* Cauchy residual  r_{k+1} = ||E^{k+1} - E^k|| / ||E^{k+1} + eps0||, Frobenius
  norms summed over all points (the paper names neither norm nor denominator);
* effective stress  sigma_bar = (1/m) sum_y C(y):(E_y + eps0), the pattern mean
  of the definition of C^eff (Sec. 3.1) at the samples;
* the real part: strain fields are real (Sym_d(R)); for every kernel except the
  literal Dirichlet one Gamma^p is even in h and the real part changes nothing.
"""
from __future__ import annotations

import numpy as np

from . import dft
from . import green
from .lattice import Pattern


def stiffness_field(C_phases_voigt, phase):
    """Per-point Mandel stiffness (m, 6, 6) from per-phase Voigt matrices."""
    Cm = green.voigt_stiffness_to_mandel(np.asarray(C_phases_voigt, dtype=np.float64))
    return Cm[np.asarray(phase, dtype=np.int64)]


def basic_scheme(P: Pattern, Gamma, C_phases_voigt, C0_voigt, phase, eps0_voigt,
                 tol=1e-10, max_iter=1000, E_init=None, n_iter=None):
    """Run the fixed point of eq. (pde_coefficients).

    Parameters
    ----------
    Gamma : (m, 6, 6) Gamma^p_h in frequency storage order (``green.gamma_periodised``).
    eps0_voigt : macroscopic strain, Voigt with engineering shear.
    E_init : optional start (m, 6) Mandel; its mean is removed.
    n_iter : if given, run exactly this many iterations (no stopping test).

    Returns dict(E (m,6) Mandel, sigma_voigt (6,), iterations, history).
    """
    m = P.m
    C = stiffness_field(C_phases_voigt, phase)
    C0 = green.voigt_stiffness_to_mandel(C0_voigt)
    Delta = C - C0[None]
    eps0 = green.voigt_strain_to_mandel(eps0_voigt)
    if E_init is None:
        E = np.zeros((m, 6))
    else:
        E = np.array(E_init, dtype=np.float64).reshape(m, 6)
        E = E - E.mean(axis=0, keepdims=True)
    history = []
    it = 0
    limit = n_iter if n_iter is not None else max_iter
    while it < limit:
        tau = np.einsum("yij,yj->yi", Delta, E + eps0)          # (C - C0):(E + eps0)
        tau_hat = dft.pattern_dft(P, tau)                          # F(M), unnormalised
        E_hat = -np.einsum("bij,bj->bi", Gamma, tau_hat)           # -Gamma^p_h tau_hat_h
        E_new = dft.pattern_idft(P, E_hat).real                    # inverse pattern DFT
        num = np.sqrt(np.sum((E_new - E) ** 2))
        den = np.sqrt(np.sum((E_new + eps0) ** 2))
        r = num / den
        E = E_new
        it += 1
        history.append(r)
        if n_iter is None and r <= tol:
            break
    sigma = np.einsum("yij,yj->i", C, E + eps0) / m
    return dict(E=E, sigma_voigt=green.mandel_stress_to_voigt(sigma), iterations=it,
                history=np.array(history))


def effective_stiffness(P: Pattern, Gamma, C_phases_voigt, C0_voigt, phase, tol=1e-10,
                        max_iter=1000, n_iter=None):
    """C^eff in Voigt form: column j is sigma_bar for the unit Voigt load e_j (Sec. 3.1)."""
    Ceff = np.zeros((6, 6))
    its = []
    for j in range(6):
        e = np.zeros(6)
        e[j] = 1.0
        res = basic_scheme(P, Gamma, C_phases_voigt, C0_voigt, phase, e, tol=tol,
                           max_iter=max_iter, n_iter=n_iter)
        Ceff[:, j] = res["sigma_voigt"]
        its.append(res["iterations"])
    return Ceff, its


def _dense_pieces(M, C0_voigt, kind, params, C_phases_voigt, phase_by_point):
    """Fourier matrix of eq. (Fouriermatrix) over brute-force enumerations of P(M)
    and G(M^T), Gamma^p at those h (alias sum written out), and the per-point
    Mandel stiffness.  Returns (F, Y, G (m,6,6), Cm_points (m,6,6), C0 Mandel)."""
    F, H, Y = dft.fourier_matrix(M)
    from .lattice import brute_force_points
    Yf = brute_force_points(M)
    m = len(Yf)
    P = Pattern(M)
    C0 = green.voigt_stiffness_to_mandel(C0_voigt)
    Cm = green.voigt_stiffness_to_mandel(np.asarray(C_phases_voigt, dtype=np.float64))
    ph = np.array([phase_by_point[y] for y in Yf], dtype=np.int64)
    MT = np.array(P.MT, dtype=np.int64)
    Minv_T = np.linalg.inv(np.array(P.M, dtype=np.float64)).T
    g = green.weight_fn(kind, params)
    Z = green.alias_offsets(kind, params, P.d)
    G = np.zeros((m, 6, 6))
    for r, h in enumerate(H):
        if not np.any(h):
            continue
        x = Minv_T @ h
        num = np.zeros((6, 6))
        den = 0.0
        for z in Z:
            w = g((x + z)[None])[0] ** 2
            if w > 0:
                num += w * green.gamma0(C0_voigt, (h + MT @ z)[None])[0]
                den += w
        G[r] = num / den
    return F, Y, G, Cm[ph], C0


def _dense_operator(F, G, D):
    """Matrix of E (m*6) -> Re F^H Gamma F (D E) for per-point 6x6 blocks D."""
    m = F.shape[0]
    Fh = F.conj().T
    A = np.zeros((m * 6, m * 6))
    for p in range(m):
        for j in range(6):
            v = np.zeros((m, 6))
            v[p] = D[p][:, j]                # column j of D at point p
            vh = F @ v                       # (m, 6) spectrum
            A[:, p * 6 + j] = (Fh @ np.einsum("hij,hj->hi", G, vh)).real.reshape(-1)
    return A


def dense_fixed_point(M, C0_voigt, kind, params, C_phases_voigt, phase_by_point, eps0_voigt):
    """Solve eq. (pde_coefficients) directly as a dense linear system (tiny m).

    Independent of the SNF path: the pattern DFT is the matrix of
    eq. (Fouriermatrix) over brute-force enumerations of P(M) and G(M^T), and
    Gamma^p_h is evaluated at those h.  Unknowns are E_y (6 per point):
        (I + R) E = -R eps0,   R = Re F^H diag(Gamma_h) F (C - C0).
    ``phase_by_point`` maps each brute-force point (tuple of Fractions) to its
    phase.  Returns (Y, E) with Y the points and E (m, 6) Mandel.
    """
    F, Y, G, Cp, C0 = _dense_pieces(M, C0_voigt, kind, params, C_phases_voigt, phase_by_point)
    m = len(Y)
    A = -_dense_operator(F, G, Cp - C0[None])
    eps0 = green.voigt_strain_to_mandel(eps0_voigt)
    rhs = (A @ np.tile(eps0, m))
    # E = A (E + eps0)  ->  (I - A) E = A eps0
    E = np.linalg.solve(np.eye(m * 6) - A, rhs).reshape(m, 6)
    return Y, E


def dense_variational_point(M, C0_voigt, kind, params, C_phases_voigt, phase_by_point, eps0_voigt):
    """Solve eq. (pde_coefficients_variational) directly (tiny m): with
    R = Re F^H diag(Gamma_h) F (symmetric), find E in range(R) with
    R C (E + eps0) = 0.  E = Q c over an orthonormal basis Q of range(R):
        (Q^T R C Q) c = -Q^T R C eps0.
    Returns (Y, E) as dense_fixed_point."""
    F, Y, G, Cp, C0 = _dense_pieces(M, C0_voigt, kind, params, C_phases_voigt, phase_by_point)
    m = len(Y)
    R = _dense_operator(F, G, np.broadcast_to(np.eye(6), (m, 6, 6)))
    R = 0.5 * (R + R.T)
    w, V = np.linalg.eigh(R)
    Q = V[:, np.abs(w) > 1e-10 * np.abs(w).max()]
    Cb = np.zeros((m * 6, m * 6))
    for p in range(m):
        Cb[6 * p:6 * p + 6, 6 * p:6 * p + 6] = Cp[p]
    eps0 = np.tile(green.voigt_strain_to_mandel(eps0_voigt), m)
    K = Q.T @ R @ Cb
    c = np.linalg.solve(K @ Q, -K @ eps0)
    return Y, (Q @ c).reshape(m, 6)


def variational_scheme(P: Pattern, Gamma, C_phases_voigt, C0_voigt, phase, eps0_voigt,
                       tol=1e-10, max_iter=1000, E_init=None, n_iter=None):
    """Fixed point for the variational discretisation, eq. (pde_coefficients_variational).

    Thm. (ls_discretization): the sample values E_y satisfy
        F^{-1}[ Gamma^p_h F[C:(E + eps0)]_h ] = 0      (C0 in front is invertible).
    Iterated in the strain-update form
        E^{k+1} = E^k - Re F^{-1}[ Gamma^p_h F[C:(E^k + eps0)]_h ],
    whose fixed points are exactly the solutions in the range of Gamma^p.  For the
    Dirichlet kernel Gamma^p C0 is a projection that fixes the iterates, and the
    iterates coincide with the polarisation form (Remark (constants)); for the
    other kernels they do not.  Residual, output and arguments as basic_scheme.
    """
    m = P.m
    C = stiffness_field(C_phases_voigt, phase)
    eps0 = green.voigt_strain_to_mandel(eps0_voigt)
    if E_init is None:
        E = np.zeros((m, 6))
    else:
        E = np.array(E_init, dtype=np.float64).reshape(m, 6)
        E = E - E.mean(axis=0, keepdims=True)
    history = []
    it = 0
    limit = n_iter if n_iter is not None else max_iter
    while it < limit:
        s = np.einsum("yij,yj->yi", C, E + eps0)                    # C:(E + eps0)
        s_hat = dft.pattern_dft(P, s)
        corr = dft.pattern_idft(P, np.einsum("bij,bj->bi", Gamma, s_hat)).real
        E_new = E - corr
        num = np.sqrt(np.sum((E_new - E) ** 2))
        den = np.sqrt(np.sum((E_new + eps0) ** 2))
        r = num / den
        E = E_new
        it += 1
        history.append(r)
        if n_iter is None and r <= tol:
            break
    sigma = np.einsum("yij,yj->i", C, E + eps0) / m
    return dict(E=E, sigma_voigt=green.mandel_stress_to_voigt(sigma), iterations=it,
                history=np.array(history))


def conjugate_gradient(P: Pattern, Gamma, C_phases_voigt, C0_voigt, phase, eps0_voigt,
                       tol=1e-10, max_iter=1000, E_init=None, n_iter=None, trace=False):
    """Conjugate gradients for the Dirichlet kernel's system (Sec. 1 names Krylov
    solvers as the alternative to the fixed-point iteration).

    For the Dirichlet kernel on a pattern without Nyquist faces (m odd: no bin
    with x_i = -1/2) the operator G: v -> Re F^{-1}[Gamma^p_h F[v]_h] satisfies
    G C0 G = G: G C0 projects onto the compatible fields (Def. (projection)),
    and eq. (pde_coefficients) is equivalent to its variational form
    (Remark (constants)): E compatible with G C (E + eps0) = 0.  On the
    compatible fields v -> G C v is symmetric positive definite in the C0
    inner product <a, C0 b>, so CG applies.  With the stress R = C(E + eps0)
    the residual is z = -G R (a compatible strain, the step one fixed-point
    iteration would take), and
        rho = <z, C0 z>,  alpha = rho / <p, C p>,  E += alpha p,  R += alpha C p,
        z = -G R,  beta = rho_new / rho,  p = z + beta p,
    starting from p = z.  rho is taken as <z, C0 z> (a sum of non-negative
    terms); the equal <R, G R> cancels: R is large and mostly in G's null space,
    and its rounding stalls the iteration near the square root of the unit
    roundoff.

    Stopping rule: r_k = ||z_k|| / ||E_k + z_k + eps0|| <= tol, the Basic
    Scheme's Cauchy residual one fixed-point step from E_k would show.
    history[k] = r_k; `iterations` counts applications of G (the start's one
    included), the unit of the fixed-point schemes.  n_iter runs exactly that
    many.  trace=True also returns the directions p_k, stresses R_k and
    residuals z_k (for the conjugacy pins).
    """
    m = P.m
    C = stiffness_field(C_phases_voigt, phase)
    C0 = green.voigt_stiffness_to_mandel(C0_voigt)
    eps0 = green.voigt_strain_to_mandel(eps0_voigt)

    def apply_G(v):
        return -dft.pattern_idft(P, np.einsum("bij,bj->bi", Gamma, dft.pattern_dft(P, v))).real

    def c0_norm2(v):
        return float(np.sum(v * (v @ C0)))

    if E_init is None:
        E = np.zeros((m, 6))
    else:
        E = np.array(E_init, dtype=np.float64).reshape(m, 6)
        E = E - E.mean(axis=0, keepdims=True)
    R = np.einsum("yij,yj->yi", C, E + eps0)
    z = apply_G(R)
    rho = c0_norm2(z)
    p = z.copy()
    history = []
    tr = {"p": [], "R": [], "z": []}
    limit = n_iter if n_iter is not None else max_iter
    it = 0
    while it < limit:
        r = np.sqrt(np.sum(z ** 2)) / np.sqrt(np.sum((E + z + eps0) ** 2))
        history.append(r)
        it += 1
        if n_iter is None and r <= tol:
            break
        if it == limit:
            break
        q = np.einsum("yij,yj->yi", C, p)
        pq = np.sum(p * q)
        alpha = rho / pq if pq > 0 else 0.0
        if trace:
            tr["p"].append(p.copy())
            tr["R"].append(R.copy())
            tr["z"].append(z.copy())
        E = E + alpha * p
        R = R + alpha * q
        z = apply_G(R)
        rho_new = c0_norm2(z)
        beta = rho_new / rho if rho > 0 else 0.0
        rho = rho_new
        p = z + beta * p
    sigma = np.einsum("yij,yj->i", C, E + eps0) / m
    out = dict(E=E, sigma_voigt=green.mandel_stress_to_voigt(sigma), iterations=it, history=np.array(history))
    if trace:
        out["trace"] = tr
    return out
