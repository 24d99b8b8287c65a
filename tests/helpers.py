"""Shared helpers for the parity tests: build a problem once, run the oracle and
the HIP library on the same seeded inputs, and map between their orderings."""
from __future__ import annotations

import numpy as np

import lsh_inputs as li
from oracle import green, scheme
from oracle.lattice import Pattern as OPattern

BOX_CFG3 = {"Xi": np.array([[1, 0, 0, 1], [0, 1, 0, 1], [0, 0, 1, 0]], float), "R": 16}


def perm_to_oracle(gpu_pattern, opattern):
    """Index array q with gpu_point[q[i]] == oracle_point[i] (exact numerators)."""
    g = gpu_pattern.point_numerators()
    o = opattern.point_numerators()
    key = {tuple(r): i for i, r in enumerate(g.tolist())}
    return np.array([key[tuple(r)] for r in o.tolist()], dtype=np.int64)


def two_phase(E1=1.0, E2=10.0, nu=0.3):
    Cp = np.stack([li.isotropic_voigt(E1, nu), li.isotropic_voigt(E2, nu)])
    return Cp, li.mean_reference(Cp)


def oracle_kernel_params(kind, params):
    if kind == "box":
        return {"Xi": np.asarray(params["Xi"], float), "R": params.get("R", 16), "tail": bool(params.get("tail"))}
    if kind == "dlvp":
        return {"alpha": list(params["alpha"])}
    return {}


class Problem:
    """One pattern + kernel + two-phase material, on both sides."""

    def __init__(self, M, kind, params, phase_fn, Cp=None, C0=None):
        from paper_1701_04685_amd import lsh
        self.M = M
        self.kind = kind
        self.params = params or {}
        self.O = OPattern(M)
        self.G = lsh.Pattern(M)
        self.q = perm_to_oracle(self.G, self.O)
        Y = self.O.points()
        self.phase_o = phase_fn(Y).astype(np.uint8)
        self.phase_g = np.empty_like(self.phase_o)
        self.phase_g[self.q] = self.phase_o
        if Cp is None:
            Cp, C0 = two_phase()
        self.Cp, self.C0 = Cp, C0
        self.G.set_kernel(kind, self.params if self.params else None)
        self.G.set_stiffness(Cp, C0, self.phase_g)
        self._gamma = None

    def bind(self, prec):
        self.G.bind(prec)

    def gamma_oracle(self):
        if self._gamma is None:
            self._gamma, _ = green.gamma_periodised(self.O, self.C0, self.kind,
                                                    oracle_kernel_params(self.kind, self.params))
        return self._gamma

    def oracle_solve(self, eps0, tol=1e-10, max_iter=1000, n_iter=None):
        return scheme.basic_scheme(self.O, self.gamma_oracle(), self.Cp, self.C0, self.phase_o, eps0,
                                   tol=tol, max_iter=max_iter, n_iter=n_iter)

    def oracle_solve_ve(self, eps0, tol=1e-10, max_iter=1000, n_iter=None):
        return scheme.variational_scheme(self.O, self.gamma_oracle(), self.Cp, self.C0, self.phase_o, eps0,
                                         tol=tol, max_iter=max_iter, n_iter=n_iter)

    def gpu_E_to_oracle_mandel(self, E):
        """GPU field [6][m] (Voigt, engineering shear) -> oracle order (m, 6) Mandel."""
        E = np.asarray(E).reshape(6, -1)[:, self.q].T
        return green.voigt_strain_to_mandel(E)


BOX_PLANE8 = {"Xi": np.array([[1, 0, 1, 0, 1, 0, 1, 0], [0, 1, 0, 1, 0, 1, 0, 1]], float), "R": 16}


class PlaneProblem:
    """A two-dimensional pattern + kernel + plane-strain phases, on both sides
    (oracle/plane.py and the library's d = 2 path)."""

    def __init__(self, M, kind, params, phase_fn, E=(1.0, 10.0), nu=0.3):
        from paper_1701_04685_amd import lsh
        from oracle import plane
        self.plane = plane
        self.kind = kind
        self.params = params or {}
        self.O = OPattern(M)
        self.G = lsh.Pattern(M)
        self.q = perm_to_oracle(self.G, self.O)
        self.phase_o = phase_fn(self.O.points()).astype(np.uint8)
        self.phase_g = np.empty_like(self.phase_o)
        self.phase_g[self.q] = self.phase_o
        self.Cp = np.stack([li.isotropic_voigt_plane(e, nu) for e in E])
        self.C0 = li.mean_reference(self.Cp)
        self.G.set_kernel(kind, self.params if self.params else None)
        self.G.set_stiffness(self.Cp, self.C0, self.phase_g)
        self._gamma = None

    def gamma_oracle(self):
        if self._gamma is None:
            self._gamma, _ = self.plane.gamma_periodised(self.O, self.C0, self.kind,
                                                         oracle_kernel_params(self.kind, self.params))
        return self._gamma

    def oracle_solve(self, eps0, tol=1e-10, max_iter=1000, n_iter=None):
        return self.plane.basic_scheme(self.O, self.gamma_oracle(), self.Cp, self.C0, self.phase_o, eps0,
                                       tol=tol, max_iter=max_iter, n_iter=n_iter)

    def gpu_E_to_oracle_mandel(self, E):
        """GPU field [3][m] (Voigt, engineering shear) -> oracle order (m, 3) Mandel."""
        E = np.asarray(E).reshape(3, -1)[:, self.q].T
        return self.plane.voigt_strain_to_mandel(E)
