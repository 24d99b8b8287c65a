"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle.

Tolerances: FP64 path 1e-10 relative on sigma_bar / C^eff and on E (the
target for the double path); FP32 mixed path 1e-5 relative on sigma_bar and
E (single-precision FFT and Green multiply, double residuals and averages).
Lock-step runs fix the iteration count on both sides (tol < 0 on the GPU,
n_iter in the oracle) so that the comparison is not blurred by the stopping
iteration.
"""
import numpy as np
import pytest

import lsh_inputs as li
from helpers import BOX_CFG3, Problem, two_phase

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-5


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def random_phase(seed, frac=0.4):
    rng = np.random.default_rng(seed)
    return lambda Y: (rng.random(len(Y)) < frac).astype(np.uint8)


def spheres(seed, frac=0.3):
    def f(Y):
        m = len(Y)
        c, r = li.rsa_spheres(seed, li.lattice_unit(m), frac, rmin=1.5, rmax=3.0)
        return li.spheres_phase(Y, c, r)
    return f


LAMINATE = lambda Y: li.laminate_phase(Y, 0)
KERNELS = [("dirichlet", {}), ("dirichlet_modified", {}), ("dlvp", {"alpha": [0.75] * 3}),
           ("box", {"Xi": BOX_CFG3["Xi"], "R": 3})]


# ------------------------------------------------------------- Gamma^p ---
@pytest.mark.parametrize("M", [np.diag([8, 8, 8]), [[4, 1, 0], [0, 4, 0], [0, 0, 2]], [[6, -3, 2], [1, 4, 0], [2, 0, 3]]])
@pytest.mark.parametrize("kind,params", KERNELS)
def test_gamma_probe_all_bins(M, kind, params):
    """Green operator at every half-spectrum bin == symmetrised oracle value at the
    same frequency h = V^T b (V: the library's own SNF factor)."""
    from oracle import green
    pr = Problem(M, kind, params, random_phase(1))
    pr.bind("fp64")
    e = pr.G.e
    bins = np.array([(a, b, c) for a in range(e[0] // 2 + 1) for b in range(e[1]) for c in range(e[2])])
    got = pr.G.gamma_probe(bins)
    _, V = pr.G.snf()
    ref, den = green.gamma_symmetrised_at(pr.O, pr.C0, kind, params, bins @ V)
    assert np.all(den > 0)
    iu = np.triu_indices(6)
    np.testing.assert_allclose(got, ref[:, iu[0], iu[1]], rtol=0, atol=1e-13)


def test_gamma_probe_sampled_cfg2_dlvp():
    """128^3 dlVP (alpha = 3/4): 300 random bins, on-the-fly alias sums vs oracle."""
    from oracle import green
    from paper_1701_04685_amd import lsh
    from oracle.lattice import Pattern as OP
    M = np.diag([128, 128, 128])
    P = lsh.Pattern(M)
    Cp, C0 = two_phase()
    P.set_kernel("dlvp", {"alpha": [0.75] * 3})
    P.set_stiffness(Cp, C0, np.zeros(P.m, np.uint8))
    P.bind("fp64")
    rng = np.random.default_rng(0)
    bins = np.stack([rng.integers(0, 65, 300), rng.integers(0, 128, 300), rng.integers(0, 128, 300)], 1)
    bins[0] = (64, 64, 64)  # a corner of the -1/2 faces
    got = P.gamma_probe(bins)
    _, V = P.snf()
    ref, _ = green.gamma_symmetrised_at(OP(M), C0, "dlvp", {"alpha": [0.75] * 3}, bins @ V)
    iu = np.triu_indices(6)
    np.testing.assert_allclose(got, ref[:, iu[0], iu[1]], rtol=0, atol=1e-13)


def test_gamma_table_sampled_cfg3_box():
    """M = [[128,32,0],[0,128,0],[0,0,64]], Box {e1,e2,e3,e1+e2}, R = 16: the
    GPU table (FP64 alias sums over 35,937 terms) at 40 random bins vs oracle."""
    from oracle import green
    from paper_1701_04685_amd import lsh
    from oracle.lattice import Pattern as OP
    M = [[128, 32, 0], [0, 128, 0], [0, 0, 64]]
    P = lsh.Pattern(M)
    Cp, C0 = two_phase(1.0, 100.0)
    P.set_kernel("box", BOX_CFG3)
    P.set_stiffness(Cp, C0, np.zeros(P.m, np.uint8))
    P.bind("fp64")
    rng = np.random.default_rng(1)
    e = P.e
    bins = np.stack([rng.integers(0, e[0] // 2 + 1, 40), rng.integers(0, e[1], 40), rng.integers(0, e[2], 40)], 1)
    got = P.gamma_probe(bins)
    _, V = P.snf()
    ref, _ = green.gamma_symmetrised_at(OP(M), C0, "box", BOX_CFG3, bins @ V)
    iu = np.triu_indices(6)
    np.testing.assert_allclose(got, ref[:, iu[0], iu[1]], rtol=0, atol=5e-12)


def _anisotropic_C0():
    """An elliptic, cubic-anisotropic reference stiffness (not isotropic)."""
    C = li.isotropic_voigt(4.0, 0.25)
    C[0, 1] = C[1, 0] = C[0, 1] + 0.3
    C[3, 3] += 0.4
    C[5, 5] -= 0.2
    return C


@pytest.mark.parametrize("kind,params", KERNELS)
def test_gamma_probe_anisotropic_C0(kind, params):
    """General (non-isotropic) C0: the on-the-fly general form (Dirichlet) and
    the tabled alias sums (dlVP, Box) against the oracle at every bin."""
    from oracle import green
    Cp, _ = two_phase()
    C0 = _anisotropic_C0()
    pr = Problem([[6, -3, 2], [1, 4, 0], [2, 0, 3]], kind, params, random_phase(2), Cp, C0)
    pr.bind("fp64")
    e = pr.G.e
    bins = np.array([(a, b, c) for a in range(e[0] // 2 + 1) for b in range(e[1]) for c in range(e[2])])
    got = pr.G.gamma_probe(bins)
    _, V = pr.G.snf()
    ref, _ = green.gamma_symmetrised_at(pr.O, C0, kind, params, bins @ V)
    iu = np.triu_indices(6)
    np.testing.assert_allclose(got, ref[:, iu[0], iu[1]], rtol=0, atol=1e-13)


@pytest.mark.parametrize("kind,params", [KERNELS[0], KERNELS[2]])
def test_lockstep_anisotropic_C0(kind, params):
    Cp, _ = two_phase()
    pr = Problem(np.diag([8, 12, 10]), kind, params, random_phase(9), Cp, _anisotropic_C0())
    _lockstep(pr, "fp64", np.array([0.3, -0.2, 0.1, 0.4, -0.1, 0.25]), 6, FP64_TOL)


# --------------------------------------------------------------- solver ---
def _lockstep(pr, prec, eps0, n_iter, tol_rel):
    pr.bind(prec)
    res = pr.G.solve(eps0[None], tol=-1.0, max_iter=n_iter, return_E=True, history=True)
    ref = pr.oracle_solve(eps0, n_iter=n_iter)
    assert res["iterations"][0] == n_iter
    # Cauchy residual history: same iterates, same norms (computed in another domain)
    np.testing.assert_allclose(res["history"][0], ref["history"], rtol=100 * tol_rel, atol=1e-14)
    Eg = pr.gpu_E_to_oracle_mandel(res["E"].cpu().numpy()[0])
    assert rel(res["sigma"][0], ref["sigma_voigt"]) < tol_rel
    assert rel(Eg, ref["E"]) < tol_rel
    return res, ref


@pytest.mark.parametrize("kind,params", KERNELS)
def test_laminate_closed_form_gpu(kind, params):
    """16^3 laminate: sigma_bar = (350/143, 150/143, 150/143, 0, 0, 0), stop at iteration 2."""
    pr = Problem(np.diag([16, 16, 16]), kind, params, LAMINATE)
    pr.bind("fp64")
    res = pr.G.solve(np.array([[1.0, 0, 0, 0, 0, 0]]), tol=1e-10, max_iter=100)
    assert res["iterations"][0] == 2
    np.testing.assert_allclose(res["sigma"][0], [350 / 143, 150 / 143, 150 / 143, 0, 0, 0], rtol=0, atol=1e-12)


def test_homogeneous_one_iteration_gpu():
    Cp = np.stack([li.isotropic_voigt(3.0, 0.2)])
    C0 = li.isotropic_voigt(1.0, 0.3)
    pr = Problem([[4, 1, 0], [0, 4, 0], [0, 0, 2]], "dlvp", {"alpha": [0.5] * 3}, lambda Y: np.zeros(len(Y)), Cp, C0)
    pr.bind("fp64")
    eps0 = np.array([0.3, -0.1, 0.2, 0.05, -0.4, 0.1])
    res = pr.G.solve(eps0[None], tol=1e-12, max_iter=10, return_E=True)
    assert res["iterations"][0] == 1
    assert float(res["E"].abs().max()) < 1e-15
    np.testing.assert_allclose(res["sigma"][0], Cp[0] @ eps0, rtol=1e-14)


CASES = [
    (np.diag([8, 8, 8]), random_phase(3)),
    ([[4, 1, 0], [0, 4, 0], [0, 0, 2]], random_phase(4)),          # SNF (1, 2, 16)
    ([[6, -3, 2], [1, 4, 0], [2, 0, 3]], random_phase(5)),         # non-diagonal, odd det
    (np.diag([5, 5, 7]), random_phase(6)),                          # SNF (1, 5, 35): radix 5 and 7
    (np.diag([6, 12, 12]), random_phase(7)),                        # radix 3, ragged tiles
    (np.diag([24, 20, 18]), spheres(8)),                            # several tiles + tails
]


@pytest.mark.parametrize("case", range(len(CASES)))
@pytest.mark.parametrize("kind,params", KERNELS)
def test_lockstep_fp64(case, kind, params):
    M, ph = CASES[case]
    pr = Problem(M, kind, params, ph)
    eps0 = np.array([0.3, -0.2, 0.1, 0.4, -0.1, 0.25])
    _lockstep(pr, "fp64", eps0, 7, FP64_TOL)


@pytest.mark.parametrize("case", [0, 3, 5])
@pytest.mark.parametrize("kind,params", [KERNELS[0], KERNELS[2], KERNELS[3]])
def test_lockstep_fp32(case, kind, params):
    M, ph = CASES[case]
    pr = Problem(M, kind, params, ph)
    eps0 = np.array([0.3, -0.2, 0.1, 0.4, -0.1, 0.25])
    _lockstep(pr, "fp32", eps0, 7, FP32_TOL)


def test_multi_load_effective_tensor_fp64():
    """Six unit loads side by side, converged: C^eff matches the oracle and is symmetric."""
    pr = Problem(np.diag([12, 12, 12]), "dlvp", {"alpha": [0.75] * 3}, spheres(11))
    pr.bind("fp64")
    res = pr.G.solve(np.eye(6), tol=1e-12, max_iter=2000)
    C = res["sigma"].T
    from oracle import scheme
    Cref, its = scheme.effective_stiffness(pr.O, pr.gamma_oracle(), pr.Cp, pr.C0, pr.phase_o, tol=1e-12, max_iter=2000)
    assert list(res["iterations"]) == list(its)
    assert rel(C, Cref) < 1e-10
    assert np.linalg.norm(C - C.T) / np.linalg.norm(C) < 1e-10


def test_warm_start_from_converged_field():
    """Starting from the oracle's converged field, the first Cauchy residual is tiny."""
    import torch
    pr = Problem(np.diag([8, 8, 8]), "dirichlet", {}, random_phase(12))
    pr.bind("fp64")
    eps0 = np.array([1.0, 0, 0, 0, 0, 0])
    ref = pr.oracle_solve(eps0, tol=1e-14, max_iter=3000)
    Ev = np.zeros((6, pr.O.m))
    from oracle import green
    Ev[:, pr.q] = green.mandel_strain_to_voigt(ref["E"]).T
    E0 = torch.tensor(Ev[None], dtype=torch.float64, device="cuda")
    res = pr.G.solve(eps0[None], tol=1e-10, max_iter=50, E_init=E0, history=True)
    assert res["iterations"][0] == 1
    assert res["history"][0, 0] < 1e-12
    assert rel(res["sigma"][0], ref["sigma_voigt"]) < 1e-12


@pytest.mark.parametrize("case", [0, 2, 5])
def test_lockstep_warm_start_random(case):
    """A random start field (mean removed on both sides): residual history and
    final field agree with the oracle started from the same field."""
    import torch
    from oracle import green, scheme
    M, ph = CASES[case]
    pr = Problem(M, "dlvp", {"alpha": [0.5] * 3}, ph)
    pr.bind("fp64")
    rng = np.random.default_rng(20 + case)
    Eo = rng.standard_normal((pr.O.m, 6)) * 0.1 + 0.05          # Mandel, oracle order, nonzero mean
    Ev = np.zeros((6, pr.O.m))
    Ev[:, pr.q] = green.mandel_strain_to_voigt(Eo).T
    eps0 = np.array([0.1, 0.2, -0.3, 0.05, 0.0, 0.15])
    res = pr.G.solve(eps0[None], tol=-1.0, max_iter=5, E_init=torch.tensor(Ev[None], device="cuda"),
                     return_E=True, history=True)
    ref = scheme.basic_scheme(pr.O, pr.gamma_oracle(), pr.Cp, pr.C0, pr.phase_o, eps0, n_iter=5, E_init=Eo)
    np.testing.assert_allclose(res["history"][0], ref["history"], rtol=1e-8)
    assert rel(pr.gpu_E_to_oracle_mandel(res["E"][0].cpu().numpy()), ref["E"]) < FP64_TOL
    assert rel(res["sigma"][0], ref["sigma_voigt"]) < FP64_TOL


def test_not_converged_status_and_outputs():
    pr = Problem(np.diag([8, 8, 8]), "dirichlet", {}, random_phase(13))
    pr.bind("fp64")
    res = pr.G.solve(np.eye(6)[:1], tol=1e-14, max_iter=3, allow_notconverged=True, history=True)
    assert res["status"] == -5
    assert res["iterations"][0] == 3 and np.all(np.isfinite(res["history"][0, :3]))
    ref = pr.oracle_solve(np.eye(6)[0], n_iter=3)
    assert rel(res["sigma"][0], ref["sigma_voigt"]) < 1e-10


def test_workspace_too_small_rejected():
    from paper_1701_04685_amd import lsh
    import torch
    pr = Problem(np.diag([8, 8, 8]), "dirichlet", {}, random_phase(14))
    pr.bind("fp64")
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(lsh.LshError) as e:
        lsh._check(lsh._lib.lsh_solve(pr.G._h, 1, lsh._dptr(np.eye(6)[0].copy()), 1e-6, 10, 0,
                                      lsh.ctypes.c_void_p(small.data_ptr()), 16, lsh._stream(), None, None,
                                      lsh._dptr(np.zeros(6)), None, None))
    assert e.value.status == -8


def test_profile_select_times_only_chosen_passes():
    """lsh_profile_select limits the event timing to the chosen slots;
    lsh_profile_enable times every slot again."""
    from paper_1701_04685_amd import lsh
    pr = Problem(np.diag([8, 8, 8]), "dirichlet", {}, random_phase(15))
    pr.bind("fp64")
    lsh.profile_enable(True)
    try:
        lsh.profile_select([2])
        pr.G.solve(np.eye(6)[:1], tol=-1.0, max_iter=5)
        ms, cnt = lsh.profile_read()
        assert cnt[2] == 5 and ms[2] > 0
        assert all(cnt[i] == 0 for i in range(8) if i != 2), cnt
        lsh.profile_enable(True)
        pr.G.solve(np.eye(6)[:1], tol=-1.0, max_iter=2)
        ms, cnt = lsh.profile_read()
        assert list(cnt[:6]) == [2, 2, 2, 2, 2, 1], cnt
    finally:
        lsh.profile_enable(False)


# ------------------------------------------------------ full-size configs ---
def test_cfg2_fullsize_lockstep_3_iterations():
    """128^3, dlVP alpha = 3/4, centred sphere f = 0.2, contrast 10, six loads in
    the launch configuration the benchmark uses: 3 lock-step iterations against
    the oracle on two of the loads (the oracle at this size costs seconds per
    iteration)."""
    r = li.centred_sphere_radius(0.2)
    pr = Problem(np.diag([128, 128, 128]), "dlvp", {"alpha": [0.75] * 3},
                 lambda Y: li.sphere_phase(Y, np.zeros(3), r))
    pr.bind("fp64")
    loads = np.eye(6)
    import torch
    ws = torch.empty(pr.G.workspace_bytes(6), dtype=torch.uint8, device="cuda")
    pr.G.autotune(nload=6, workspace=ws)  # the variants the benchmark runs: the autotuner's choice
    res = pr.G.solve(loads, tol=-1.0, max_iter=3, return_E=True, workspace=ws)
    for j in (0, 4):
        ref = pr.oracle_solve(loads[j], n_iter=3)
        assert rel(res["sigma"][j], ref["sigma_voigt"]) < FP64_TOL
        Eg = pr.gpu_E_to_oracle_mandel(res["E"][j].cpu().numpy())
        assert rel(Eg, ref["E"]) < FP64_TOL


# ---------------------------------------------------------------- batches ---
def test_batch_matches_single_solves():
    """Uneven pattern sizes and materials in one batched call: every task's
    sigma_bar and iteration count equal a single solve of the same task, and
    the oracle in lock-step for one of them."""
    from paper_1701_04685_amd import lsh
    rng = np.random.default_rng(30)
    specs = [(np.diag([8, 8, 8]), 3.0, 0.3), (np.diag([12, 12, 12]), 20.0, 0.25), (np.diag([8, 8, 8]), 10.0, 0.4),
             (np.diag([6, 10, 12]), 5.0, 0.2)]
    pats, loads, singles = [], [], []
    for i, (M, contrast, frac) in enumerate(specs):
        Cp = np.stack([li.isotropic_voigt(1.0, 0.3), li.isotropic_voigt(contrast, 0.3)])
        C0 = li.mean_reference(Cp)
        P = lsh.Pattern(M)
        ph = (rng.random(P.m) < frac).astype(np.uint8)
        P.set_kernel("dirichlet")
        P.set_stiffness(Cp, C0, ph)
        P.bind("fp32")
        pats.append(P)
        loads.append(np.eye(6)[: 2 + i])
    out = lsh.solve_batch(pats, loads, tol=1e-5, max_iter=500, precision="fp32")
    for P, e, o in zip(pats, loads, out):
        ref = P.solve(e, tol=1e-5, max_iter=500)
        assert list(o["iterations"]) == list(ref["iterations"])
        np.testing.assert_allclose(o["sigma"], ref["sigma"], rtol=1e-6, atol=1e-7)
        assert np.all(o["converged"])


def test_batch_lockstep_against_oracle():
    from paper_1701_04685_amd import lsh
    prs = [Problem(np.diag([8, 8, 8]), "dlvp", {"alpha": [0.5] * 3}, random_phase(31)),
           Problem(np.diag([6, 6, 10]), "dlvp", {"alpha": [0.5] * 3}, random_phase(32))]
    for pr in prs:
        pr.bind("fp64")
    eps = [np.array([[0.1, 0.2, -0.3, 0.05, 0.0, 0.15]]), np.eye(6)[[0, 3]]]
    out = lsh.solve_batch([pr.G for pr in prs], eps, tol=-1.0, max_iter=6, precision="fp64")
    for pr, e, o in zip(prs, eps, out):
        for j in range(len(e)):
            ref = pr.oracle_solve(e[j], n_iter=6)
            assert rel(o["sigma"][j], ref["sigma_voigt"]) < FP64_TOL
