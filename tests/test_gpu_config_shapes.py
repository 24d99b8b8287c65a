"""GPU parity at the benchmark workloads' own shapes, in the launch
configurations the benchmark runs (autotuned variants, six loads per call).

The compile-time line lengths 48, 96, 256 and 512 and the SNF grid of the
non-diagonal pattern M = [[128,32,0],[0,128,0],[0,0,64]] (32 x 64 x 512) are
checked element by element against the FP64 oracle in lock step (a fixed
iteration count on both sides):

* the non-diagonal pattern itself with the Dirichlet and dlVP kernels (the
  Green pass on 512-point lines, moment form), FP64 and FP32, RSA spheres of
  fraction 0.3 and contrast 100 (seed 3);
* the Box spline on a pattern with the same first two rows and SNF
  (4, 32, 512) (the Green pass on 512-point lines, table form), FP64 and FP32;
  at the full non-diagonal workload (R = 16, whose alias sums the oracle cannot
  evaluate at every bin in seconds) the table is compared at sampled bins and
  the converged C^eff through properties that hold at any size;
* the batched size classes n = 32, 48, 64, 96 in one lsh_solve_batch call in
  FP32, and the same patterns solved one by one in FP64;
* lines of 256 and 512 points along each axis;
* the 128^3 benchmark problem in FP32.

Tolerances: 1e-10 relative on E and sigma_bar for the FP64 path, 1e-5 for the
FP32 path (the targets of each precision), as in test_gpu_parity.py.
"""
import numpy as np
import pytest

import lsh_inputs as li
from helpers import BOX_CFG3, Problem, two_phase

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-10
FP32_TOL = 1e-5
CFG3_M = [[128, 32, 0], [0, 128, 0], [0, 0, 64]]
LOADS = np.eye(6)


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def rsa_phase(seed, frac, rmin=6.0, rmax=12.0):
    def f(Y):
        c, r = li.rsa_spheres(seed, li.lattice_unit(len(Y)), frac, rmin=rmin, rmax=rmax, max_attempts=200_000)
        return li.spheres_phase(Y, c, r)
    return f


_ORACLE = {}


def oracle_runs(key, pr, loads, n_iter):
    """Oracle lock-step results for the given load indices, cached per problem key."""
    out = {}
    for j in loads:
        k = (key, j, n_iter)
        if k not in _ORACLE:
            _ORACLE[k] = pr.oracle_solve(LOADS[j], n_iter=n_iter)
        out[j] = _ORACLE[k]
    return out


def check_against(pr, res, refs, tol):
    for j, ref in refs.items():
        assert rel(res["sigma"][j], ref["sigma_voigt"]) < tol, (j, rel(res["sigma"][j], ref["sigma_voigt"]))
        Eg = pr.gpu_E_to_oracle_mandel(res["E"][j].cpu().numpy())
        assert rel(Eg, ref["E"]) < tol, (j, rel(Eg, ref["E"]))


def lockstep_six_loads(pr, prec, n_iter, tuned=True):
    import torch
    pr.G.bind(prec)
    ws = torch.empty(pr.G.workspace_bytes(6), dtype=torch.uint8, device="cuda")
    if tuned:
        pr.G.autotune(nload=6, workspace=ws)
    else:
        pr.G.tune_reset()
    res = pr.G.solve(LOADS, tol=-1.0, max_iter=n_iter, return_E=True, workspace=ws, history=True)
    assert list(res["iterations"]) == [n_iter] * 6
    return res


# ------------------------------------------- the non-diagonal SNF grid ---
_CFG3 = {}


def cfg3_problem(kind):
    if kind not in _CFG3:
        Cp, C0 = two_phase(1.0, 100.0)
        params = {"alpha": [0.75] * 3} if kind == "dlvp" else {}
        _CFG3[kind] = Problem(CFG3_M, kind, params, rsa_phase(3, 0.3), Cp, C0)
    return _CFG3[kind]


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
@pytest.mark.parametrize("kind", ["dirichlet", "dlvp"])
def test_cfg3_grid_lockstep(kind, prec, tol):
    """SNF (32, 64, 512), six loads, 3 iterations, loads e11 and e23 against the oracle."""
    pr = cfg3_problem(kind)
    assert tuple(pr.G.e) == (32, 64, 512)
    res = lockstep_six_loads(pr, prec, 3)
    refs = oracle_runs(("cfg3", kind), pr, [0, 3], 3)
    check_against(pr, res, refs, tol)
    for j, ref in refs.items():
        np.testing.assert_allclose(res["history"][j], ref["history"], rtol=100 * tol)


_BOX512 = {}


def box512_problem():
    if "pr" not in _BOX512:
        Cp, C0 = two_phase(1.0, 100.0)
        _BOX512["pr"] = Problem([[128, 32, 0], [0, 128, 0], [0, 0, 4]], "box", {"Xi": BOX_CFG3["Xi"], "R": 1},
                                rsa_phase(5, 0.3, rmin=2.0, rmax=4.0), Cp, C0)
    pr = _BOX512["pr"]
    assert tuple(pr.G.e) == (4, 32, 512)
    return pr


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_box_512_lines_lockstep(prec, tol):
    """Box {e1,e2,e3,e1+e2} (R = 1) on M = [[128,32,0],[0,128,0],[0,0,4]], SNF
    (4, 32, 512): the tabled Green pass on 512-point lines, all six loads."""
    pr = box512_problem()
    res = lockstep_six_loads(pr, prec, 4)
    check_against(pr, res, oracle_runs("box512", pr, range(6), 4), tol)


@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
def test_box_512_lines_every_green_variant(prec, tol):
    """The same problem with each Green-pass variant built for the table form
    forced in turn (one load per block in chunks of six, three or two loads),
    all six loads, 4 iterations, against the oracle."""
    import torch
    pr = box512_problem()
    pr.G.bind(prec)
    ws = torch.empty(pr.G.workspace_bytes(6), dtype=torch.uint8, device="cuda")
    info = pr.G.autotune(nload=6, workspace=ws)
    ms = info["green"]["ms"]
    built = [c for c in range(len(ms)) if ms[c] > 0]
    assert len(built) >= 3, ms
    refs = oracle_runs("box512", pr, range(6), 4)
    for c in built:
        print(f"Green variant {c} {prec}", flush=True)
        pr.G.tune_set([info["stress"]["choice"], info["axis2"]["choice"], c, 0])
        res = pr.G.solve(LOADS, tol=-1.0, max_iter=4, return_E=True, workspace=ws, history=True)
        check_against(pr, res, refs, tol)
    pr.G.tune_reset()


@pytest.mark.parametrize("prec,atol", [("fp64", 5e-12), ("fp32", 2e-7)])
def test_cfg3_box_table_sampled_both_precisions(prec, atol):
    """The full workload's Box table (R = 16, 35,937 aliases per bin, double
    sums, stored at the path's precision) at 200 random bins against the oracle;
    the bins include the Nyquist planes and the origin."""
    from oracle import green
    from oracle.lattice import Pattern as OP
    from paper_1701_04685_amd import lsh
    P = lsh.Pattern(CFG3_M)
    Cp, C0 = two_phase(1.0, 100.0)
    P.set_kernel("box", BOX_CFG3)
    P.set_stiffness(Cp, C0, np.zeros(P.m, np.uint8))
    P.bind(prec)
    rng = np.random.default_rng(7)
    e = P.e
    bins = np.stack([rng.integers(0, e[0] // 2 + 1, 200), rng.integers(0, e[1], 200), rng.integers(0, e[2], 200)], 1)
    bins[0] = (0, 0, 0)
    bins[1] = (e[0] // 2, e[1] // 2, e[2] // 2)
    bins[2] = (e[0] // 2, 0, e[2] // 2)
    got = P.gamma_probe(bins)
    _, V = P.snf()
    ref, _ = green.gamma_symmetrised_at(OP(CFG3_M), C0, "box", BOX_CFG3, bins @ V)
    iu = np.triu_indices(6)
    np.testing.assert_allclose(got, ref[:, iu[0], iu[1]], rtol=0, atol=atol)


def test_cfg3_box_fullsize_properties():
    """The full non-diagonal Box workload (R = 16, RSA spheres seed 3, f = 0.3,
    contrast 100, six loads) solved to 1e-6: C^eff symmetric (exact for the
    fixed point, so within the iteration error) and the FP32 path equal to the
    FP64 path at the FP64 run's iteration counts within the FP32 bar."""
    import torch
    Cp, C0 = two_phase(1.0, 100.0)
    from paper_1701_04685_amd import lsh
    P = lsh.Pattern(CFG3_M)
    c, r = li.rsa_spheres(3, li.lattice_unit(P.m), 0.3)
    ph = li.spheres_phase(P.points(), c, r)
    P.set_kernel("box", BOX_CFG3)
    P.set_stiffness(Cp, C0, ph)
    P.bind("fp64")
    ws = torch.empty(P.workspace_bytes(6), dtype=torch.uint8, device="cuda")
    P.autotune(nload=6, workspace=ws)
    r64 = P.solve(LOADS, tol=1e-6, max_iter=3000, workspace=ws)
    assert np.all(r64["converged"])
    C64 = r64["sigma"].T
    assert np.linalg.norm(C64 - C64.T) / np.linalg.norm(C64) < 1e-5
    P.bind("fp32")
    ws32 = torch.empty(P.workspace_bytes(1), dtype=torch.uint8, device="cuda")
    P.autotune(nload=1, workspace=ws32)
    C32 = np.zeros((6, 6))
    for j in range(6):
        r32 = P.solve(LOADS[j:j + 1], tol=-1.0, max_iter=int(r64["iterations"][j]), workspace=ws32)
        C32[:, j] = r32["sigma"][0]
    assert rel(C32, C64) < FP32_TOL, rel(C32, C64)


# ----------------------------------------------------- batch size classes ---
_CFG4 = {}


def cfg4_problems():
    """One packing per size class, drawn like the batched workload (seed 4000 + i,
    radii 6-12 grid steps, fraction and contrast from the same ranges)."""
    if not _CFG4:
        for i, n in enumerate([32, 48, 64, 96]):
            rng = np.random.Generator(np.random.PCG64(4000 + i))
            frac = float(rng.uniform(0.1, 0.4))
            contrast = float(rng.uniform(5.0, 50.0))
            Cp, C0 = two_phase(1.0, contrast)
            _CFG4[n] = Problem(np.diag([n, n, n]), "dirichlet", {}, rsa_phase(4000 + i, frac), Cp, C0)
    return _CFG4


def test_cfg4_size_classes_batch_fp32_lockstep():
    """n = 32, 48, 64, 96 with six loads each in one lsh_solve_batch call (FP32,
    each class autotuned on its pattern as the benchmark does), 3 iterations:
    loads e11 and e12 of every instance against the oracle."""
    import torch
    from paper_1701_04685_amd import lsh
    prs = cfg4_problems()
    for n, pr in prs.items():
        pr.G.bind("fp32")
    nb = lsh.batch_workspace_bytes([pr.G for pr in prs.values()], [6] * len(prs), "fp32")
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    for pr in prs.values():
        pr.G.autotune(nload=6, workspace=ws)
    out = lsh.solve_batch([pr.G for pr in prs.values()], [LOADS] * len(prs), tol=-1.0, max_iter=3,
                          precision="fp32", workspace=ws, return_E=True)
    for (n, pr), o in zip(prs.items(), out):
        assert list(o["iterations"]) == [3] * 6
        check_against(pr, o, oracle_runs(("cfg4", n), pr, [0, 5], 3), FP32_TOL)


@pytest.mark.parametrize("n", [48, 96])
def test_cfg4_size_classes_fp64_lockstep(n):
    """The FP64 builds of the 48- and 96-point lines (stress, axis-2 and Green
    passes), autotuned, six loads, 3 iterations."""
    pr = cfg4_problems()[n]
    res = lockstep_six_loads(pr, "fp64", 3)
    check_against(pr, res, oracle_runs(("cfg4", n), pr, [0, 5], 3), FP64_TOL)


def test_batch_start_fields_mixed_with_zero_starts():
    """lsh_solve_batch with a start field for some tasks and a zero start for
    others, field output for all: each task equals the oracle started from the
    same field (mean removed), in lock step (FP64)."""
    import torch
    from oracle import green, scheme
    from paper_1701_04685_amd import lsh
    prs = [Problem(np.diag([8, 8, 8]), "dlvp", {"alpha": [0.5] * 3}, rsa_phase(41, 0.3, 1.0, 2.0)),
           Problem(np.diag([6, 6, 10]), "dirichlet", {}, rsa_phase(42, 0.3, 1.0, 2.0)),
           Problem(np.diag([8, 8, 8]), "dlvp", {"alpha": [0.5] * 3}, rsa_phase(43, 0.2, 1.0, 2.0))]
    eps = [np.eye(6)[[0, 3]], np.array([[0.1, 0.2, -0.3, 0.05, 0.0, 0.15]]), np.eye(6)[[1]]]
    rng = np.random.default_rng(44)
    starts, starts_o = [], []
    for i, (pr, e) in enumerate(zip(prs, eps)):
        pr.bind("fp64")
        if i == 1:
            starts.append(None)
            starts_o.append(None)
            continue
        Eo = rng.standard_normal((len(e), pr.O.m, 6)) * 0.05 + 0.01
        Ev = np.zeros((len(e), 6, pr.O.m))
        for j in range(len(e)):
            Ev[j][:, pr.q] = green.mandel_strain_to_voigt(Eo[j]).T
        starts.append(torch.tensor(Ev, device="cuda"))
        starts_o.append(Eo)
    out = lsh.solve_batch([pr.G for pr in prs], eps, tol=-1.0, max_iter=5, precision="fp64",
                          E_init=starts, return_E=True)
    for pr, e, o, Eo in zip(prs, eps, out, starts_o):
        for j in range(len(e)):
            ref = scheme.basic_scheme(pr.O, pr.gamma_oracle(), pr.Cp, pr.C0, pr.phase_o, e[j], n_iter=5,
                                      E_init=None if Eo is None else Eo[j])
            assert rel(o["sigma"][j], ref["sigma_voigt"]) < FP64_TOL
            assert rel(pr.gpu_E_to_oracle_mandel(o["E"][j].cpu().numpy()), ref["E"]) < FP64_TOL


# -------------------------------------------------- 256- and 512-point lines ---
LONG = [
    (np.diag([256, 16, 16]), "axis 1: 256"),
    (np.diag([16, 256, 16]), "axis 2: 256"),
    (np.diag([8, 16, 256]), "axis 3: 256"),
    (np.diag([512, 8, 16]), "axis 1: 512"),
    (np.diag([8, 512, 16]), "axis 2: 512"),
    (np.diag([4, 8, 512]), "axis 3: 512"),
]


@pytest.mark.parametrize("tuned", [False, True])
@pytest.mark.parametrize("prec,tol", [("fp64", FP64_TOL), ("fp32", FP32_TOL)])
@pytest.mark.parametrize("case", range(len(LONG)))
def test_long_lines_lockstep(case, prec, tol, tuned):
    M, _ = LONG[case]
    key = ("long", case)
    if key not in _ORACLE:
        _ORACLE[key] = Problem(M, "dlvp", {"alpha": [0.75] * 3}, rsa_phase(50 + case, 0.3, 1.5, 3.0))
    pr = _ORACLE[key]
    res = lockstep_six_loads(pr, prec, 4, tuned=tuned)
    check_against(pr, res, oracle_runs(key, pr, [0, 4], 4), tol)


# ------------------------------------------------------ 128^3 in FP32 ---
def test_cfg2_fullsize_fp32_lockstep():
    """The 128^3 dlVP benchmark problem (centred sphere f = 0.2, contrast 10) on
    the FP32 path, six loads autotuned, 3 iterations: load e11 against the oracle."""
    r = li.centred_sphere_radius(0.2)
    pr = Problem(np.diag([128, 128, 128]), "dlvp", {"alpha": [0.75] * 3},
                 lambda Y: li.sphere_phase(Y, np.zeros(3), r))
    res = lockstep_six_loads(pr, "fp32", 3)
    check_against(pr, res, oracle_runs("cfg2", pr, [0], 3), FP32_TOL)
