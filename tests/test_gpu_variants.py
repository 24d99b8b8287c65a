"""Every kernel variant the autotuner can pick gives the oracle's iterates.

lsh_tune_set forces each combination of variants (stress pass plain or
fused, axis-2 tile width, one or two load cases per Green-pass block) on a
pattern whose SNF line lengths all have variants, and the lock-step run is
compared with the FP64 oracle as in test_gpu_parity (7 iterations, FP64
1e-10 / FP32 1e-5 relative).  lsh_autotune itself must report a valid choice
and keep the answer.
"""
import itertools

import numpy as np
import pytest

import lsh_inputs as li
from helpers import Problem

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "fp32": 1e-5}
EPS0 = np.array([0.3, -0.2, 0.1, 0.4, -0.1, 0.25])


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def spheres(seed, frac=0.3):
    def f(Y):
        c, r = li.rsa_spheres(seed, li.lattice_unit(len(Y)), frac, rmin=1.5, rmax=3.0)
        return li.spheres_phase(Y, c, r)
    return f


@pytest.fixture(scope="module", params=[("dlvp", {"alpha": [0.75] * 3}),
                                        ("box", {"Xi": np.array([[1, 0, 0, 1], [0, 1, 0, 1], [0, 0, 1, 0]], float),
                                                 "R": 2})])
def problem(request):
    kind, params = request.param
    pr = Problem(np.diag([16, 32, 64]), kind, params, spheres(31))
    ref = pr.oracle_solve(EPS0, n_iter=7)
    return pr, ref


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_every_variant_matches_oracle(problem, prec):
    pr, ref = problem
    pr.bind(prec)
    info = pr.G.autotune(nload=1)           # reports how many candidates each pass has
    ncand = [len(info[k]["ms"]) for k in ("stress", "axis2", "green")]
    assert ncand[0] >= 5 and ncand[1] >= 3 and ncand[2] >= 2, ncand
    for choice in itertools.product(*(range(n) for n in ncand)):
        print(f"variant {choice} {prec}", flush=True)
        pr.G.tune_set(choice)
        res = pr.G.solve(EPS0[None], tol=-1.0, max_iter=7, return_E=True, history=True)
        Eg = pr.gpu_E_to_oracle_mandel(res["E"].cpu().numpy()[0])
        assert rel(res["sigma"][0], ref["sigma_voigt"]) < TOL[prec], choice
        assert rel(Eg, ref["E"]) < TOL[prec], choice
        np.testing.assert_allclose(res["history"][0], ref["history"], rtol=100 * TOL[prec], atol=1e-14)
    pr.G.tune_reset()


def test_autotune_choice_and_answer(problem):
    pr, ref = problem
    pr.bind("fp64")
    info = pr.G.autotune(nload=1)
    for name in ("stress", "axis2", "green"):
        ms = info[name]["ms"]
        assert len(ms) >= 1 and all(t > 0 for t in ms)
        assert 0 <= info[name]["choice"] < len(ms)
        assert ms[info[name]["choice"]] == min(ms)
    res = pr.G.solve(EPS0[None], tol=-1.0, max_iter=7, return_E=True)
    assert rel(res["sigma"][0], ref["sigma_voigt"]) < TOL["fp64"]
    pr.G.tune_reset()


@pytest.mark.parametrize("kind,params", [("dlvp", {"alpha": [0.75] * 3}), ("dirichlet_modified", {}),
                                         ("dirichlet", {})])
def test_green_variants_fp64_128_lines(kind, params):
    """FP64 Green pass on 128-point lines (the benchmark's length), where the
    variants differ in loads per block, wave cap and loads per chunk (even
    lengths: the -1/2 faces take the Hermitian part): every Green variant
    against the oracle in lock step."""
    pr = Problem(np.diag([4, 8, 128]), kind, params, spheres(33))
    assert tuple(pr.G.e) == (4, 8, 128)
    ref = pr.oracle_solve(EPS0, n_iter=5)
    pr.bind("fp64")
    info = pr.G.autotune(nload=2)
    ng = len(info["green"]["ms"])
    assert ng >= 4, info["green"]
    for c in range(ng):
        pr.G.tune_set([0, 0, c])
        res = pr.G.solve(EPS0[None], tol=-1.0, max_iter=5, return_E=True)
        Eg = pr.gpu_E_to_oracle_mandel(res["E"].cpu().numpy()[0])
        assert rel(res["sigma"][0], ref["sigma_voigt"]) < TOL["fp64"], c
        assert rel(Eg, ref["E"]) < TOL["fp64"], c
    pr.G.tune_reset()


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_green_chunk_variants_512_lines(prec):
    """512-point lines: Green-pass variants that split the six loads into
    chunks of three or two (more blocks, the position's operator formed once
    per chunk) against the oracle, all six loads in lock step."""
    pr = Problem(np.diag([4, 8, 512]), "dlvp", {"alpha": [0.75] * 3}, spheres(34))
    assert tuple(pr.G.e) == (4, 8, 512)
    loads = np.eye(6)
    refs = [pr.oracle_solve(loads[j], n_iter=4) for j in range(6)]
    pr.bind(prec)
    info = pr.G.autotune(nload=6)
    ng = len(info["green"]["ms"])
    assert ng >= 3, info["green"]
    for c in range(ng):
        pr.G.tune_set([0, 0, c])
        res = pr.G.solve(loads, tol=-1.0, max_iter=4, return_E=True)
        for j in range(6):
            Eg = pr.gpu_E_to_oracle_mandel(res["E"][j].cpu().numpy())
            assert rel(res["sigma"][j], refs[j]["sigma_voigt"]) < TOL[prec], (c, j)
            assert rel(Eg, refs[j]["E"]) < TOL[prec], (c, j)
    pr.G.tune_reset()
