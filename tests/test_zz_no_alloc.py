"""The allocation-free entry point lsh_solve_noalloc against lsh_solve.

Called through the C ABI, twice in a row on one GPU (the second call smaller
than the first, so that whatever the first left in the fixed scratch array
must not leak into the second): sigma_bar, the residual history, iteration
counts and the output field equal lsh_solve's on the same inputs.  Both run the
same kernels in the same order on the same data, so the results agree to
rounding; the bar is the FP64 path's 1e-10 relative (FP32: 1e-5), as for the
parity tests.  Also: a solve beyond the array's size is refused before any
GPU work.
"""
import ctypes

import numpy as np
import pytest

import lsh_inputs as li
from helpers import Problem, two_phase

pytestmark = pytest.mark.gpu


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / max(np.linalg.norm(np.asarray(b)), 1e-300)


def noalloc_solve(lsh, P, eps, tol, max_iter, E_init=None):
    """lsh_solve_noalloc through the C ABI, with the same outputs as Pattern.solve."""
    import torch
    eps = np.ascontiguousarray(np.asarray(eps, dtype=np.float64).reshape(-1, P.nc))
    nload = eps.shape[0]
    Eout = torch.empty((nload, P.nc, P.m), dtype=torch.float64, device="cuda")
    sig = np.zeros((nload, P.nc))
    stats = (lsh.Stats * nload)()
    hist = np.full((nload, max_iter), np.nan)
    stream = torch.cuda.current_stream()
    rc = lsh._lib.lsh_solve_noalloc(P._h, nload, lsh._dptr(eps), float(tol), int(max_iter), P._prec,
                                    ctypes.c_void_p(stream.cuda_stream),
                                    ctypes.c_void_p(E_init.data_ptr()) if E_init is not None else None,
                                    ctypes.c_void_p(Eout.data_ptr()), lsh._dptr(sig), stats, lsh._dptr(hist))
    lsh._check(rc, allow=(-5,))
    return dict(sigma=sig, E=Eout, history=hist, iterations=np.array([s.iterations for s in stats]))


def compare(ref, got, tol):
    assert list(got["iterations"]) == list(ref["iterations"])
    assert rel(got["sigma"], ref["sigma"]) < tol
    assert rel(got["E"].cpu().numpy(), ref["E"].cpu().numpy()) < tol
    h0, h1 = ref["history"], got["history"]
    assert np.array_equal(np.isnan(h0), np.isnan(h1))
    np.testing.assert_allclose(h1[~np.isnan(h1)], h0[~np.isnan(h0)], rtol=tol)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
def test_noalloc_matches_solve_twice_second_smaller(prec, tol):
    from paper_1701_04685_amd import lsh
    big = Problem(np.diag([24, 20, 18]), "dlvp", {"alpha": [0.75] * 3},
                  lambda Y: (np.random.default_rng(1).random(len(Y)) < 0.3).astype(np.uint8))
    small = Problem(np.diag([8, 8, 8]), "dirichlet", {},
                    lambda Y: (np.random.default_rng(2).random(len(Y)) < 0.4).astype(np.uint8))
    big.bind(prec)
    small.bind(prec)
    loads_big = np.eye(6)
    loads_small = np.array([[0.3, -0.2, 0.1, 0.4, -0.1, 0.25]])
    for pr, loads in ((big, loads_big), (small, loads_small)):
        ref = pr.G.solve(loads, tol=1e-8, max_iter=400, return_E=True, history=True, allow_notconverged=True)
        got = noalloc_solve(lsh, pr.G, loads, 1e-8, 400)
        compare(ref, got, tol)


def test_noalloc_start_field_and_fixed_count():
    """A start field and the fixed-count mode (tol < 0) through the same array."""
    import torch
    from paper_1701_04685_amd import lsh
    pr = Problem(np.diag([12, 12, 12]), "dlvp", {"alpha": [0.5] * 3},
                 lambda Y: (np.random.default_rng(3).random(len(Y)) < 0.3).astype(np.uint8))
    pr.bind("fp64")
    rng = np.random.default_rng(4)
    E0 = torch.tensor(rng.standard_normal((2, 6, pr.G.m)) * 0.05, device="cuda")
    loads = np.eye(6)[[0, 4]]
    ref = pr.G.solve(loads, tol=-1.0, max_iter=7, E_init=E0, return_E=True, history=True)
    got = noalloc_solve(lsh, pr.G, loads, -1.0, 7, E_init=E0)
    compare(ref, got, 1e-10)


def test_noalloc_refuses_beyond_the_array():
    """128^3 with six loads in FP64 needs far more than the array holds: refused
    with LSH_EWORKSPACE before any GPU work, and the next call still works."""
    from paper_1701_04685_amd import lsh
    P = lsh.Pattern(np.diag([128, 128, 128]))
    Cp, C0 = two_phase()
    P.set_kernel("dirichlet")
    P.set_stiffness(Cp, C0, np.zeros(P.m, np.uint8))
    P.bind("fp64")
    assert P.workspace_bytes(6) > 64 * 1024 * 1024
    eps = np.eye(6)
    sig = np.zeros((6, 6))
    rc = lsh._lib.lsh_solve_noalloc(P._h, 6, lsh._dptr(np.ascontiguousarray(eps)), 1e-6, 10, P._prec, None, None,
                                    None, lsh._dptr(sig), None, None)
    assert rc == -8
    assert "allocation-free" in lsh._lib.lsh_last_error().decode()
    small = Problem(np.diag([8, 8, 8]), "dirichlet", {},
                    lambda Y: (np.random.default_rng(5).random(len(Y)) < 0.4).astype(np.uint8))
    small.bind("fp64")
    ref = small.G.solve(np.eye(6)[:1], tol=1e-10, max_iter=300, return_E=True, history=True)
    compare(ref, noalloc_solve(lsh, small.G, np.eye(6)[:1], 1e-10, 300), 1e-10)
