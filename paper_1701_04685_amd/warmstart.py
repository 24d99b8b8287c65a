"""Learned warm start for the Basic Scheme (Sec. 4): data, training, evaluation.

The Basic Scheme converges from any start field; its iteration count depends
on how far the start is from the fixed point.  The fixed point of
eq. (pde_coefficients) is linear in the macroscopic strain eps0, so a network
that maps the phase map to the six unit-load fluctuation fields predicts the
start for every eps0 (include/lsh_unet.h).  Everything numerical runs in the
library's kernels: the solver produces the training fields, the U-Net kernels
train on them, and the solver's Cauchy residual judges each prediction.

Fallback: the learned start and the zero start run side by side for `check`
iterations; the solve continues from the learned iterate only if its residual
has not grown and is below the zero start's, else from the zero start's
iterate.  Resuming from an iterate continues the same iteration (the scheme's
state is the field E alone).
"""
from __future__ import annotations

import time

import numpy as np

import lsh_inputs as li
from . import lsh

# two-phase isotropic microstructure of the learned-start workload
MATRIX = (1.0, 0.3)


def grid_pattern(n, phase, contrast, kind="dirichlet", kparams=None, precision="fp32"):
    """A bound pattern for M = diag(n, n, n) with the phase map in grid order."""
    P = lsh.Pattern(np.diag([n, n, n]))
    P.set_kernel(kind, kparams if kparams is not None else ({"alpha": [0.75] * 3} if kind == "dlvp" else None))
    C = [li.isotropic_voigt(*MATRIX), li.isotropic_voigt(MATRIX[0] * contrast, MATRIX[1])]
    P.set_stiffness(C, li.mean_reference(C), phase)
    P.bind(precision)
    return P


def check_grid_order(P, n):
    """The U-Net reads fields in plain (z, y, x) grid order; for M = diag(n, n, n)
    the pattern's storage order must be that order."""
    if not np.array_equal(P.point_numerators(), li.grid_points_numerators(n)):
        raise RuntimeError("pattern storage order is not the plain grid order")


def packing(seed, n, fraction=0.3, rmin=6.0, rmax=12.0):
    """Seeded random sphere packing on the n^3 grid (radii in grid steps)."""
    c, r = li.rsa_spheres(seed, 1.0 / n, fraction, rmin=rmin, rmax=rmax)
    return li.spheres_phase_grid(n, c, r)


def unit_load_fields(P, tol=1e-6, max_iter=3000, workspace=None):
    """Fluctuation fields [6][6][m] (Voigt) of the six unit Voigt loads.  A load
    that stops at max_iter (the FP32 path's residual floor can sit near tol)
    still gives a field accurate far beyond what training needs."""
    out = P.solve(li.unit_loads(), tol=tol, max_iter=max_iter, return_E=True, workspace=workspace,
                  allow_notconverged=True)
    return out["E"], out


def make_dataset(seeds, n, contrast, tol=1e-6, fraction=0.3, rmin=6.0, rmax=12.0, log=None):
    """(phase, target) device pairs: phase uint8 [n^3], target float32 [n^3][36]."""
    import torch
    data = []
    iters = []
    for k, s in enumerate(seeds):
        ph = packing(s, n, fraction, rmin, rmax)
        P = grid_pattern(n, ph, contrast)
        if k == 0:
            check_grid_order(P, n)
        E, out = unit_load_fields(P, tol=tol)
        iters.append(int(out["iterations"].max()))
        T = lsh.UNet.pack_target(E, n)
        data.append((torch.from_numpy(ph).cuda(), T))
        del P, E
        if log and (k + 1) % 50 == 0:
            log(f"dataset {k + 1}/{len(seeds)} packings, max iterations {iters[-1]}")
    return data, np.array(iters)


def train(net, data, n, epochs, lr=1e-3, lr_final=1e-4, seed=0, log=None):
    """Adam over the samples in a seeded order per epoch, learning rate decayed
    geometrically from lr to lr_final.  Returns the mean loss per epoch."""
    rng = np.random.Generator(np.random.PCG64(seed))
    total = epochs * len(data)
    step = 0
    means = []
    for ep in range(epochs):
        order = rng.permutation(len(data))
        ls = []
        for i in order:
            a = lr * (lr_final / lr) ** (step / max(total - 1, 1))
            ph, T = data[i]
            ls.append(net.train_step(ph, T, n, a))
            step += 1
        means.append(float(np.mean(ls)))
        if log:
            log(f"epoch {ep + 1}/{epochs} mean loss {means[-1]:.4e}")
    return np.array(means)


def residual_grew(history, check):
    """Fallback rule over the first `check` residuals of a solve (NaN marks
    iterations after it stopped): true if one is infinite or the last exceeds
    the first."""
    h = np.asarray(history[:check], dtype=np.float64)
    h = h[~np.isnan(h)]
    if h.size == 0 or not np.all(np.isfinite(h)):
        return True
    return bool(h[-1] > h[0])


def solve_plain(P, eps0, tol=1e-6, max_iter=3000, workspace=None):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = P.solve(eps0, tol=tol, max_iter=max_iter, workspace=workspace, allow_notconverged=True)
    t = time.perf_counter() - t0
    return dict(seconds=t, iterations=int(out["iterations"][0]), sigma=out["sigma"][0],
                converged=bool(out["converged"][0]))


def solve_learned(P, net, phase_dev, n, eps0, tol=1e-6, max_iter=3000, check=10, workspace=None, E_start=None):
    """Learned start (inference included in the time) judged against the zero start.

    The first `check` iterations run the learned start and the zero start side
    by side (two load cases of one solve with the same eps0).  The solve then
    continues from the learned iterate only if its residual has not grown and
    is below the zero start's; otherwise it continues from the zero start's
    iterate (the fallback).  E_start, if given, replaces the network's
    prediction (used to exercise the fallback with a start known to be bad).
    """
    import torch
    eps0 = np.reshape(np.asarray(eps0, dtype=np.float64), 6)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # the prediction for the pair (eps0, 0) is (learned start, zero start)
    pair = np.stack([eps0, np.zeros(6)])
    if E_start is None:
        E0 = net.predict(phase_dev, n, pair)
    else:
        E0 = torch.zeros((2, 6, P.m), dtype=torch.float64, device="cuda")
        E0[0].copy_(E_start.reshape(6, P.m))
    both = np.stack([eps0, eps0])
    try:
        first = P.solve(both, tol=tol, max_iter=check, E_init=E0, return_E=True, history=True,
                        workspace=workspace, allow_notconverged=True)
    except lsh.LshError as e:
        if e.status != -6:            # a non-finite residual sends the solve to the fallback
            raise
        first = None
    if first is None:
        pick, its0 = 1, 0
        out = P.solve(eps0, tol=tol, max_iter=max_iter, workspace=workspace, allow_notconverged=True)
    else:
        r = first["residual"]
        hist = first["history"]
        good = (not residual_grew(hist[0], check)) and np.isfinite(r[0])
        pick = 0 if good and (first["converged"][0] or r[0] <= r[1]) else 1
        its0 = int(first["iterations"][pick])
        if first["converged"][pick]:
            out = dict(sigma=first["sigma"][pick:pick + 1], iterations=np.array([0]),
                       converged=np.array([True]))
        else:
            out = P.solve(eps0, tol=tol, max_iter=max_iter - its0, E_init=first["E"][pick:pick + 1],
                          workspace=workspace, allow_notconverged=True)
    t = time.perf_counter() - t0
    return dict(seconds=t, iterations=its0 + int(out["iterations"][0]), sigma=out["sigma"][0],
                converged=bool(out["converged"][0]), fell_back=pick == 1)
