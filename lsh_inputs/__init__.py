"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only builds inputs: isotropic phase stiffnesses from (E, nu),
phase maps from point coordinates (laminates, spheres, random sequential
addition sphere packings) and load cases.  It holds none of the solver's
arithmetic: point coordinates are passed in by the caller, who takes them from
its own pattern code.

Geometry: the unit cell is the torus [-1/2, 1/2)^3; a point is inside a sphere
if its periodic minimum-image distance to the centre is below the radius.
"""
from __future__ import annotations

import numpy as np


def lame(E, nu):
    """Lame constants (lambda, mu) of an isotropic material."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return lam, mu


def isotropic_voigt(E, nu):
    """6x6 Voigt stiffness (order 11,22,33,23,13,12; tensor components)."""
    lam, mu = lame(E, nu)
    C = np.zeros((6, 6))
    C[:3, :3] = lam
    C[0, 0] = C[1, 1] = C[2, 2] = lam + 2 * mu
    C[3, 3] = C[4, 4] = C[5, 5] = mu
    return C


def isotropic_voigt_plane(E, nu):
    """3x3 Voigt stiffness (order 11, 22, 12; tensor components) of an isotropic
    material in plane strain: the in-plane block of the three-dimensional one."""
    return isotropic_voigt(E, nu)[np.ix_([0, 1, 5], [0, 1, 5])]


def confocal_ellipses_phase(points, c=(0.05, 0.35), rho=0.09, angle_deg=60.0):
    """Two confocal ellipses x1^2/(c1^2 + r) + x2^2/(c2^2 + r) = 1, r = 0 (core)
    and r = rho (coating), rotated by angle_deg about the cell centre, in the
    periodic cell [-1/2, 1/2)^2: phase 0 core, 1 coating, 2 matrix."""
    y = np.asarray(points, dtype=np.float64)
    y = y - np.round(y)
    t = np.deg2rad(angle_deg)
    # coordinates in the frame of the unrotated ellipses
    u = np.cos(t) * y[:, 0] + np.sin(t) * y[:, 1]
    v = -np.sin(t) * y[:, 0] + np.cos(t) * y[:, 1]
    inner = u ** 2 / c[0] ** 2 + v ** 2 / c[1] ** 2 <= 1.0
    outer = u ** 2 / (c[0] ** 2 + rho) + v ** 2 / (c[1] ** 2 + rho) <= 1.0
    return np.where(inner, 0, np.where(outer, 1, 2)).astype(np.uint8)


def mean_reference(C_phases):
    """Reference stiffness C0 = arithmetic mean of the phase stiffnesses."""
    return np.mean(np.asarray(C_phases, dtype=np.float64), axis=0)


def laminate_phase(points, axis=0):
    """Two-phase laminate: phase 1 where y_axis >= 0, else phase 0 (layers normal to e_axis)."""
    y = np.asarray(points)
    return (y[:, axis] >= 0).astype(np.uint8)


def _periodic_dist2(points, center):
    d = np.asarray(points, dtype=np.float64) - np.asarray(center, dtype=np.float64)[None, :]
    d -= np.round(d)
    return np.einsum("ij,ij->i", d, d)


def sphere_phase(points, center, radius):
    """Phase 1 inside the periodic sphere, 0 outside."""
    return (_periodic_dist2(points, center) < radius * radius).astype(np.uint8)


def centred_sphere_radius(fraction):
    """Radius (cell units) of one sphere of the given volume fraction."""
    return (3.0 * fraction / (4.0 * np.pi)) ** (1.0 / 3.0)


def rsa_spheres(seed, lattice_unit, fraction, rmin=6.0, rmax=12.0, max_attempts=1_000_000):
    """Random sequential addition of non-overlapping periodic spheres.

    Radii r ~ U[rmin, rmax] * lattice_unit, centres ~ U[-1/2, 1/2)^3, PRNG
    numpy PCG64(seed).  A sphere is accepted if its periodic distance to every
    accepted sphere is at least the sum of radii.  Stops when the summed
    sphere volume reaches ``fraction``; the last radius is shrunk to hit it
    exactly while it stays >= rmin * lattice_unit.  Returns (centres (k,3), radii (k,)).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    centres, radii = [], []
    vol = 0.0
    target = float(fraction)
    rlo = rmin * lattice_unit
    attempts = 0
    batch = 2048
    while attempts < max_attempts and vol < target:
        # draws in the same order as one attempt at a time: r, c0, c1, c2
        u = rng.random((batch, 4))
        cand_r = (rmin + (rmax - rmin) * u[:, 0]) * lattice_unit
        cand_c = -0.5 + u[:, 1:]
        # candidates already overlapping an accepted sphere at their largest radius
        if centres:
            C = np.array(centres)
            d = cand_c[:, None, :] - C[None, :, :]
            d -= np.round(d)
            dist = np.sqrt(np.einsum("kij,kij->ki", d, d))
            hit = np.any(dist < np.array(radii)[None, :] + cand_r[:, None], axis=1)
        else:
            hit = np.zeros(batch, dtype=bool)
        vk = 4.0 / 3.0 * np.pi * cand_r ** 3
        k = 0
        while k < batch and attempts < max_attempts and vol < target:
            # next candidate that is not already excluded (or that the final
            # shrink could still admit); the skipped ones count as attempts
            live = np.flatnonzero(~hit[k:] | (vk[k:] > target - vol))
            if len(live) == 0:
                attempts += batch - k
                break
            j = k + int(live[0])
            attempts += j - k
            if attempts >= max_attempts:
                break
            attempts += 1
            k = j + 1
            r = cand_r[j]
            c = cand_c[j]
            rest = target - vol
            v = vk[j]
            if v > rest:
                r_fit = (3.0 * rest / (4.0 * np.pi)) ** (1.0 / 3.0)
                if r_fit >= rlo:
                    r = r_fit
                    v = rest
            if centres:
                C = np.array(centres)
                d = C - c[None, :]
                d -= np.round(d)
                if np.any(np.sqrt(np.einsum("ij,ij->i", d, d)) < np.array(radii) + r):
                    continue
            centres.append(c)
            radii.append(r)
            vol += v
    return np.array(centres).reshape(-1, 3), np.array(radii)


def spheres_phase(points, centres, radii):
    """Phase 1 inside any of the spheres."""
    y = np.asarray(points, dtype=np.float64)
    ph = np.zeros(len(y), dtype=np.uint8)
    for c, r in zip(np.asarray(centres), np.asarray(radii)):
        ph |= (_periodic_dist2(y, c) < r * r).astype(np.uint8)
    return ph


def unit_loads():
    """The six unit Voigt strains (engineering shear); columns of C^eff."""
    return np.eye(6)


def random_unit_load(rng):
    """A Voigt strain drawn uniformly on the unit 6-sphere."""
    v = rng.standard_normal(6)
    return v / np.linalg.norm(v)


def lattice_unit(m):
    """Length of one lattice step of an m-point pattern in cell units: m^{-1/3}."""
    return float(m) ** (-1.0 / 3.0)


def grid_points_numerators(n):
    """Numerators (over n^3) of the points of the regular n x n x n pattern in
    row-major index order, each coordinate a_i/n wrapped into [-1/2, 1/2).
    Used to check that a pattern's storage order is this plain grid order."""
    a = np.arange(n)
    c = ((a + n // 2) % n) - n // 2           # a/n wrapped, times n
    g = np.stack(np.meshgrid(c, c, c, indexing="ij"), -1).reshape(-1, 3)
    return g.astype(np.int64) * (n * n)


def spheres_phase_grid(n, centres, radii):
    """spheres_phase for the regular n^3 grid in row-major order, touching only
    each sphere's bounding box (same inside rule: periodic distance < r)."""
    ph = np.zeros((n, n, n), dtype=np.uint8)
    for c, r in zip(np.asarray(centres), np.asarray(radii)):
        rg = int(np.ceil(r * n)) + 1
        axes = []
        for i in range(3):
            k0 = int(np.floor(c[i] * n))
            ks = np.arange(k0 - rg, k0 + rg + 2)
            y = ks / n
            d = y - c[i]
            d -= np.round(d)
            axes.append((ks % n, d))
        (i0, d0), (i1, d1), (i2, d2) = axes
        inside = (d0[:, None, None] ** 2 + d1[None, :, None] ** 2 + d2[None, None, :] ** 2) < r * r
        ii = np.ix_(i0, i1, i2)
        ph[ii] |= inside.astype(np.uint8)
    return ph.reshape(-1)


def unet_init_params(seed, layers):
    """Initial U-Net parameters (float32): He-normal weights [t][co][ci] per layer
    in layer order, then zero biases; layers = [(cin, cout, ks), ...]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ws, bs = [], []
    for cin, cout, ks in layers:
        fan_in = ks ** 3 * cin
        ws.append((rng.standard_normal(ks ** 3 * cin * cout) * np.sqrt(2.0 / fan_in)).astype(np.float32))
        bs.append(np.zeros(cout, dtype=np.float32))
    return np.concatenate(ws + bs)
