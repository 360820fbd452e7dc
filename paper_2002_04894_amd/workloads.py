"""Seeded synthetic point clouds and charges.

This module only draws inputs; it holds none of the method's arithmetic, so
both the CPU reference (test infrastructure) and the GPU path may consume its
output.  The paper runs on synthetic distributions only (uniform cube,
spherical Gaussian, shell, helix, galaxy; Section 3.2 and Section 3.3); the
shapes below follow those workloads and the configurations benchmarked here.

Every generator uses NumPy's PCG64 (`numpy.random.default_rng(seed)`), draws
positions before charges, and returns float64 SoA arrays (x, y, z, q).
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "uniform_cube",
    "gaussian_mixture",
    "plummer",
    "sphere_surface",
    "spherical_gaussian",
    "spherical_shell",
    "helix",
    "workload",
    "WORKLOADS",
    "sample_targets",
    "RESPONSE_DISTRIBUTIONS",
]


def _charges(rng: np.random.Generator, n: int, kind: str) -> np.ndarray:
    if kind == "pm1":  # uniform in [-1, 1]
        return rng.uniform(-1.0, 1.0, n)
    if kind == "pos":  # uniform in (0, 1]
        return 1.0 - rng.random(n)
    raise ValueError(f"unknown charge kind {kind!r}")


def uniform_cube(n: int, seed: int = 0, charges: str = "pm1"):
    """N points uniform in [0,1)^3 (an (N,3) draw), charges after positions."""
    rng = np.random.default_rng(seed)
    pts = rng.random((n, 3))
    q = _charges(rng, n, charges)
    return (np.ascontiguousarray(pts[:, 0]), np.ascontiguousarray(pts[:, 1]),
            np.ascontiguousarray(pts[:, 2]), q)


def gaussian_mixture(n: int, seed: int = 0, sigmas=(0.01, 0.03, 0.1, 0.2),
                     charges: str = "pm1"):
    """Isotropic Gaussian mixture: centres uniform in [0,1)^3, one sigma per
    component, n/len(sigmas) points per component (the remainder goes to the
    last one), concatenated, unclipped."""
    rng = np.random.default_rng(seed)
    k = len(sigmas)
    centres = rng.random((k, 3))
    counts = [n // k] * k
    counts[-1] += n - sum(counts)
    parts = []
    for c, s, m in zip(centres, sigmas, counts):
        parts.append(c + s * rng.standard_normal((m, 3)))
    pts = np.concatenate(parts, axis=0)
    q = _charges(rng, n, charges)
    return (np.ascontiguousarray(pts[:, 0]), np.ascontiguousarray(pts[:, 1]),
            np.ascontiguousarray(pts[:, 2]), q)


def plummer(n: int, a: float = 0.05, rmax: float = 1.0, seed: int = 0,
            charges: str = "pos"):
    """Plummer sphere of scale radius `a`, truncated at radius `rmax`, by
    inverse-CDF sampling of the enclosed fraction, isotropic directions."""
    rng = np.random.default_rng(seed)
    u_max = (rmax * rmax / (rmax * rmax + a * a)) ** 1.5  # enclosed fraction at rmax
    u = u_max * (1.0 - rng.random(n))                      # in (0, u_max]
    r = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    pts = d * r[:, None]
    q = _charges(rng, n, charges)
    return (np.ascontiguousarray(pts[:, 0]), np.ascontiguousarray(pts[:, 1]),
            np.ascontiguousarray(pts[:, 2]), q)


def sphere_surface(n: int, seed: int = 0, charges: str = "pm1"):
    """Points on the unit sphere surface (normalised Gaussian vectors)."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    q = _charges(rng, n, charges)
    return (np.ascontiguousarray(d[:, 0]), np.ascontiguousarray(d[:, 1]),
            np.ascontiguousarray(d[:, 2]), q)


def spherical_gaussian(n: int, seed: int = 0, sigma: float = 1.0, charges: str = "pm1"):
    """One isotropic Gaussian about the origin, standard deviation `sigma`
    per axis (the spherical Gaussian of Section 3.2)."""
    rng = np.random.default_rng(seed)
    pts = sigma * rng.standard_normal((n, 3))
    q = _charges(rng, n, charges)
    return (np.ascontiguousarray(pts[:, 0]), np.ascontiguousarray(pts[:, 1]),
            np.ascontiguousarray(pts[:, 2]), q)


def spherical_shell(n: int, seed: int = 0, r_in: float = 0.9, r_out: float = 1.0,
                    charges: str = "pm1"):
    """Points uniform in the volume between radii r_in and r_out (the
    spherical shell of Section 3.2): radius by inverse CDF, r^3 uniform
    between r_in^3 and r_out^3, then an isotropic direction."""
    rng = np.random.default_rng(seed)
    u = rng.random(n)
    r = np.cbrt(r_in ** 3 + u * (r_out ** 3 - r_in ** 3))
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    pts = d * r[:, None]
    q = _charges(rng, n, charges)
    return (np.ascontiguousarray(pts[:, 0]), np.ascontiguousarray(pts[:, 1]),
            np.ascontiguousarray(pts[:, 2]), q)


def helix(n: int, seed: int = 0, turns: float = 5.0, radius: float = 1.0, height: float = 2.0,
          jitter: float = 0.02, charges: str = "pm1"):
    """Points along a circular helix about the z axis (the helix of Section
    3.2): parameter t uniform in [0, 1), angle 2*pi*turns*t, z from
    -height/2 to height/2, then an isotropic Gaussian offset of standard
    deviation `jitter` per axis."""
    rng = np.random.default_rng(seed)
    t = rng.random(n)
    a = 2.0 * np.pi * turns * t
    pts = np.stack([radius * np.cos(a), radius * np.sin(a), height * (t - 0.5)], axis=1)
    pts += jitter * rng.standard_normal((n, 3))
    q = _charges(rng, n, charges)
    return (np.ascontiguousarray(pts[:, 0]), np.ascontiguousarray(pts[:, 1]),
            np.ascontiguousarray(pts[:, 2]), q)


# The four distributions of the parameter-response study (Section 3.2).
RESPONSE_DISTRIBUTIONS = {
    "cube": uniform_cube,
    "gaussian": spherical_gaussian,
    "shell": spherical_shell,
    "helix": helix,
}


# Named workloads: sizes, parameters and generator of each benchmarked case.
WORKLOADS = {
    # uniform cube, 20,000 points, 3 levels (512 leaves), theta 0.5, p 10
    "uniform20k": dict(gen="uniform", n=20_000, seed=0, levels=3, theta=0.5, p=10),
    # 4-component Gaussian mixture, 2^20 points, 5 levels, theta 0.5, p 15
    "gmix1m": dict(gen="gmix", n=1 << 20, seed=0, levels=5, theta=0.5, p=15),
    # Plummer a=0.05, 2^24 points, 6 levels
    "plummer16m": dict(gen="plummer", n=1 << 24, seed=0, levels=6, theta=0.5, p=12, a=0.05),
    # Plummer a=0.02, 2^27 points, 7 levels, charges in [-1, 1]
    "plummer134m": dict(gen="plummer", n=1 << 27, seed=0, levels=7, theta=0.5, p=12, a=0.02,
                        charges="pm1"),
}


def workload(name: str, n: int | None = None):
    """Return (x, y, z, q, params) for a named workload; `n` overrides the size."""
    w = dict(WORKLOADS[name])
    if n is not None:
        w["n"] = int(n)
    g = w["gen"]
    if g == "uniform":
        arrs = uniform_cube(w["n"], w["seed"])
    elif g == "gmix":
        arrs = gaussian_mixture(w["n"], w["seed"])
    elif g == "plummer":
        arrs = plummer(w["n"], a=w.get("a", 0.05), seed=w["seed"],
                       charges=w.get("charges", "pos"))
    else:
        raise ValueError(g)
    return (*arrs, w)


def sample_targets(n: int, k: int, seed: int = 1) -> np.ndarray:
    """k distinct target indices in [0, n), sorted (int64)."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, k, replace=False)).astype(np.int64)
