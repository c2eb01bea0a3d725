"""Seeded synthetic inputs for the point-charge Laplace FMM workloads.

This module holds random-number recipes only: no part of the method's
arithmetic lives here.  Both the GPU library's tests/benchmark and the CPU
oracle draw their inputs from these functions, so both sides see the same
FP64 bits.  Every generator uses numpy's PCG64 (``numpy.random.default_rng``)
and draws positions first, then charges, then any sample indices.

Workloads (the paper measures only synthetic distributions: points uniform in
a cube and on a sphere surface, Sec. III.A; the non-uniform, batched and
Plummer sets below are synthetic stress cases of the same method):

* ``uniform_cube``      -- positions U[0,1)^3, charges U[-1,1)
* ``clustered``         -- 8 isotropic Gaussians (sigma=0.01) around random
                           centres in the unit cube plus 5% of the points on a
                           unit sphere shell centred at (0.5,0.5,0.5); charges
                           +-1 with equal probability
* ``plummer``           -- Plummer sphere of scale a (radius drawn by inverting
                           the cumulative mass profile), isotropic directions,
                           charges in (0,1]
* ``uneven_problem_sizes`` -- problem sizes log-uniform in [1e4, 5e5]
* ``sphere_surface``    -- positions uniform on a sphere surface (the
                           paper's second distribution, Sec. III.A),
                           charges U[-1,1)
* ``shielding``         -- the active-shielding geometry of Sec. III.B:
                           128 shield charges spaced regularly on a sphere of
                           radius 2, 256 external charges of random position
                           on a sphere of radius 5 and random charge, 1024
                           probes evenly on radius 1.5 and 1024 on radius 2.5
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "uniform_cube",
    "clustered",
    "plummer",
    "uneven_problem_sizes",
    "sample_targets",
    "sphere_surface",
    "fibonacci_sphere",
    "shielding",
    "WORKLOADS",
]


def uniform_cube(n: int, seed: int = 0, nrhs: int = 0):
    """Positions uniform in the unit cube, charges uniform in [-1, 1).

    Returns ``(pos[n,3] f64, q)`` where ``q`` is ``[n]`` when ``nrhs == 0``
    and ``[nrhs, n]`` otherwise.
    """
    rng = np.random.default_rng(seed)
    pos = rng.random((n, 3))
    if nrhs:
        q = rng.uniform(-1.0, 1.0, (nrhs, n))
    else:
        q = rng.uniform(-1.0, 1.0, n)
    return pos, q


def clustered(n: int, seed: int = 0, n_clusters: int = 8, sigma: float = 0.01,
              shell_frac: float = 0.05):
    """Mixture of isotropic Gaussians plus points on a unit sphere shell.

    Draw order: cluster centres, shell directions, cluster labels, Gaussian
    offsets, then charges.  Returns ``(pos[n,3], q[n])`` with q = +-1.
    """
    rng = np.random.default_rng(seed)
    centres = rng.random((n_clusters, 3))
    n_shell = int(round(shell_frac * n))
    n_cl = n - n_shell
    g = rng.standard_normal((n_shell, 3))
    g /= np.sqrt((g * g).sum(axis=1))[:, None]
    shell = 0.5 + g
    lab = rng.integers(0, n_clusters, n_cl)
    cl = centres[lab] + sigma * rng.standard_normal((n_cl, 3))
    pos = np.concatenate([shell, cl], axis=0)
    q = (2 * rng.integers(0, 2, n) - 1).astype(np.float64)
    return pos, q


def plummer(n: int, seed: int = 0, a: float = 0.1):
    """Plummer-sphere positions (scale ``a``, centred at the origin, no
    truncation) and charges in (0, 1].

    The radius inverts the enclosed-mass fraction U = r^3/(r^2+a^2)^{3/2}:
    r = a / sqrt(U^{-2/3} - 1).  U = 0 is redrawn as the smallest positive
    double so that r > 0.
    """
    rng = np.random.default_rng(seed)
    u = rng.random(n)
    u = np.where(u <= 0.0, np.finfo(np.float64).tiny, u)
    r = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
    d = rng.standard_normal((n, 3))
    d /= np.sqrt((d * d).sum(axis=1))[:, None]
    pos = r[:, None] * d
    q = 1.0 - rng.random(n)
    return pos, q


def sphere_surface(n: int, seed: int = 0, radius: float = 1.0, centre=(0.0, 0.0, 0.0)):
    """Positions uniform on the sphere |x - centre| = radius (normalised
    standard normal vectors), charges uniform in [-1, 1)."""
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((n, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    pos = np.asarray(centre, dtype=np.float64) + radius * v
    q = rng.uniform(-1.0, 1.0, n)
    return pos, q


def fibonacci_sphere(n: int, radius: float = 1.0):
    """``n`` points spread evenly over a sphere of the given radius (the
    golden-angle spiral: equal-area bands in z, azimuth advanced by the
    golden angle)."""
    k = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * k + 1.0) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = k * (math.pi * (3.0 - math.sqrt(5.0)))
    return radius * np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)


def shielding(seed: int = 0, n_sh: int = 128, n_ext: int = 256, n_in: int = 1024,
              n_out: int = 1024, r_sh: float = 2.0, r_ext: float = 5.0, r_in: float = 1.5,
              r_out: float = 2.5):
    """Geometry of the active-shielding example (Sec. III.B): shield charge
    positions (regular on radius r_sh), external charges (uniformly random
    positions on radius r_ext, charges U[-1,1)), inner and outer probe
    points (even on radii r_in and r_out).  Shield charges start at zero."""
    ext_pos, ext_q = sphere_surface(n_ext, seed, r_ext)
    return dict(shield=fibonacci_sphere(n_sh, r_sh), ext=ext_pos, q_ext=ext_q,
                inner=fibonacci_sphere(n_in, r_in), outer=fibonacci_sphere(n_out, r_out))


def uneven_problem_sizes(k: int = 16, seed: int = 100, lo: float = 1e4,
                         hi: float = 5e5):
    """``k`` problem sizes log-uniform in [lo, hi]; problem j is then drawn
    with ``uniform_cube(size_j, seed + 1 + j)``."""
    rng = np.random.default_rng(seed)
    return [int(round(math.exp(x))) for x in
            rng.uniform(math.log(lo), math.log(hi), k)]


def sample_targets(n: int, k: int, seed: int = 1):
    """``k`` distinct target indices out of ``n`` (sorted)."""
    rng = np.random.default_rng(seed)
    k = min(k, n)
    return np.sort(rng.choice(n, k, replace=False))


# Named workloads with their method parameters (s = splits per level,
# theta = separation parameter of the admissibility test).
WORKLOADS = {
    "cube4k_p6": dict(gen="uniform_cube", n=4096, p=6, leaf=64, s=2, theta=0.6),
    "cube1m_p8": dict(gen="uniform_cube", n=1 << 20, p=8, leaf=128, s=2, theta=0.6),
    "cluster1m_p10": dict(gen="clustered", n=1 << 20, p=10, leaf=128, s=2, theta=0.6),
    "cube256k_p8_r32": dict(gen="uniform_cube", n=1 << 18, p=8, leaf=128, s=2,
                            theta=0.6, nrhs=32),
    "plummer1m_p8": dict(gen="plummer", n=1 << 20, p=8, leaf=128, s=2, theta=0.6),
}


def generate(name: str, n: int | None = None, seed: int = 0):
    """Positions and charges of a named workload (optionally resized)."""
    w = WORKLOADS[name]
    n = w["n"] if n is None else n
    if w["gen"] == "uniform_cube":
        return uniform_cube(n, seed, w.get("nrhs", 0))
    if w["gen"] == "clustered":
        return clustered(n, seed)
    if w["gen"] == "plummer":
        return plummer(n, seed)
    raise KeyError(name)
