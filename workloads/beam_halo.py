"""Beam-with-halo particle clouds (numpy PCG64), the synthetic stand-in for the
paper's Gaussian-beam-with-halo workloads (Sec. 5.1, eq. GaussianDist; Sec. 5.2).

Recipe (all in the unit cube [0,1)^3, structure-of-arrays float64, shape (3, N)):
  * core: round(N*(1-halo_frac)) points ~ N(centre, diag(sigma^2)), each point
    re-drawn until it lies inside [0,1)^3;
  * halo: the remaining points with radius r, r^3 ~ U[r_in^3, r_out^3], about the
    centre, in an isotropic direction (normalised Gaussian triple).
Draw order: the core block first, then the halo block, from one Generator.
"""
from __future__ import annotations

import numpy as np

CENTRE = (0.5, 0.5, 0.5)

# Named workloads: particle count, seed, core sigma, halo fraction, octree depth,
# GFD order and the error-balance constant used with them.
CONFIGS = {
    "beam_halo_1e5": dict(N=100_000, seed=1, sigma=(0.08, 0.08, 0.08), halo_frac=0.05,
                          max_depth=6, order=2, c=0.35),
    "beam_halo_1e7": dict(N=10_000_000, seed=2, sigma=(0.08, 0.08, 0.08), halo_frac=0.05,
                          max_depth=10, order=2, c=0.04),
    "beam_halo_1e8_k4": dict(N=100_000_000, seed=5, sigma=(0.05, 0.05, 0.2), halo_frac=0.03,
                             max_depth=12, order=4, c=0.007),
    # the anisotropic recipe at 3e4 particles (about 3.4e4 nodes): the clouds the
    # fourth-order learned preconditioner is trained and evaluated on
    "beam_halo_k4_3e4": dict(N=30_000, seed=6, sigma=(0.05, 0.05, 0.2), halo_frac=0.03,
                             max_depth=6, order=4, c=0.004),
}


# many clouds of uneven size: batch_specs(master_seed, count) gives each cloud's
# N, sigma and halo fraction; all share the tree and fit parameters below
BATCH = dict(master_seed=3, count=64, max_depth=8, order=2, c=0.35)


def _core(rng: np.random.Generator, n: int, sigma) -> np.ndarray:
    sig = np.asarray(sigma, dtype=np.float64).reshape(3, 1)
    cen = np.asarray(CENTRE, dtype=np.float64).reshape(3, 1)
    out = np.empty((3, n), dtype=np.float64)
    todo = np.arange(n)
    while todo.size:
        pts = cen + sig * rng.standard_normal((3, todo.size))
        ok = np.all((pts >= 0.0) & (pts < 1.0), axis=0)
        out[:, todo[ok]] = pts[:, ok]
        todo = todo[~ok]
    return out


def _halo(rng: np.random.Generator, n: int, r_in: float, r_out: float) -> np.ndarray:
    cen = np.asarray(CENTRE, dtype=np.float64).reshape(3, 1)
    u = rng.random(n)
    r = np.cbrt(r_in ** 3 + u * (r_out ** 3 - r_in ** 3))
    d = rng.standard_normal((3, n))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    return cen + r * d


def beam_halo(N: int, seed: int, sigma=(0.08, 0.08, 0.08), halo_frac: float = 0.05,
              shell=(0.25, 0.4)) -> np.ndarray:
    """Return a (3, N) float64 SoA array of particle positions in [0,1)^3."""
    rng = np.random.default_rng(seed)
    n_core = int(round(N * (1.0 - halo_frac)))
    n_halo = N - n_core
    core = _core(rng, n_core, sigma)
    halo = _halo(rng, n_halo, shell[0], shell[1])
    xyz = np.ascontiguousarray(np.concatenate([core, halo], axis=1))
    return xyz


def batch_specs(master_seed: int = 3, count: int = 64):
    """Per-cloud parameters of the many-cloud workload: N log-uniform in [1e4, 1e6],
    core sigma in [0.05, 0.15], halo fraction in [0.01, 0.1]; cloud i's positions
    use seed 3000 + i."""
    rng = np.random.default_rng(master_seed)
    specs = []
    for i in range(count):
        n = int(round(10.0 ** rng.uniform(4.0, 6.0)))
        s = float(rng.uniform(0.05, 0.15))
        hf = float(rng.uniform(0.01, 0.1))
        specs.append(dict(N=n, seed=3000 + i, sigma=(s, s, s), halo_frac=hf))
    return specs


def uniform_lattice_points(depth: int) -> np.ndarray:
    """One point at the centre of every cell of the uniform 2^depth grid on [0,1)^3,
    shape (3, 8**depth).  Used to force a uniform octree."""
    m = 1 << depth
    g = (np.arange(m, dtype=np.float64) + 0.5) / m
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    return np.ascontiguousarray(np.stack([x.ravel(), y.ravel(), z.ravel()]))


def gaussian_blob(M: int, seed: int, sigma: float = 0.03, centre=(0.40, 0.5, 0.5),
                  velocity=(1.0, 0.0, 0.0), v_spread: float = 0.05):
    """The test particle of the single-particle self-force test (Sec. 5): a sharp
    Gaussian cloud of M points, N(centre, sigma^2 I) re-drawn until inside
    [0,1)^3, moving with a common velocity plus N(0, v_spread^2) per component.
    Returns (xyz, vel), each (3, M) float64.  Draw order: positions, velocities."""
    rng = np.random.default_rng(seed)
    c = np.asarray(centre, dtype=np.float64)[:, None]
    xyz = c + sigma * rng.standard_normal((3, M))
    bad = np.any((xyz < 0.0) | (xyz >= 1.0), axis=0)
    while bad.any():
        xyz[:, bad] = c + sigma * rng.standard_normal((3, int(bad.sum())))
        bad = np.any((xyz < 0.0) | (xyz >= 1.0), axis=0)
    vel = np.asarray(velocity, dtype=np.float64)[:, None] + v_spread * rng.standard_normal((3, M))
    return np.ascontiguousarray(xyz), np.ascontiguousarray(vel)


# The 3-D Gaussian beam with halo of Sec. 5.2 (eq. GaussianDist, read with 2 tau^2 in
# the exponents): rho = a1 [exp(-|x|^2 / (2 tau1^2)) + a2 exp(-|x|^2 / (2 tau2^2))] on
# Omega = [-1, 1]^3, a1 normalising the charge in Omega to 1.
BEAM3D = dict(tau1=0.02, tau2=0.3, a2=1e-5, lo=(-1.0, -1.0, -1.0), L=2.0)


def paper_beam_3d(N: int, seed: int):
    """N particles of the 3-D beam with halo, (3, N) float64: each particle is drawn
    from the halo with the halo's share of the charge in Omega (binomial count),
    else from the core, each an isotropic Gaussian truncated to Omega by
    re-drawing.  Draw order: the halo count, the core block, the halo block."""
    import math
    t1, t2, a2 = BEAM3D["tau1"], BEAM3D["tau2"], BEAM3D["a2"]

    def mass(t):  # integral of exp(-|x|^2 / (2 t^2)) over [-1, 1]^3
        return (math.sqrt(2 * math.pi) * t * math.erf(1 / (math.sqrt(2) * t))) ** 3

    rng = np.random.default_rng(seed)
    p_halo = a2 * mass(t2) / (mass(t1) + a2 * mass(t2))
    nh = int(rng.binomial(N, p_halo))

    def truncated(n, t):
        out = np.empty((3, 0))
        while out.shape[1] < n:
            x = t * rng.standard_normal((3, 2 * (n - out.shape[1]) + 16))
            out = np.concatenate([out, x[:, np.all(np.abs(x) <= 1.0, axis=0)]], axis=1)
        return out[:, :n]

    return np.ascontiguousarray(np.concatenate([truncated(N - nh, t1), truncated(nh, t2)], axis=1))


# The 2-D beam with halo of Sec. 5.1 on Omega = [-1, 1]^2 (the paper prints tau1 = 0.02,
# a2 = 1e-5, tau2 = 0.3, a1 = 396.1), read with 2 tau^2 in the exponents:
# rho = a1 [exp(-|x|^2/(2 tau1^2)) + a2 exp(-|x|^2/(2 tau2^2))], under which a1 = 396.1
# normalises the charge in Omega to 1 (with tau^2 it would be 0.50).
BEAM2D = dict(tau1=0.02, tau2=0.3, a2=1e-5, a1=396.1)


def paper_beam_2d(N: int, seed: int):
    """N particles of the 2-D beam with halo, (2, N) float64: each from the halo with
    the halo's share of the charge in Omega (binomial count), else from the core,
    each an isotropic Gaussian of standard deviation tau truncated to Omega by
    re-drawing.  Draw order: the halo count, the core block, the halo block."""
    import math
    t1, t2, a2 = BEAM2D["tau1"], BEAM2D["tau2"], BEAM2D["a2"]

    def mass(t):  # integral of exp(-|x|^2 / (2 t^2)) over [-1, 1]^2
        return (math.sqrt(2 * math.pi) * t * math.erf(1 / (math.sqrt(2) * t))) ** 2

    rng = np.random.default_rng(seed)
    p_halo = a2 * mass(t2) / (mass(t1) + a2 * mass(t2))
    nh = int(rng.binomial(N, p_halo))

    def truncated(n, t):
        out = np.empty((2, 0))
        while out.shape[1] < n:
            x = t * rng.standard_normal((2, 2 * (n - out.shape[1]) + 16))
            out = np.concatenate([out, x[:, np.all(np.abs(x) <= 1.0, axis=0)]], axis=1)
        return out[:, :n]

    return np.ascontiguousarray(np.concatenate([truncated(N - nh, t1), truncated(nh, t2)], axis=1))

