"""Pin of the oracle's Poisson solve against the closed-form potential of a
uniformly charged sphere (radius R, density rho_0 = 1, centre c, Delta phi = rho):
phi = r^2 / 6 - R^2 / 2 inside, -R^3 / (3 r) outside -- continuous with its first
derivative at r = R, and Delta phi = 1 inside, 0 outside.  The Dirichlet data g are
the closed form at the boundary nodes; the right-hand side is the density averaged
over each node's cell (8^3 midpoint samples, the density being discontinuous).
The GFD solution converges to the closed form at about second order on uniform
lattices (a discontinuous density allows between first and second)."""
import numpy as np
import pytest

from oracle import oracle as om
from workloads import uniform_lattice_points

R = 0.3
C0 = np.array([0.5, 0.5, 0.5])


def phi_exact(p):
    r = np.linalg.norm(p - C0[:, None], axis=0)
    return np.where(r < R, r * r / 6 - R * R / 2, -R ** 3 / (3 * np.maximum(r, 1e-300)))


def rho_cell_average(p, h, k=8):
    s = (np.arange(k) + 0.5) / k - 0.5
    acc = np.zeros(p.shape[1])
    for a in s:
        for b in s:
            for c in s:
                q = p + h * np.array([a, b, c])[:, None]
                acc += np.linalg.norm(q - C0[:, None], axis=0) < R
    return acc / k ** 3


def test_closed_form_is_the_sphere_potential():
    # Delta phi by central differences: 1 inside, 0 outside, away from r = R
    h = 1e-3
    for p, want in (([0.55, 0.47, 0.52], 1.0), ([0.9, 0.2, 0.5], 0.0), ([0.5, 0.5, 0.71], 1.0)):
        p = np.array(p)[:, None]
        lap = sum((phi_exact(p + h * e[:, None]) - 2 * phi_exact(p) + phi_exact(p - h * e[:, None]))
                  / h ** 2 for e in np.eye(3))
        assert abs(lap[0] - want) <= 1e-6
    # continuity of phi and of its radial derivative (R / 3 on both sides) at r = R
    at = lambda r: phi_exact(C0[:, None] + np.array([[r], [0.0], [0.0]]))[0]
    assert abs(at(R - 1e-12) - at(R + 1e-12)) <= 1e-11
    d = 1e-6
    assert abs((at(R) - at(R - d)) / d - R / 3) <= 1e-5
    assert abs((at(R + d) - at(R)) / d - R / 3) <= 1e-5


@pytest.mark.parametrize("order", [2, 4])
def test_uniform_sphere_convergence(order):
    errs = []
    for depth in (3, 4, 5):
        O = om.OracleCloud(uniform_lattice_points(depth), order=order, c=1e-3, max_depth=depth)
        pos = O.positions()
        rho = rho_cell_average(pos[:, :O.n], 1.0 / 2 ** depth)
        g = phi_exact(pos[:, O.n:])
        phi, st = O.poisson_solve(rho, g, tol=1e-13, maxit=20000, precond=1)
        assert st["status"] == 0
        np.testing.assert_array_equal(phi[O.n:], g)
        e = phi[:O.n] - phi_exact(pos[:, :O.n])
        errs.append(np.sqrt(np.mean(e * e)))
    ratios = [errs[k] / errs[k + 1] for k in range(2)]
    assert all(r >= 2.5 for r in ratios), (errs, ratios)
    assert errs[-1] <= 1e-4 * (1 if order == 2 else 0.5)
