"""Pins of the benchmark solution of the 3-D Gaussian beam with halo (Sec. 5.2),
oracle/beam_exact.py, against the values the paper prints and against the 1-D
radial problem solved by quadrature (the paper's own route to its benchmark).

* a1 and the largest |phi| and |phi_x| agree with the printed values
  (tests/golden/beam3d_sec5_2.txt); they also fix the reading of eq. GaussianDist
  (2 tau^2 in the exponents) and of the radius-2 ball with phi = 0 on its sphere;
* phi' equals the enclosed charge over r^2 and phi equals minus the integral of
  phi' out to r = 2, both by adaptive quadrature of the density;
* finite differences of the 3-D fields: Delta phi = rho and grad phi.
"""
import os

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import beam_exact as B

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "beam3d_sec5_2.txt")


def golden():
    vals, rows = {}, []
    for line in open(GOLDEN):
        f = line.split()
        if not f or f[0].startswith("#"):
            continue
        if f[0] == "row":
            rows.append(tuple(float(x) for x in f[1:]))
        else:
            vals[f[0]] = float(f[1])
    return vals, rows


def test_printed_normalisation_and_norms():
    vals, rows = golden()
    # the paper prints a1 to four digits (7677); the normalisation gives 7678.2
    assert abs(B.a1() - vals["a1"]) / vals["a1"] < 3e-4
    r = np.concatenate([[0.0], np.geomspace(1e-5, np.sqrt(3.0), 200_000)])
    assert round(float(np.abs(B.potential_r(r)).max()), 3) == vals["phi_inf"]
    # the printed maximum is over particles, so at most the field's maximum
    gmax = float(np.abs(B.dpotential_r(r[1:])).max())
    assert vals["phi_x_inf"] <= gmax <= 1.001 * vals["phi_x_inf"]
    assert len(rows) == 4


@pytest.mark.parametrize("r", [1e-3, 0.01, 0.02, 0.05, 0.3, 0.9, 1.5])
def test_radial_solution_by_quadrature(r):
    enclosed = lambda s: quad(lambda u: B.density(u) * u * u, 0.0, s, points=[0.02, 0.06],
                              epsabs=0, epsrel=1e-13, limit=400)[0]
    dphi = lambda s: enclosed(s) / (s * s)
    assert float(B.dpotential_r(np.array(r))) == pytest.approx(dphi(r), rel=1e-9)
    phi = -quad(dphi, r, B.R_OUT, points=[0.02, 0.06, 0.3] if r < 0.02 else None,
                epsabs=0, epsrel=1e-11, limit=400)[0]
    assert float(B.potential_r(np.array(r))) == pytest.approx(phi, rel=1e-8)


def test_fields_by_finite_differences():
    rng = np.random.default_rng(4)
    d = rng.standard_normal((3, 40))
    x = d / np.linalg.norm(d, axis=0) * rng.uniform(0.03, 0.9, 40)
    h = 1e-4  # the core's width is 0.02: truncation error (h / 0.02)^2 / 12
    lap = -6 * B.potential(x)
    grad = np.zeros_like(x)
    for k in range(3):
        e = np.zeros((3, 1))
        e[k] = h
        lap = lap + B.potential(x + e) + B.potential(x - e)
        grad[k] = (B.potential(x + e) - B.potential(x - e)) / (2 * h)
    lap /= h * h
    rho = B.density(np.linalg.norm(x, axis=0))
    np.testing.assert_allclose(lap, rho, rtol=2e-3, atol=1e-6)
    np.testing.assert_allclose(grad, B.gradient(x), rtol=1e-5, atol=1e-9)
