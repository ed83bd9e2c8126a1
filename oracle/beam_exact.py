"""Benchmark solution of the 3-D Gaussian beam with halo (Sec. 5.2) -- test
infrastructure only.

Only the test suite may import this module; it shares no code with the HIP
library.

The paper embeds the spherically symmetric problem Delta phi = rho in the ball of
radius 2 with phi = 0 on its sphere, solves it in 1-D, and uses that solution both
as the Dirichlet data on the faces of Omega = [-1, 1]^3 and as the reference the
errors are measured against.  The density (eq. GaussianDist, with 2 tau^2 in the
exponents, the reading under which the printed normalisation constants come out)
is a sum of two Gaussians, so the 1-D solution has a closed form: a Gaussian
charge of total Q and width tau has the free-space potential
    -Q erf(r / (sqrt(2) tau)) / (4 pi r)
(Delta of -1 / (4 pi r) is the unit point charge), and phi = 0 at r = 2 only
shifts it by a constant.  The radial derivative is the enclosed charge over
4 pi r^2:
    phi'(r) = a tau^3 [sqrt(pi/2) erf(r / (sqrt(2) tau)) - (r / tau) exp(-r^2 / (2 tau^2))] / r^2
per component a exp(-r^2 / (2 tau^2)).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf

TAU1, TAU2, A2, R_OUT = 0.02, 0.3, 1e-5, 2.0


def _cube_mass(t: float) -> float:
    """Integral of exp(-|x|^2 / (2 t^2)) over [-1, 1]^3."""
    return (math.sqrt(2 * math.pi) * t * math.erf(1 / (math.sqrt(2) * t))) ** 3


def a1() -> float:
    """The normalisation a1: the charge of rho in Omega is 1."""
    return 1.0 / (_cube_mass(TAU1) + A2 * _cube_mass(TAU2))


def _components():
    a = a1()
    return [(a, TAU1), (a * A2, TAU2)]


def density(r):
    r = np.asarray(r, dtype=np.float64)
    return sum(a * np.exp(-r * r / (2 * t * t)) for a, t in _components())


def _free(a, t, r):
    """Free-space potential of the component a exp(-r^2 / (2 t^2)); r = 0 takes the limit."""
    Q = a * (2 * math.pi * t * t) ** 1.5
    r = np.asarray(r, dtype=np.float64)
    safe = np.where(r > 0, r, 1.0)
    ratio = np.where(r > 0, erf(safe / (math.sqrt(2) * t)) / safe, math.sqrt(2 / math.pi) / t)
    return -Q * ratio / (4 * math.pi)


def potential_r(r):
    """phi(r) of the ball problem, r >= 0."""
    return sum(_free(a, t, r) - _free(a, t, R_OUT) for a, t in _components())


def dpotential_r(r):
    """phi'(r), r > 0."""
    r = np.asarray(r, dtype=np.float64)
    out = np.zeros_like(r)
    for a, t in _components():
        out = out + a * t ** 3 * (math.sqrt(math.pi / 2) * erf(r / (math.sqrt(2) * t))
                                  - (r / t) * np.exp(-r * r / (2 * t * t))) / (r * r)
    return out


def potential(xyz):
    """phi at points xyz (3 x M)."""
    return potential_r(np.sqrt((np.asarray(xyz, dtype=np.float64) ** 2).sum(axis=0)))


def gradient(xyz):
    """grad phi at points xyz (3 x M), zero at the centre."""
    x = np.asarray(xyz, dtype=np.float64)
    r = np.sqrt((x ** 2).sum(axis=0))
    safe = np.where(r > 0, r, 1.0)
    return np.where(r > 0, dpotential_r(safe) / safe, 0.0) * x
