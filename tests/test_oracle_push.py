"""Pins of the oracle's leapfrog particle push (the time step of the Vlasov-Poisson
loop, Sec. 1) against closed forms and an independent exact reflection.

* constant force: kick-drift leapfrog with a half kick first reproduces the
  parabola x0 + v0 t + a t^2 / 2 exactly (dyadic data, no rounding anywhere);
* harmonic force grad = -w^2 x: the leapfrog recurrence
  x_{n+1} - 2 x_n + x_{n-1} = -(w dt)^2 x_n has the closed form
  x_n = x0 cos(n th) + (dt v0 / sin th) sin(n th), cos th = 1 - (w dt)^2 / 2,
  which fails if the drift came before the kick or the kick were not staggered;
* walls: the fold u -> r or 1 - r of the oracle against repeated mirror images in
  exact rational arithmetic (a different algorithm), with one velocity sign
  change per crossing.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle


def test_constant_force_parabola_exact():
    a = np.array([0.25, -0.5, 0.125])[:, None]
    x0 = np.array([0.5, 0.75, 0.25])[:, None]
    v0 = np.array([0.125, -0.0625, 0.25])[:, None]
    dt = 1.0 / 64
    x, v = oracle.push(x0, v0, a, dt / 2, dt)  # half kick, then full steps
    for n in range(1, 33):
        t = n * dt
        np.testing.assert_array_equal(x, x0 + v0 * t + a * t * t / 2)
        np.testing.assert_array_equal(v, v0 + a * (t - dt / 2))
        x, v = oracle.push(x, v, a, dt, dt)


def test_harmonic_oscillator_closed_form():
    w, dt = 3.0, 0.01
    x0 = np.array([0.5, -0.3, 0.2])
    v0 = np.array([0.0, 0.4, -0.7])
    lo, L = (-2.0, -2.0, -2.0), 4.0
    h = w * dt
    th = np.arccos(1.0 - h * h / 2)
    x, v = oracle.push(x0[:, None], v0[:, None], -w * w * x0[:, None], dt / 2, dt, lo, L)
    for n in range(1, 400):
        ref = x0 * np.cos(n * th) + dt * v0 / np.sin(th) * np.sin(n * th)
        np.testing.assert_allclose(x[:, 0], ref, rtol=0, atol=1e-11)
        x, v = oracle.push(x, v, -w * w * x, dt, dt, lo, L)


def _mirror(xf, lo, hi):
    """Exact repeated mirror images of a rational position into [lo, hi]."""
    x, flips = Fraction(xf), 0
    lo, hi = Fraction(lo), Fraction(hi)
    while x < lo or x > hi:
        x = 2 * hi - x if x > hi else 2 * lo - x
        flips += 1
    return x, flips


@pytest.mark.parametrize("lo,L", [(0.0, 1.0), (-0.75, 2.5), (3.0, 0.3)])
def test_walls_against_exact_mirrors(lo, L):
    rng = np.random.default_rng(11)
    n = 400
    x0 = lo + L * rng.random((3, n))
    # displacements from inside a step to several lengths away, both signs
    v0 = L * rng.uniform(-7.5, 7.5, (3, n))
    v0[:, :40] = L * rng.uniform(-0.2, 0.2, (3, 40))  # mostly no wall
    dt = 1.0
    x, v = oracle.push(x0, v0, np.zeros_like(x0), 0.0, dt, (lo,) * 3, L)
    hi = lo + L
    for d in range(3):
        for i in range(n):
            pre = x0[d, i] + dt * v0[d, i]  # IEEE double, as the oracle's drift
            ex, flips = _mirror(pre, lo, lo + L)
            assert lo <= x[d, i] <= hi
            assert abs(Fraction(x[d, i]) - ex) <= Fraction(8 * np.spacing(L * (1 + abs(pre - lo) / L)))
            assert v[d, i] == (v0[d, i] if flips % 2 == 0 else -v0[d, i])
            if lo <= pre <= hi:
                assert x[d, i] == pre and flips == 0


def test_wall_hits_and_edge_values():
    # ends exactly on a wall after one or two crossings; exactly on a wall without one
    lo, L = 0.0, 1.0
    x0 = np.array([[0.5, 0.5, 0.5, 0.5, 0.25]] * 3)
    v0 = np.array([[1.5, -0.5, 0.5, 2.5, -2.25]] * 3)
    x, v = oracle.push(x0, v0, np.zeros_like(x0), 0.0, 1.0, (lo,) * 3, L)
    np.testing.assert_array_equal(x[0], [0.0, 0.0, 1.0, 1.0, 0.0])
    np.testing.assert_array_equal(v[0], [1.5, -0.5, 0.5, -2.5, -2.25])


def test_invalid_arguments():
    x = np.zeros((3, 2))
    with pytest.raises(RuntimeError):
        oracle.push(x, x, x, np.nan, 1.0)
    with pytest.raises(RuntimeError):
        oracle.push(x, x, x, 1.0, np.inf)
    with pytest.raises(RuntimeError):
        oracle.push(x, x, x, 1.0, 1.0, L=0.0)


@pytest.mark.parametrize("lo,L", [(0.0, 1.0), (-0.75, 2.5)])
def test_periodic_wrap_against_exact_residue(lo, L):
    # on a periodic domain a free particle moves on the torus: its position is
    # lo + ((x + dt v - lo) mod L), exactly, and its velocity never changes
    rng = np.random.default_rng(12)
    n = 300
    x0 = lo + L * rng.random((3, n))
    v0 = L * rng.uniform(-7.5, 7.5, (3, n))
    v0[:, :30] = L * rng.uniform(-0.2, 0.2, (3, 30))
    x, v = oracle.push(x0, v0, np.zeros_like(x0), 0.0, 1.0, (lo,) * 3, L, periodic=1)
    np.testing.assert_array_equal(v, v0)
    for d in range(3):
        for i in range(n):
            pre = x0[d, i] + v0[d, i]
            ex = Fraction(lo) + (Fraction(pre) - Fraction(lo)) % Fraction(L)
            assert lo <= x[d, i] <= lo + L
            assert abs(Fraction(x[d, i]) - ex) <= Fraction(8 * np.spacing(L * (1 + abs(pre - lo) / L)))
            if lo <= pre <= lo + L:
                assert x[d, i] == pre


def test_periodic_wrap_edge_values():
    # one and two lengths across a face; leaving by lo re-enters near lo + L
    x0 = np.array([[0.5, 0.5, 0.5, 0.25]] * 3)
    v0 = np.array([[1.25, -0.75, 2.0, -2.5]] * 3)
    x, v = oracle.push(x0, v0, np.zeros_like(x0), 0.0, 1.0, periodic=1)
    np.testing.assert_array_equal(x[0], [0.75, 0.75, 0.5, 0.75])
    np.testing.assert_array_equal(v, v0)
