"""Pins of the oracle's CIC and TSC charge-assignment kernels (eq. density_apcloud
with Phi the tent or the quadratic B-spline instead of the node's own cell).

What fixes the values: the kernels' moments in closed form (the tent is the
convolution of two unit boxes, the B-spline of three, so their moments are those
of a sum of independent uniform variables) and by quadrature; the B-spline
identities on a uniform lattice (the weights of one particle sum to 1 and
reproduce linear functions; the B-spline's also its variance 1/4); and the
density rows, which must turn the nodal values of a polynomial into the
kernel-weighted average of that polynomial over Omega (divided by the kernel's
mass inside Omega) -- by Gauss-Legendre quadrature of the piecewise polynomial
kernel here, beside the walls too, where odd and mixed moments enter.
"""
import itertools
import math

import numpy as np
import pytest
from scipy.integrate import quad

from oracle import oracle as om
from workloads import beam_halo, uniform_lattice_points

# the kernels as piecewise polynomials in u (their definitions), pieces [a, b]
PIECES = {
    om.KERNEL_CIC: [(-1.0, 0.0, lambda u: 1.0 + u), (0.0, 1.0, lambda u: 1.0 - u)],
    om.KERNEL_TSC: [(-1.5, -0.5, lambda u: 0.5 * (1.5 + u) ** 2),
                    (-0.5, 0.5, lambda u: 0.75 - u * u),
                    (0.5, 1.5, lambda u: 0.5 * (1.5 - u) ** 2)],
}


def phi(kernel, u):
    for a, b, f in PIECES[kernel]:
        if a <= u <= b:
            return f(u)
    return 0.0


def uniform_moment(e, n):
    """E[S^e] for S the sum of n independent U(-1/2, 1/2) (e <= 4)."""
    m2, m4 = 1.0 / 12.0, 1.0 / 80.0
    if e % 2:
        return 0.0
    return {0: 1.0, 2: n * m2, 4: n * m4 + 3 * n * (n - 1) * m2 * m2}[e]


@pytest.mark.parametrize("kernel,nbox", [(om.KERNEL_CIC, 2), (om.KERNEL_TSC, 3)])
def test_moments_closed_form(kernel, nbox):
    for e in range(5):
        assert abs(om.kernel_moment(kernel, e) - uniform_moment(e, nbox)) <= 4e-16, e
    # NGP: the cell, one box
    for e in range(5):
        assert abs(om.kernel_moment(om.KERNEL_NGP, e) - uniform_moment(e, 1)) <= 4e-16


@pytest.mark.parametrize("kernel", [om.KERNEL_CIC, om.KERNEL_TSC])
def test_truncated_moments_against_quadrature(kernel):
    cuts = [(-np.inf, np.inf), (-0.5, np.inf), (-np.inf, 0.5), (-0.5, 0.5), (-1.5, 0.25),
            (0.3, 2.0), (-3.0, -0.7), (1.2, 1.4), (-0.5, 1.0)]
    for tlo, thi in cuts:
        for e in range(5):
            lo, hi = max(tlo, -1.5), min(thi, 1.5)
            want = 0.0
            if hi > lo:
                want = quad(lambda u: u ** e * phi(kernel, u), lo, hi,
                            points=[-1.5, -1.0, -0.5, 0.0, 0.5, 1.0, 1.5], epsabs=1e-15,
                            epsrel=1e-14, limit=200)[0]
            got = om.kernel_moment(kernel, e, tlo, thi)
            assert abs(got - want) <= 1e-14, (tlo, thi, e, got, want)
    # the kernel of a node at half a cell from a wall: CIC keeps 7/8 of its mass,
    # TSC 5/6
    m = om.kernel_moment(kernel, 0, -0.5, np.inf)
    assert abs(m - (7 / 8 if kernel == om.KERNEL_CIC else 5 / 6)) <= 1e-15


def lattice_with_particle(depth, p, kernel):
    """Uniform lattice cloud (one particle per cell centre) plus one particle at p;
    with max_depth = depth the cloud stays the lattice."""
    xyz = np.concatenate([uniform_lattice_points(depth), np.array(p, float).reshape(3, 1)], 1)
    C = om.OracleCloud(xyz, order=2, c=1e-3, max_depth=depth, kernel=kernel)
    q = np.zeros(C.N)
    q[-1] = 1.0
    return C, q


@pytest.mark.parametrize("kernel", [om.KERNEL_CIC, om.KERNEL_TSC])
def test_single_particle_weights_on_a_lattice(kernel):
    """One unit charge on the 8^3 lattice, at points at least the kernel's reach
    from the walls: h^3 rho_M over the nodes are the particle's weights; they sum
    to 1, reproduce linear functions (sum w (y - p) = 0) and, for the B-spline,
    have second moment h^2/4 per axis."""
    depth, h = 3, 1.0 / 8
    rng = np.random.default_rng(5)
    for _ in range(6):
        # two cells from the walls: every node with a weight has its whole
        # kernel inside Omega (a_0 = 1)
        p = 2 * h + (1 - 4 * h) * rng.random(3)
        C, q = lattice_with_particle(depth, p, kernel)
        r = C.deposit(q)[:C.n]
        w = r * h ** 3
        pos = C.positions()[:, :C.n]
        assert abs(w.sum() - 1.0) <= 1e-14
        for d in range(3):
            assert abs(np.dot(w, pos[d] - p[d])) <= 1e-15
        if kernel == om.KERNEL_TSC:
            for d in range(3):
                assert abs(np.dot(w, (pos[d] - p[d]) ** 2) - h * h / 4) <= 1e-15
        # support: every node with a weight is within the reach of the kernel
        s = 1.0 if kernel == om.KERNEL_CIC else 1.5
        near = np.all(np.abs(pos - np.array(p)[:, None]) < s * h, axis=0)
        assert np.all(w[~near] == 0.0) and np.all(w[near] >= 0.0)
    # a particle on a node: CIC gives that node everything, TSC the B-spline's
    # values at the integers, 3/4 and 1/8
    y = np.array([2.5, 3.5, 4.5]) * h
    C, q = lattice_with_particle(depth, y, kernel)
    w = C.deposit(q)[:C.n] * h ** 3
    pos = C.positions()[:, :C.n]
    off = np.rint((pos - y[:, None]) / h).astype(int)
    for j in np.flatnonzero(w):
        want = 1.0
        for d in range(3):
            a = abs(off[d, j])
            want *= (1.0 if a == 0 else 0.0) if kernel == om.KERNEL_CIC else (0.75 if a == 0 else 0.125)
        assert abs(w[j] - want) <= 1e-15, (j, w[j], want)
    assert np.count_nonzero(w) == (1 if kernel == om.KERNEL_CIC else 27)


@pytest.mark.parametrize("kernel", [om.KERNEL_CIC, om.KERNEL_TSC])
def test_deposit_wall_normalisation(kernel):
    """A unit charge on the centre of a node of the wall layer: that node's kernel
    keeps the mass a_0 (7/8 CIC, 5/6 TSC) inside Omega and rho_M is divided by it;
    the raw weights h^3 a_0 rho_M are the kernel's values at the lattice offsets
    that exist -- all of them for CIC (the node itself), for TSC all but the
    offset -1 across the wall (B-spline value 1/8), summing to 7/8."""
    depth, h = 3, 1.0 / 8
    p = np.array([0.5 * h, 3.5 * h, 4.5 * h])  # on the centre of a wall-layer node
    C, q = lattice_with_particle(depth, p, kernel)
    r = C.deposit(q)[:C.n]
    pos = C.positions()[:, :C.n]
    a0 = np.ones(C.n)
    for d in range(3):
        for j in range(C.n):
            tlo, thi = -pos[d, j] / h, (1.0 - pos[d, j]) / h
            a0[j] *= quad(lambda u: phi(kernel, u), max(tlo, -1.5), min(thi, 1.5),
                          points=[-1.0, -0.5, 0.0, 0.5, 1.0], epsabs=1e-15)[0]
    want = 1.0 if kernel == om.KERNEL_CIC else 7 / 8
    assert abs((r * h ** 3 * a0).sum() - want) <= 1e-14
    j0 = int(np.argmin(np.abs(pos - p[:, None]).sum(0)))
    assert abs(a0[j0] - (7 / 8 if kernel == om.KERNEL_CIC else 5 / 6)) <= 1e-14


# ---------------------------------------------------------------- density rows


def kernel_axis_integrals(kernel, y, h, lo, hi, amax=4, npts=6):
    """I[a] = (1/h) int_{[lo,hi]} x^a phi((x - y)/h) dx, a = 0..amax, by
    Gauss-Legendre on each polynomial piece of the kernel (exact)."""
    xg, wg = np.polynomial.legendre.leggauss(npts)
    out = np.zeros(amax + 1)
    for a, b, f in PIECES[kernel]:
        xa, xb = max(y + a * h, lo), min(y + b * h, hi)
        if xb <= xa:
            continue
        x = 0.5 * (xb - xa) * xg + 0.5 * (xb + xa)
        fw = np.array([f((xi - y) / h) for xi in x]) * wg * 0.5 * (xb - xa) / h
        for e in range(amax + 1):
            out[e] += np.dot(fw, x ** e)
    return out


def kernel_average(P, kernel, y, h):
    """(1/a_0) (1/h^3) int_Omega P(x) Phi((x - y)/h) dx over Omega = [0, 1]^3."""
    I = [kernel_axis_integrals(kernel, y[d], h, 0.0, 1.0) for d in range(3)]
    tot = sum(c * I[0][a[0]] * I[1][a[1]] * I[2][a[2]] for a, c in P.items())
    return tot / (I[0][0] * I[1][0] * I[2][0])


def rand_poly(rng, k):
    return {a: rng.standard_normal() for a in itertools.product(range(k + 1), repeat=3)
            if sum(a) <= k}


def poly_eval(P, x, y, z):
    return sum(c * x ** a[0] * y ** a[1] * z ** a[2] for a, c in P.items())


def apply_rows(C, bw, bd, f):
    nd = C.nodes()
    m = np.diff(nd["st_off"])
    rows = np.repeat(np.arange(C.n), m)
    return bd * f[:C.n] + np.bincount(rows, weights=bw * f[nd["st_idx"]], minlength=C.n)


def wall_layer(C):
    """Nodes whose kernel support (CIC or TSC) reaches past a wall: the cell's
    centre within 1.5 cell edges of a face."""
    nd = C.nodes()
    pos = C.positions()[:, :C.n]
    h = C.L / 2.0 ** nd["level"]
    return np.any((pos < 1.5 * h) | (pos > 1.0 - 1.5 * h), axis=0)


@pytest.mark.parametrize("kernel", [om.KERNEL_CIC, om.KERNEL_TSC])
@pytest.mark.parametrize("order", [2, 4])
def test_density_rows_give_kernel_averages(kernel, order):
    """eq. density_apcloud with a CIC or TSC kernel: a row of order k applied to
    the nodal values of a polynomial of degree <= k gives that polynomial's
    kernel-weighted average over Omega divided by a_0 -- also at the nodes beside
    the walls, whose rows carry first-derivative and mixed terms.  Identity rows
    (order 0) give it for constants."""
    rng = np.random.default_rng(40 + 3 * kernel + order)
    if order == 2:
        C = om.OracleCloud(beam_halo(20000, seed=9), order=2, c=0.35, max_depth=6, kernel=kernel)
    else:
        C = om.OracleCloud(beam_halo(20000, seed=31), order=4, c=0.05, max_depth=5, kernel=kernel)
    nd = C.nodes()
    pos = C.positions()
    bw, bd = C.density_rows()
    dord = C.density_orders()
    wall = wall_layer(C)
    absum = np.add.reduceat(np.abs(bw), nd["st_off"][:-1])
    assert np.all(absum <= 0.5 * bd * (1 + 1e-14))
    checked_wall = 0
    for deg in sorted(set(np.unique(dord).tolist()), reverse=True):
        rows = np.flatnonzero(dord == deg)
        P = rand_poly(rng, deg)
        f = poly_eval(P, *pos)
        got = apply_rows(C, bw, bd, f)
        pick = np.concatenate([rows[wall[rows]][:60],
                               rng.choice(rows, size=min(rows.size, 60), replace=False)])
        for i in pick:
            h = C.L / 2.0 ** int(nd["level"][i])
            want = kernel_average(P, kernel, pos[:, i], h)
            assert abs(got[i] - want) <= 1e-10 * max(1.0, np.abs(f).max()), (deg, i)
            checked_wall += int(wall[i] and deg > 0)
    # the walls' odd moments were exercised by rows that kept a derivative order
    assert checked_wall >= 10, checked_wall


@pytest.mark.parametrize("kernel", [om.KERNEL_CIC, om.KERNEL_TSC])
def test_kernel_density_solve(kernel):
    """The density system with a CIC or TSC kernel is well posed (every row within
    the stability bound): the solve converges in a handful of iterations, and a
    wider kernel widens the perturbation of the identity (fewer rows keep order 2
    than with NGP)."""
    xyz = beam_halo(20000, seed=9)
    C = om.OracleCloud(xyz, order=2, c=0.35, max_depth=6, kernel=kernel)
    C0 = om.OracleCloud(xyz, order=2, c=0.35, max_depth=6)
    rt, st = C.density_solve(C.deposit(), tol=1e-12)
    assert st["status"] == 0 and st["iters"] <= 15, st
    assert (C.density_orders() == 2).sum() <= (C0.density_orders() == 2).sum()
    # same cloud, other deposit: the NGP one counts the cell's own particles only
    assert C.n == C0.n and not np.allclose(C.deposit(), C0.deposit())


def test_ngp_kernel_is_the_cell_deposit():
    xyz = beam_halo(5000, seed=2)
    C = om.OracleCloud(xyz, order=2, c=0.35, max_depth=5, kernel=om.KERNEL_NGP)
    nd = C.nodes()
    h = C.L / 2.0 ** nd["level"]
    np.testing.assert_array_equal(C.deposit()[:C.n], nd["count"] * (1.0 / C.N) / h ** 3)
