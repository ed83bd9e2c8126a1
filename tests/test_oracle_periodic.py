"""Periodic domains in the oracle (CPU).

On a periodic domain (every axis) face neighbours wrap around, there are no
boundary nodes, stencil offsets are minimum images and the Poisson problem is
Delta phi = c (rho~ - mean) with phi of mean 0.  Pins: the structure of a uniform
lattice (every node the full 2-ring, the seam nodes too), invariance of the whole
construction under the shift by half the domain (a symmetry of the periodic
domain that moves every cell onto another cell), the second-order convergence of
the GFD solve on a periodic manufactured solution, and the order-4 lattice
stencils at the seam.
"""
import numpy as np
import pytest

from oracle.oracle import OracleCloud
from workloads import beam_halo, uniform_lattice_points




def lattice(depth, order=2):
    return OracleCloud(uniform_lattice_points(depth), order=order, c=1e-3, max_depth=depth,
                       periodic=1)


def test_periodic_lattice_structure():
    """8^3 lattice: 512 nodes, no boundary node, 6 face neighbours each, and every
    stencil the uniform 2-ring of 24 nodes at minimum-image offsets -- also at the
    seam, where the ring wraps."""
    O = lattice(3)
    assert (O.n, O.nb) == (512, 0)
    off, idx = O.ring1()
    assert np.all(np.diff(off) == 6)
    nd = O.nodes()
    crd = O.coords().astype(np.int64)
    S = 2 ** (3 + 1)
    assert np.all(np.diff(nd["st_off"]) == 24)
    rows = np.repeat(np.arange(O.n), 24)
    d = crd[:, nd["st_idx"]] - crd[:, rows]
    d = (d + S // 2) % S - S // 2
    sp = 2  # one cell at level 3 in units of 2^-(D+1)
    q = np.abs(d) // sp
    assert np.all(np.abs(d) % sp == 0)
    assert np.all(q.sum(axis=0) <= 2) and np.all((q ** 2).sum(axis=0) >= 1)
    # each row: 6 + 12 + 6 neighbours at r^2 = 1, 2, 4 cells, all distinct
    r2 = (q ** 2).sum(axis=0).reshape(O.n, 24)
    assert np.all(np.sort(r2, axis=1) == np.array([1] * 6 + [2] * 12 + [4] * 6))


def _shifted_pair(order=2):
    xyz = beam_halo(6000, seed=41)
    kw = dict(order=order, c=0.3 if order == 2 else 0.06, max_depth=5, periodic=1)
    A = OracleCloud(xyz, **kw)
    xs = xyz.copy()
    xs[0] = (xs[0] + 0.5) % 1.0
    B = OracleCloud(xs, **kw)
    return A, B


@pytest.mark.parametrize("order", [2, 4])
def test_periodic_half_shift_invariance(order):
    """Shifting every particle by L/2 along x maps the periodic domain onto itself
    and every cell onto a cell: the shifted cloud has the same nodes moved by L/2,
    with the same levels and the same face adjacency (wrap-around included).  Ties
    in (r^2, index) are broken by node index, which the shift reorders, so a
    stencil may pick another of two equally near candidates; every node whose
    stencil maps onto the shifted node's stencil has the same weights (minimum-
    image offsets), and that is most of them."""
    A, B = _shifted_pair(order)
    assert (A.n, A.nb) == (B.n, B.nb) and A.nb == 0
    S = 2 ** (A.max_depth + 1)
    ca, cb = A.coords().astype(np.int64), B.coords().astype(np.int64)
    moved = ca.copy()
    moved[0] = (moved[0] + S // 2) % S
    key = lambda c: (c[0] * S + c[1]) * S + c[2]
    kb = {int(k): j for j, k in enumerate(key(cb))}
    perm = np.array([kb[int(k)] for k in key(moved)])  # node j of A is node perm[j] of B
    na, nb_ = A.nodes(), B.nodes()
    assert np.array_equal(na["level"], nb_["level"][perm])
    oa, ia = A.ring1()
    ob, ib = B.ring1()
    for j in range(A.n):
        assert {int(perm[v]) for v in ia[oa[j]:oa[j + 1]]} == set(ib[ob[perm[j]]:ob[perm[j] + 1]].tolist())
    wa, da = A.assemble()
    wb, db = B.assemble()
    same = 0
    for j in range(A.n):
        a0, a1 = na["st_off"][j], na["st_off"][j + 1]
        b0, b1 = nb_["st_off"][perm[j]], nb_["st_off"][perm[j] + 1]
        sa = {int(perm[v]): w for v, w in zip(na["st_idx"][a0:a1], wa[a0:a1])}
        sb = {int(v): w for v, w in zip(nb_["st_idx"][b0:b1], wb[b0:b1])}
        if sa.keys() != sb.keys():
            continue
        same += 1
        assert abs(db[perm[j]] - da[j]) <= 1e-12 * abs(da[j]), j
        for v in sa:
            assert abs(sa[v] - sb[v]) <= 1e-12 * abs(da[j]), (j, v)
    assert same >= 0.8 * A.n, (same, A.n)


def test_periodic_manufactured_second_order():
    """phi = sin(2 pi x) sin(2 pi y) sin(2 pi z) (mean 0), rho = Delta phi on the
    periodic 8^3, 16^3, 32^3 lattices: the GFD solution's largest error falls by
    about 4 per refinement (second order)."""
    errs = []
    for depth in (3, 4, 5):
        O = lattice(depth)
        x, y, z = O.positions()[:, :O.n]
        phi = np.sin(2 * np.pi * x) * np.sin(2 * np.pi * y) * np.sin(2 * np.pi * z)
        rho = -12 * np.pi ** 2 * phi
        got, st = O.poisson_solve(rho, tol=1e-13, maxit=20000, precond=1)
        assert st["status"] == 0
        errs.append(np.abs(got[:O.n] - phi).max())
    ratios = [errs[k] / errs[k + 1] for k in range(2)]
    assert all(3.5 <= r <= 4.6 for r in ratios), (errs, ratios)


def test_periodic_solution_mean_zero_and_lu():
    """The iterative and the direct solve agree and both have volume-weighted mean 0
    (adaptive cloud: cells of several levels)."""
    xyz = beam_halo(3000, seed=43)
    O = OracleCloud(xyz, order=2, c=0.3, max_depth=4, periodic=1)
    rho_t, _ = O.density_solve(O.deposit(), tol=1e-13)
    phi, st = O.poisson_solve(rho_t[:O.n], tol=1e-13, maxit=20000, precond=1)
    phi_lu = O.poisson_lu(rho_t[:O.n])
    h = O.L / 2.0 ** O.nodes()["level"]
    assert abs(np.sum(phi[:O.n] * h ** 3)) <= 1e-12 * np.abs(phi).max()
    assert np.abs(phi - phi_lu).max() <= 1e-9 * np.abs(phi_lu).max()


def test_periodic_order4_lattice_seam():
    """Fourth order on the periodic 8^3 lattice: every node (seam included) has the
    56-node stencil at minimum-image offsets r^2 = 1..5 cells."""
    O = lattice(3, order=4)
    nd = O.nodes()
    assert O.nb == 0 and np.all(np.diff(nd["st_off"]) == 56)
    crd = O.coords().astype(np.int64)
    S = 16
    rows = np.repeat(np.arange(O.n), 56)
    d = crd[:, nd["st_idx"]] - crd[:, rows]
    d = (d + S // 2) % S - S // 2
    r2 = ((d // 2) ** 2).sum(axis=0).reshape(O.n, 56)
    assert np.all(r2 == np.repeat(np.arange(1, 6), [6, 12, 8, 6, 24])[None, :])


def test_periodic_rejects_shallow_depth():
    with pytest.raises(Exception):
        OracleCloud(uniform_lattice_points(1), order=2, c=1e-3, max_depth=1, periodic=1)
