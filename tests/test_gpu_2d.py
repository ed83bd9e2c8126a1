"""The two-dimensional variant (quadtree, k = 2) on the GPU against the FP64 oracle.

Bars as in three dimensions: quadtree, nodes, boundary nodes, stencils and integer
coordinates bit-exact; Laplacian and density rows within 1e-12 (both sides fit in
FP64, the GPU by the normal equations, the oracle by Householder QR), their orders
equal; deposit within 1e-13; Krylov solutions within kappa_2 (t_gpu + t_oracle);
derivatives and interpolation of the same phi within 1e-10.
"""
import math
import sys

import numpy as np
import pytest
from scipy.special import erf, exp1

from linalg_bounds import interior_matrix, kappa2, solve_bar
from workloads import BEAM2D, paper_beam_2d

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def note(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def apc():
    from paper_1603_04039_amd import apcloud
    apcloud.load_library()
    assert torch.cuda.is_available()
    return apcloud


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def lattice(m):
    g = (np.arange(m) + 0.5) / m
    X, Y = np.meshgrid(g, g, indexing="ij")
    return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel()]))


CASES = {
    "beam_c0.1": (lambda: paper_beam_2d(100000, seed=1), dict(lo=(-1.0, -1.0), L=2.0, c=0.1,
                                                              max_depth=12)),
    "beam_c0.02": (lambda: paper_beam_2d(200000, seed=2), dict(lo=(-1.0, -1.0), L=2.0, c=0.02,
                                                               max_depth=12)),
    "random_m12": (lambda: np.random.default_rng(5).random((2, 50000)),
                   dict(c=0.3, max_depth=9, m_cap=12)),
    "lattice": (lambda: lattice(32), dict(c=1e-3, max_depth=5)),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def pair(request, apc, oracle_mod):
    mk, kw = CASES[request.param]
    xy = mk()
    note(f"2-D {request.param}: {xy.shape[1]} particles")
    O = oracle_mod.OracleCloud2D(xy, order=2, **kw)
    G = apc.Cloud2D(cuda(xy), order=2, **kw)
    G.assemble()
    torch.cuda.synchronize()
    yield request.param, xy, O, G
    G.close()


def test_2d_structure_bit_exact(pair):
    name, xy, O, G = pair
    assert (G.n, G.nb, G.nnz, G.n_opened) == (O.n, O.nb, O.nnz, O.n_opened)
    a, b = O.nodes(), G.nodes()
    np.testing.assert_array_equal(a["perm"], b["perm"].astype(np.int64))
    for k in ("code", "level", "first", "count", "bowner", "bface", "st_off", "st_idx"):
        np.testing.assert_array_equal(a[k].astype(np.int64), b[k].astype(np.int64), err_msg=k)
    np.testing.assert_array_equal(O.coords(), b["ixy"])
    note(f"  {name}: n={G.n} nb={G.nb} nnz={G.nnz} opened={G.n_opened}")


def test_2d_rows(pair):
    name, xy, O, G = pair
    w_g, d_g, bw_g, bd_g, ord_g = G.operator()
    w_o, d_o = O.assemble()
    bw_o, bd_o, ord_o = O.density_rows()
    m = np.diff(O.nodes()["st_off"])
    ew = np.max(np.abs(w_g - w_o) / np.repeat(np.abs(d_o), m))
    ed = np.max(np.abs(d_g - d_o) / np.abs(d_o))
    np.testing.assert_array_equal(ord_g, ord_o)
    eb = max(np.abs(bw_g - bw_o).max(), np.abs(bd_g - bd_o).max())
    note(f"  {name}: rows {ew:.2e}, diag {ed:.2e}, density {eb:.2e}, identity rows "
         f"{int((ord_g == 0).sum())}")
    assert ew <= 1e-12 and ed <= 1e-12 and eb <= 1e-12


def test_2d_chain(pair):
    """deposit -> density solve -> Poisson solve -> derivatives and interpolation."""
    name, xy, O, G = pair
    nd = O.nodes()
    q = np.random.default_rng(3).uniform(0.5, 1.5, xy.shape[1])
    rm_o = O.deposit(q)
    rm_g = G.deposit(cuda(q)).cpu().numpy()
    assert np.max(np.abs(rm_g - rm_o) / np.maximum(np.abs(rm_o), 1e-300)) <= 1e-13
    rt_o, sto = O.density_solve(rm_o, tol=1e-13)
    rt, std = G.density_solve(cuda(rm_o), tol=1e-13)
    bw, bd, _ = O.density_rows()
    kB = kappa2(interior_matrix(nd["st_off"], nd["st_idx"], bw, bd, O.n), direct=False)
    e_rho = np.linalg.norm(rt.cpu().numpy() - rt_o) / np.linalg.norm(rt_o)
    assert std["status"] == 0 and e_rho <= solve_bar(kB, 1e-13, 1e-13, cap=1e-12)
    g = 0.01 * np.random.default_rng(4).standard_normal(O.nb)
    rhs = rt_o[:O.n].copy()
    phi_o, sto = O.poisson_solve(rhs, g, tol=1e-10, precond=1)
    phi, st = G.solve(cuda(rhs), cuda(g), tol=1e-10, precond=1)
    w, d = O.assemble()
    kL = kappa2(interior_matrix(nd["st_off"], nd["st_idx"], w, d, O.n))
    e_phi = np.linalg.norm(phi.cpu().numpy() - phi_o) / np.linalg.norm(phi_o)
    note(f"  {name}: density {e_rho:.2e} ({std['iters']} it), Poisson {e_phi:.2e} "
         f"(gpu {st['iters']} it, oracle {sto['iters']}, kappa_L {kL:.2e})")
    assert st["status"] == 0 and sto["status"] == 0
    assert e_phi <= solve_bar(kL, 1e-10, 1e-10, cap=1e-6)
    np.testing.assert_array_equal(phi.cpu().numpy()[O.n:], g)
    D_o = O.node_derivs(phi_o)
    D_g = G.node_derivs(cuda(phi_o)).cpu().numpy()
    assert np.max(np.abs(D_g - D_o) / (np.abs(D_o).max(axis=0) + 1e-300)) <= 1e-10
    pp_o, gp_o = O.interpolate(phi_o)
    pp, gp = G.interpolate_force(cuda(phi_o))
    assert np.abs(pp.cpu().numpy() - pp_o).max() <= 1e-12 * np.abs(pp_o).max()
    assert np.abs(gp.cpu().numpy() - gp_o).max() <= 1e-10 * np.abs(gp_o).max()


def beam_benchmark(r):
    t1, t2, a2, a1 = BEAM2D["tau1"], BEAM2D["tau2"], BEAM2D["a2"], BEAM2D["a1"]

    def F(s, t):
        return np.log(s) + 0.5 * exp1(s * s / (2 * t * t))

    r = np.maximum(r, 1e-300)
    return -(a1 * t1 * t1 * (F(2.0, t1) - F(r, t1)) + a1 * a2 * t2 * t2 * (F(2.0, t2) - F(r, t2)))


def test_2d_beam_against_benchmark(apc, oracle_mod):
    """The paper's 2-D beam with halo (Sec. 5.1), 1e6 particles: the GPU's field
    (deposit, density solve, Poisson solve with the benchmark on the boundary) and
    the oracle's agree within the solve bar, and their error against the radial
    benchmark is reported."""
    xy = paper_beam_2d(1000000, seed=7)
    kw = dict(lo=(-1.0, -1.0), L=2.0, c=0.03, max_depth=12)
    O = oracle_mod.OracleCloud2D(xy, order=2, **kw)
    G = apc.Cloud2D(cuda(xy), order=2, **kw)
    G.assemble()
    pos = O.positions()
    r = np.hypot(pos[0], pos[1])
    g = beam_benchmark(r[O.n:])
    rho_M = G.deposit()
    rt, _ = G.density_solve(rho_M, tol=1e-12)
    phi, st = G.solve(rt[:G.n].contiguous(), cuda(g), tol=1e-10)
    rt_o, _ = O.density_solve(O.deposit(), tol=1e-12)
    phi_o, _ = O.poisson_solve(rt_o[:O.n], g, tol=1e-10)
    ex = beam_benchmark(r[:O.n])
    pg = phi.cpu().numpy()[:O.n]
    e_g = np.sqrt(np.mean((pg - ex) ** 2)) / np.abs(ex).max()
    e_o = np.sqrt(np.mean((phi_o[:O.n] - ex) ** 2)) / np.abs(ex).max()
    d = np.linalg.norm(pg - phi_o[:O.n]) / np.linalg.norm(phi_o[:O.n])
    note(f"  2-D beam 1e6 particles, c = 0.03: n = {G.n}, iters {st['iters']}, error vs "
         f"benchmark {e_g:.3e} (oracle {e_o:.3e}), GPU vs oracle {d:.2e}")
    assert st["status"] == 0 and d <= 1e-6 and abs(e_g - e_o) <= 1e-3 * e_o
    G.close()


def test_2d_rejections(apc):
    x = cuda(np.random.default_rng(1).random((2, 100)))
    with pytest.raises(apc.ApcError) as e:
        apc.Cloud2D(x, order=4, max_depth=5)
    assert e.value.code == apc.APC_EINVAL
    bad = np.random.default_rng(1).random((2, 100))
    bad[0, 3] = 1.5
    with pytest.raises(apc.ApcError) as e:
        apc.Cloud2D(cuda(bad), order=2, max_depth=5)
    assert e.value.code == apc.APC_EDOMAIN
