"""CIC and TSC charge assignment on the GPU against the FP64 oracle.

The GPU gathers each node's particles from the 3 x 3 x 3 block of cells of its
size around it (Morton ranges of the sorted particles); the oracle takes every
particle against every node.  Bars: rho_M within 1e-13 relative (the sums run in
different orders), density rows within 1e-12 and their orders equal (the rows of
nodes whose kernel reaches past a wall carry odd and mixed moments and are fitted
on their own), density solves within kappa_B (1e-13 + 1e-13), and one whole field
solve (deposit, density solve, Poisson solve, interpolation) within the bounded
domain's chain bars.
"""
import sys

import numpy as np
import pytest

from linalg_bounds import interior_matrix, kappa2, solve_bar
from workloads import beam_halo

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

CIC, TSC = 1, 2
CASES = {
    (2, CIC): (dict(order=2, c=0.35, max_depth=6), 20000, 9),
    (2, TSC): (dict(order=2, c=0.35, max_depth=6), 20000, 9),
    (4, CIC): (dict(order=4, c=0.05, max_depth=5), 20000, 31),
    (4, TSC): (dict(order=4, c=0.05, max_depth=5), 20000, 31),
}


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


@pytest.fixture(scope="module", params=sorted(CASES))
def pair(request, apc, oracle_mod):
    order, kernel = request.param
    kw, N, seed = CASES[request.param]
    note(f"order {order}, kernel {'CIC' if kernel == CIC else 'TSC'}: beam_halo {N} (seed {seed})")
    xyz = beam_halo(N, seed=seed)
    O = oracle_mod.OracleCloud(xyz, kernel=kernel, **kw)
    G = apc.Cloud(cuda(xyz), precision=apc.APC_FP64, kernel=kernel, **kw)
    G.assemble_gfd()
    torch.cuda.synchronize()
    yield order, kernel, xyz, O, G
    G.close()


def test_kernel_deposit(pair):
    order, kernel, xyz, O, G = pair
    q = np.random.default_rng(3).uniform(0.5, 1.5, xyz.shape[1])
    for qq in (None, q):
        rm_o = O.deposit(qq)
        rho_M, _, _ = G.deposit(None if qq is None else cuda(qq), tol=1e-13)
        rm_g = rho_M.cpu().numpy()
        err = np.max(np.abs(rm_g - rm_o) / np.maximum(np.abs(rm_o), 1e-300))
        note(f"  deposit ({'uniform' if qq is None else 'random'} q): max rel err {err:.2e}")
        assert err <= 1e-13


def test_kernel_density_rows(pair):
    order, kernel, _, O, G = pair
    bw_g, bd_g, ord_g = G.density_operator()
    bw_o, bd_o = O.density_rows()
    ord_o = O.density_orders()
    np.testing.assert_array_equal(ord_g, ord_o)
    err = max(np.abs(bw_g - bw_o).max(), np.abs(bd_g - bd_o).max())
    nd = O.nodes()
    pos = O.positions()[:, :O.n]
    h = O.L / 2.0 ** nd["level"]
    wall = np.any((pos < 1.5 * h) | (pos > 1.0 - 1.5 * h), axis=0)
    note(f"  density rows: max err {err:.2e}; orders {np.bincount(ord_g, minlength=5).tolist()}, "
         f"wall-layer rows {int(wall.sum())} (kept order > 0: {int((wall & (ord_g > 0)).sum())})")
    assert err <= 1e-12
    off = nd["st_off"]
    assert np.all(np.add.reduceat(np.abs(bw_g), off[:-1]) <= 0.5 * bd_g * (1 + 1e-12))


def test_kernel_density_and_field_solve(pair):
    """Deposit -> density solve -> Poisson solve -> interpolation on both sides."""
    order, kernel, xyz, O, G = pair
    nd = O.nodes()
    rm_o = O.deposit()
    rt_o, st_o = O.density_solve(rm_o, tol=1e-13, maxit=4000)
    rho_M, rho_t, std = G.deposit(tol=1e-13, maxit=4000)
    bw, bd = O.density_rows()
    kB = kappa2(interior_matrix(nd["st_off"], nd["st_idx"], bw, bd, O.n), direct=False)
    e_rho = np.linalg.norm(rho_t.cpu().numpy() - rt_o) / np.linalg.norm(rt_o)
    note(f"  density solve: iters gpu {std['iters']} oracle {st_o['iters']}, kappa_B {kB:.2f}, "
         f"rel diff {e_rho:.2e}")
    assert std["status"] == 0 and st_o["status"] == 0
    assert e_rho <= solve_bar(kB, 1e-13, 1e-13, cap=1e-12)
    phi, st = G.solve(rho_t[:G.n].contiguous(), tol=1e-13, maxit=20000)
    phi_o, _ = O.poisson_solve(rt_o[:O.n], tol=1e-13, maxit=20000, precond=1)
    w, d = O.assemble()
    kL = kappa2(interior_matrix(nd["st_off"], nd["st_idx"], w, d, O.n))
    e_phi = np.linalg.norm(phi.cpu().numpy() - phi_o) / np.linalg.norm(phi_o)
    pp, gp = G.interpolate_force(phi)
    pp_o, gp_o = O.interpolate(phi_o)
    e_gp = np.linalg.norm(gp.cpu().numpy() - gp_o) / np.linalg.norm(gp_o)
    note(f"  Poisson: rel diff {e_phi:.2e} (kappa_L {kL:.2e}); grad_p {e_gp:.2e}")
    assert e_phi <= min(2.0 * kL * (2e-13 + e_rho), 1e-10)
    assert e_gp <= 1e-9


@pytest.mark.parametrize("kernel", [CIC, TSC])
def test_kernel_periodic_deposit_and_rows(apc, oracle_mod, kernel):
    """Periodic domain: the kernel wraps around (minimum-image offsets), no node is
    beside a wall, every a_0 is 1."""
    xyz = beam_halo(20000, seed=41)
    kw = dict(order=2, c=0.3, max_depth=5, periodic=1, kernel=kernel)
    O = oracle_mod.OracleCloud(xyz, **kw)
    G = apc.Cloud(cuda(xyz), precision=apc.APC_FP64, **kw)
    G.assemble_gfd()
    rm_o = O.deposit()
    rho_M, _, st = G.deposit(tol=1e-13)
    err = np.max(np.abs(rho_M.cpu().numpy() - rm_o) / np.maximum(np.abs(rm_o), 1e-300))
    bw_g, bd_g, ord_g = G.density_operator()
    bw_o, bd_o = O.density_rows()
    np.testing.assert_array_equal(ord_g, O.density_orders())
    rerr = max(np.abs(bw_g - bw_o).max(), np.abs(bd_g - bd_o).max())
    note(f"periodic kernel {kernel}: deposit {err:.2e}, rows {rerr:.2e}")
    assert err <= 1e-13 and rerr <= 1e-12 and st["status"] == 0
    # the total charge: the kernel weights of every particle sum to 1 only on a
    # uniform lattice; here the charge is conserved to the kernel's smoothing
    h = O.L / 2.0 ** O.nodes()["level"]
    tot = float((rho_M.cpu().numpy()[:G.n] * h ** 3).sum())
    assert abs(tot - 1.0) <= 0.05
    G.close()


def test_kernel_rejected_by_batches(apc):
    x = cuda(beam_halo(1000, seed=3))
    with pytest.raises(apc.ApcError) as e:
        apc.Batch([x, x], order=2, max_depth=5, kernel=CIC)
    assert e.value.code == apc.APC_EINVAL
    with pytest.raises(apc.ApcError) as e:
        apc.Cloud(x, order=2, max_depth=5, kernel=3)
    assert e.value.code == apc.APC_EINVAL


@pytest.mark.parametrize("kernel,periodic", [(CIC, 0), (TSC, 1)])
def test_kernel_deposit_deep_tree(apc, oracle_mod, kernel, periodic):
    """A tree deeper than the deposit's leaf table (levels 8 and 9 under the
    table's level 7): rho_M within 1e-13 of the oracle, bounded and periodic."""
    xyz = beam_halo(20000, seed=4, sigma=(0.03, 0.03, 0.03))
    kw = dict(order=2, c=0.01, max_depth=9, kernel=kernel, periodic=periodic)
    note(f"deep tree deposit, kernel {kernel}, periodic {periodic}")
    O = oracle_mod.OracleCloud(xyz, **kw)
    G = apc.Cloud(cuda(xyz), precision=apc.APC_FP64, **kw)
    G.assemble_gfd()
    assert G.nodes()["level"].max() >= 8
    rm_o = O.deposit()
    rho_M, _, st = G.deposit(tol=1e-12)
    err = np.max(np.abs(rho_M.cpu().numpy() - rm_o) / np.maximum(np.abs(rm_o), 1e-300))
    note(f"  n={G.n}: deposit {err:.2e}")
    assert err <= 1e-13 and st["status"] == 0
    G.close()
