"""Periodic domains on the GPU against the FP64 oracle.

On a periodic domain face neighbours wrap around, there are no boundary nodes,
stencil offsets are minimum images and the Poisson problem is
Delta phi = c (rho~ - mean rho~) with phi_0 = 0 in place of node 0's equation and
phi shifted to mean 0 afterwards (means weighted by cell volume).  Bars as for the
bounded domain: cloud, stencils and integer coordinates bit-exact, operator,
density and derivative rows within 1e-12, Krylov solutions within the condition
bar of the pinned operator, the push bit for bit.
"""
import sys

import numpy as np
import pytest

from linalg_bounds import interior_matrix, kappa2, solve_bar
from workloads import beam_halo, uniform_lattice_points

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

KW = {2: dict(order=2, c=0.3, max_depth=5, periodic=1),
      4: dict(order=4, c=0.06, max_depth=5, periodic=1)}


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


def bits(a):
    return np.ascontiguousarray(a).view(np.uint64)


@pytest.fixture(scope="module", params=[2, 4])
def pair(request, apc, oracle_mod):
    k = request.param
    note(f"periodic beam_halo 20000 (seed 41), order {k}: oracle and GPU builds")
    xyz = beam_halo(20000, seed=41)
    O = oracle_mod.OracleCloud(xyz, **KW[k])
    G = apc.Cloud(cuda(xyz), precision=apc.APC_FP64, **KW[k])
    G.assemble_gfd()
    torch.cuda.synchronize()
    yield k, xyz, O, G
    G.close()


def assert_same_cloud(O, G):
    assert (G.n, G.nb, G.nnz, G.n_opened) == (O.n, O.nb, O.nnz, O.n_opened)
    a, b = O.nodes(), G.nodes()
    np.testing.assert_array_equal(a["perm"], b["perm"].astype(np.int64))
    for k in ("code", "level", "first", "count", "st_off", "st_idx"):
        np.testing.assert_array_equal(a[k].astype(np.int64), b[k].astype(np.int64), err_msg=k)
    np.testing.assert_array_equal(O.coords(), b["ixyz"])


def test_periodic_cloud_and_rows(pair):
    k, _, O, G = pair
    note(f"periodic order {k}: structure, operator, density rows, apply")
    assert G.nb == 0
    assert_same_cloud(O, G)
    m = np.diff(O.nodes()["st_off"])
    w_g, d_g = G.operator()
    w_o, d_o = O.assemble()
    assert np.max(np.abs(w_g - w_o) / np.repeat(np.abs(d_o), m)) <= 1e-12
    assert np.max(np.abs(d_g - d_o) / np.abs(d_o)) <= 1e-12
    bw_g, bd_g, ord_g = G.density_operator()
    bw_o, bd_o = O.density_rows()
    np.testing.assert_array_equal(ord_g, O.density_orders())
    assert max(np.abs(bw_g - bw_o).max(), np.abs(bd_g - bd_o).max()) <= 1e-12
    f = np.random.default_rng(13).standard_normal(G.n)
    got = G.apply_operator(cuda(f)).cpu().numpy()
    err = np.abs(got - O.apply_laplacian(f)) / (np.abs(d_o) * np.abs(f).max())
    note(f"  n={G.n} nnz={G.nnz} apply max err {err.max():.2e}")
    assert err.max() <= 1e-12


def test_periodic_derivatives_and_interpolation(pair):
    k, _, O, G = pair
    phi = np.random.default_rng(8).standard_normal(O.n)
    D_o = O.node_derivs(phi)
    D_g = G.node_derivs(cuda(phi)).cpu().numpy()
    assert D_g.shape == D_o.shape
    err = (np.abs(D_g - D_o) / (np.abs(D_o).max(axis=0) + 1e-300)).max()
    pp_o, gp_o = O.interpolate(phi)
    pp_g, gp_g = G.interpolate_force(cuda(phi))
    e_pp = np.abs(pp_g.cpu().numpy() - pp_o).max() / np.abs(pp_o).max()
    e_gp = np.abs(gp_g.cpu().numpy() - gp_o).max() / np.abs(gp_o).max()
    note(f"periodic order {k}: derivatives {err:.2e}, phi_p {e_pp:.2e}, grad_p {e_gp:.2e}")
    assert err <= 1e-12 and e_pp <= 1e-12 and e_gp <= 1e-12


def pinned_matrix(O):
    """The oracle's Laplacian with row 0 replaced by the identity row."""
    nd = O.nodes()
    w, d = O.assemble()
    A = interior_matrix(nd["st_off"], nd["st_idx"], w, d, O.n).tolil()
    A[0, :] = 0.0
    A[0, 0] = 1.0
    return A.tocsr()


def periodic_bar(O, phi_o, t_gpu, t_oracle):
    """Relative bar for two zero-mean periodic solutions: the pinned solutions
    y = phi - phi_0 differ by at most 2 kappa (t_gpu + t_oracle) ||y|| (kappa of
    the pinned operator); phi = P y with the projection P = I - 1 v^T / sum(v)
    onto volume-weighted mean 0, of 2-norm at most 1 + sqrt(n) ||v|| / sum(v)."""
    vol = 0.5 ** (3 * O.nodes()["level"].astype(np.float64))
    kap = kappa2(pinned_matrix(O))
    pnorm = 1.0 + np.sqrt(O.n) * np.linalg.norm(vol) / vol.sum()
    y_o = phi_o - phi_o[0]
    bar = pnorm * solve_bar(kap, t_gpu, t_oracle) * np.linalg.norm(y_o) / np.linalg.norm(phi_o)
    return bar, kap, pnorm


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_periodic_solve(apc, oracle_mod, pair, precision):
    """Both sides to their tolerance; phi of volume-weighted mean 0.  FP64: within
    the condition bar of the pinned operator of the oracle's phi.  Mixed: the
    operator is the FP32 fit's, so the bar is the one of the bounded domain's
    mixed mode (1e-4, the FP32 fit's weight error carried through the solve), and
    the FP64 reference residual is not computed (-1)."""
    k, _, O, G = pair
    tol = 1e-13 if precision == "fp64" else 1e-11
    note(f"periodic order {k} Poisson solve, {precision}")
    rt_o, _ = O.density_solve(O.deposit(), tol=1e-13, maxit=4000)
    rhs = rt_o[:O.n].copy()
    phi_o, sto = O.poisson_solve(rhs, tol=1e-13, maxit=20000, precond=1)
    if precision == "fp64":
        Gs = G
    else:
        Gs = apc.Cloud(cuda(beam_halo(20000, seed=41)), precision=apc.APC_MIXED, **KW[k])
        Gs.set_diagnostics(apc.APC_DIAG_FP64_RESIDUAL)
        Gs.assemble_gfd()
    phi, st = Gs.solve(cuda(rhs), tol=tol, maxit=20000, precond=1)
    phi_g = phi.cpu().numpy()
    if Gs is not G:
        Gs.close()
    assert st["status"] == 0 and sto["status"] == 0
    assert st["rel_resid_true"] <= tol
    vol = 0.5 ** (3 * O.nodes()["level"].astype(np.float64))
    mean = np.dot(vol, phi_g) / vol.sum()
    assert abs(mean) <= 1e-13 * np.abs(phi_g).max()
    bar, kap, pnorm = periodic_bar(O, phi_o, tol, 1e-13)
    rel = np.linalg.norm(phi_g - phi_o) / np.linalg.norm(phi_o)
    note(f"  iters gpu {st['iters']} oracle {sto['iters']}, kappa {kap:.3e}, |P| {pnorm:.2f}, "
         f"rel diff {rel:.2e} (bar {bar:.2e})")
    if precision == "fp64":
        assert rel <= min(bar, 1e-8)
    else:
        assert rel <= 1e-4 and st["rel_resid_fp64ref"] == -1.0


@pytest.mark.parametrize("order,depth", [(2, 4), (4, 4), (4, 3)])
def test_periodic_lattice(apc, oracle_mod, order, depth):
    """Uniform lattice on the torus: every row has the same stencil (the seam rows
    too), so every k = 4 row is a uniform 56-node row and every 4 x 4 x 4 block is
    boxed; rows, apply and solve against the oracle."""
    xyz = uniform_lattice_points(depth)
    kw = dict(order=order, c=1e-3, max_depth=depth, periodic=1)
    note(f"periodic lattice order {order}, {2 ** depth}^3")
    O = oracle_mod.OracleCloud(xyz, **kw)
    G = apc.Cloud(cuda(xyz), precision=apc.APC_FP64, **kw)
    G.assemble_gfd()
    assert_same_cloud(O, G)
    n = 8 ** depth
    assert G.n == n and G.nb == 0
    assert np.all(np.diff(G.nodes()["st_off"]) == (24 if order == 2 else 56))
    if order == 4:
        assert G.operator_info()["n_uniform"] == n
        assert G.operator_boxes() == n // 64
    w_g, d_g = G.operator()
    w_o, d_o = O.assemble()
    assert np.ptp(d_o) <= 1e-12 * np.abs(d_o).max()
    assert np.max(np.abs(w_g - w_o) / np.abs(d_o[0])) <= 1e-12
    assert np.max(np.abs(d_g - d_o) / np.abs(d_o)) <= 1e-12
    f = np.random.default_rng(17).standard_normal(n)
    got = G.apply_operator(cuda(f)).cpu().numpy()
    err = np.abs(got - O.apply_laplacian(f)) / (np.abs(d_o) * np.abs(f).max())
    assert err.max() <= 1e-12
    pos = O.positions()
    rho = np.cos(2 * np.pi * pos[0]) * np.sin(2 * np.pi * pos[1]) + 0.3
    phi_o, _ = O.poisson_solve(rho, tol=1e-13, maxit=20000, precond=1)
    phi, st = G.solve(cuda(rho), tol=1e-13, maxit=20000, precond=1)
    rel = np.linalg.norm(phi.cpu().numpy() - phi_o) / np.linalg.norm(phi_o)
    bar, kap, _ = periodic_bar(O, phi_o, 1e-13, 1e-13)
    note(f"  apply err {err.max():.2e}, solve iters {st['iters']} rel diff {rel:.2e} "
         f"(kappa {kap:.2e}, bar {bar:.2e})")
    assert st["status"] == 0 and rel <= min(bar, 1e-8)
    G.close()


@pytest.mark.parametrize("N", [1, 100_003])
def test_periodic_push_bit_exact(apc, oracle_mod, N):
    note(f"periodic push parity N={N}")
    lo, L = (-0.5, 0.25, 1.0), 1.5
    rng = np.random.default_rng(N + 9)
    x = np.array(lo)[:, None] + L * rng.random((3, N))
    v = rng.standard_normal((3, N))
    v[:, : N // 3] *= 8 * L
    g = rng.standard_normal((3, N))
    kick, dt = 0.0125, 0.7
    xg, vg = cuda(x), cuda(v)
    apc.push(xg, vg, cuda(g), kick, dt, lo=lo, L=L, periodic=1)
    torch.cuda.synchronize()
    xo, vo = oracle_mod.push(x, v, g, kick, dt, lo, L, periodic=1)
    np.testing.assert_array_equal(bits(xg.cpu().numpy()), bits(xo))
    np.testing.assert_array_equal(bits(vg.cpu().numpy()), bits(vo))
    xs = xg.cpu().numpy()
    for d in range(3):
        assert xs[d].min() >= lo[d] and xs[d].max() <= lo[d] + L


def test_periodic_step_against_oracle_chain(apc, oracle_mod):
    note("one periodic time step, beam_halo 20000 (seed 43)")
    prm = KW[2]
    x = beam_halo(20000, seed=43)
    v = 0.1 * np.random.default_rng(2).standard_normal(x.shape)
    kick, dt = 2e-3, 1e-2
    xg, vg = cuda(x), cuda(v)
    pp, gp, st = apc.step(xg, vg, kick, dt, tol_density=1e-13, tol=1e-12, precision=apc.APC_FP64,
                          **prm)
    torch.cuda.synchronize()
    note(f"  n={st['n']} iters={st['iters']} density_iters={st['density_iters']}")
    assert st["rc"] == apc.APC_OK and st["status"] == apc.APC_OK
    O = oracle_mod.OracleCloud(x, **prm)
    rt, _ = O.density_solve(O.deposit(), tol=1e-13, maxit=20000)
    phi_o, _ = O.poisson_solve(rt[:O.n], tol=1e-12, maxit=20000, precond=1)
    pp_o, gp_o = O.interpolate(phi_o)
    assert (st["n"], st["nb"], st["nnz"]) == (O.n, 0, O.nnz)
    pp, gp = pp.cpu().numpy(), gp.cpu().numpy()
    assert np.linalg.norm(pp - pp_o) <= 1e-8 * np.linalg.norm(pp_o)
    assert np.linalg.norm(gp - gp_o) <= 1e-7 * np.linalg.norm(gp_o)
    x1, v1 = oracle_mod.push(x, v, gp, kick, dt, periodic=1)
    np.testing.assert_array_equal(bits(xg.cpu().numpy()), bits(x1))
    np.testing.assert_array_equal(bits(vg.cpu().numpy()), bits(v1))


def test_periodic_rejections(apc):
    x = cuda(beam_halo(1000, seed=3))
    with pytest.raises(apc.ApcError) as e:
        apc.Cloud(x, order=2, max_depth=1, periodic=1)
    assert e.value.code == apc.APC_EINVAL
    with pytest.raises(apc.ApcError) as e:
        apc.Batch([x, x], order=2, max_depth=5, periodic=1)
    assert e.value.code == apc.APC_EINVAL
