"""Irregular domains (a voxel mask) on the GPU against the FP64 oracle.

Omega is the box minus the cells of a uniform coarse grid that the mask excludes;
walls are the box faces and the faces onto excluded cells, each node face on a wall
carrying a boundary node at its centre.  Bars as on the box: cloud, stencils and
integer coordinates bit-exact; operator and density rows within 1e-12; deposit
within 1e-13; Krylov solutions within the condition bar; the parameter rules
enforced.
"""
import sys

import numpy as np
import pytest

from linalg_bounds import interior_matrix, kappa2, solve_bar
from workloads import beam_halo, uniform_lattice_points

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


def l_mask(ml):
    s = 1 << ml
    m = np.zeros((s, s, s), bool)
    m[s // 2:, s // 2:, :] = True
    return m


def ball_mask(ml, R=0.45):
    s = 1 << ml
    c = (np.arange(s) + 0.5) / s - 0.5
    x, y, z = np.meshgrid(c, c, c, indexing="ij")
    return x * x + y * y + z * z > R * R


def filtered(xyz, mask):
    s = mask.shape[0]
    i = np.clip(np.floor(xyz * s).astype(int), 0, s - 1)
    return np.ascontiguousarray(xyz[:, ~mask[i[0], i[1], i[2]]])


CASES = {
    "L_k2": (lambda: l_mask(3), dict(order=2, c=0.3, max_depth=6)),
    "ball_k2": (lambda: ball_mask(3), dict(order=2, c=0.3, max_depth=6)),
    "L_k4": (lambda: l_mask(3), dict(order=4, c=0.06, max_depth=5)),
}


@pytest.fixture(scope="module", params=sorted(CASES))
def pair(request, apc, oracle_mod):
    mk, kw = CASES[request.param]
    mask = mk()
    xyz = filtered(beam_halo(30000, seed=17, sigma=(0.12, 0.12, 0.12)), mask)
    note(f"irregular {request.param}: {xyz.shape[1]} particles")
    O = oracle_mod.OracleCloud(xyz, mask=mask, **kw)
    G = apc.Cloud(cuda(xyz), precision=apc.APC_FP64, mask=mask, **kw)
    G.assemble_gfd()
    torch.cuda.synchronize()
    yield request.param, xyz, O, G
    G.close()


def test_irregular_cloud_bit_exact(pair):
    name, _, O, G = pair
    assert (G.n, G.nb, G.nnz, G.n_opened) == (O.n, O.nb, O.nnz, O.n_opened)
    a, b = O.nodes(), G.nodes()
    np.testing.assert_array_equal(a["perm"], b["perm"].astype(np.int64))
    for k in ("code", "level", "first", "count", "bowner", "bface", "st_off", "st_idx"):
        np.testing.assert_array_equal(a[k].astype(np.int64), b[k].astype(np.int64), err_msg=k)
    np.testing.assert_array_equal(O.coords(), b["ixyz"])
    note(f"  {name}: n={G.n} nb={G.nb} nnz={G.nnz} opened={G.n_opened}")


def test_irregular_rows_and_solves(pair):
    name, xyz, O, G = pair
    nd = O.nodes()
    m = np.diff(nd["st_off"])
    w_g, d_g = G.operator()
    w_o, d_o = O.assemble()
    assert np.max(np.abs(w_g - w_o) / np.repeat(np.abs(d_o), m)) <= 1e-12
    assert np.max(np.abs(d_g - d_o) / np.abs(d_o)) <= 1e-12
    bw_g, bd_g, ord_g = G.density_operator()
    bw_o, bd_o = O.density_rows()
    np.testing.assert_array_equal(ord_g, O.density_orders())
    assert max(np.abs(bw_g - bw_o).max(), np.abs(bd_g - bd_o).max()) <= 1e-12
    rm_o = O.deposit()
    rho_M, rho_t, std = G.deposit(tol=1e-13, maxit=4000)
    assert np.max(np.abs(rho_M.cpu().numpy() - rm_o) / np.maximum(np.abs(rm_o), 1e-300)) <= 1e-13
    rt_o, _ = O.density_solve(rm_o, tol=1e-13, maxit=4000)
    kB = kappa2(interior_matrix(nd["st_off"], nd["st_idx"], bw_o, bd_o, O.n), direct=False)
    e_rho = np.linalg.norm(rho_t.cpu().numpy() - rt_o) / np.linalg.norm(rt_o)
    assert std["status"] == 0 and e_rho <= solve_bar(kB, 1e-13, 1e-13, cap=1e-12)
    g = 0.01 * np.random.default_rng(4).standard_normal(O.nb)
    phi_o, _ = O.poisson_solve(rt_o[:O.n], g, tol=1e-13, maxit=20000, precond=1)
    phi, st = G.solve(cuda(rt_o[:O.n].copy()), cuda(g), tol=1e-13, maxit=20000)
    kL = kappa2(interior_matrix(nd["st_off"], nd["st_idx"], w_o, d_o, O.n))
    e_phi = np.linalg.norm(phi.cpu().numpy() - phi_o) / np.linalg.norm(phi_o)
    pp, gp = G.interpolate_force(phi)
    pp_o, gp_o = O.interpolate(phi_o)
    e_gp = np.linalg.norm(gp.cpu().numpy() - gp_o) / np.linalg.norm(gp_o)
    note(f"  {name}: density {e_rho:.2e} (kappa_B {kB:.2f}), Poisson {e_phi:.2e} "
         f"(kappa_L {kL:.2e}, iters {st['iters']}), grad_p {e_gp:.2e}")
    assert st["status"] == 0 and e_phi <= solve_bar(kL, 1e-13, 1e-13, cap=1e-10)
    np.testing.assert_array_equal(phi.cpu().numpy()[O.n:], g)
    assert e_gp <= 1e-9


def test_convex_corner_cloud_bit_exact(apc, oracle_mod):
    """Ball on an 8^3 voxel grid, 2e5 beam particles, depth 8: nodes at convex
    corners of the staircase take their stencil at ring_max without the octant that
    holds no node (the oracle's pin checks the geometry); same cloud and rows as the
    oracle."""
    mask = ball_mask(3)
    xyz = filtered(beam_halo(200000, seed=2, sigma=(0.08, 0.08, 0.08), halo_frac=0.05), mask)
    kw = dict(order=2, c=0.04, max_depth=8, mask=mask)
    note(f"irregular convex corners: {xyz.shape[1]} particles")
    O = oracle_mod.OracleCloud(xyz, **kw)
    G = apc.Cloud(cuda(xyz), precision=apc.APC_FP64, **kw)
    assert (G.n, G.nb, G.nnz, G.n_opened) == (O.n, O.nb, O.nnz, O.n_opened)
    a, b = O.nodes(), G.nodes()
    for k in ("code", "level", "bowner", "bface", "st_off", "st_idx"):
        np.testing.assert_array_equal(a[k].astype(np.int64), b[k].astype(np.int64), err_msg=k)
    G.assemble_gfd()
    w_g, d_g = G.operator()
    w_o, d_o = O.assemble()
    m = np.diff(a["st_off"])
    assert np.max(np.abs(w_g - w_o) / np.repeat(np.abs(d_o), m)) <= 1e-12
    note(f"  n={G.n} nb={G.nb} nnz={G.nnz}")
    G.close()


def test_irregular_lattice_uniform_rows(apc, oracle_mod):
    """The lattice inside the L (uniform rows, boxed slices of k = 4 away from the
    walls): structure bit-exact, rows and the operator apply within 1e-12."""
    mask = l_mask(2)
    for order in (2, 4):
        pts = filtered(uniform_lattice_points(4), mask)
        kw = dict(order=order, c=1e-3, max_depth=4, mask=mask)
        O = oracle_mod.OracleCloud(pts, **kw)
        G = apc.Cloud(cuda(pts), precision=apc.APC_FP64, **kw)
        G.assemble_gfd()
        assert (G.n, G.nb, G.nnz) == (O.n, O.nb, O.nnz) == (pts.shape[1], G.nb, G.nnz)
        np.testing.assert_array_equal(O.nodes()["st_idx"], G.nodes()["st_idx"])
        w_g, d_g = G.operator()
        w_o, d_o = O.assemble()
        m = np.diff(O.nodes()["st_off"])
        assert np.max(np.abs(w_g - w_o) / np.repeat(np.abs(d_o), m)) <= 1e-12
        f = np.random.default_rng(7).standard_normal(G.n + G.nb)
        got = G.apply_operator(cuda(f)).cpu().numpy()
        err = np.abs(got - O.apply_laplacian(f)) / (np.abs(d_o) * np.abs(f).max())
        info = G.operator_info()
        note(f"  lattice in the L, k = {order}: n={G.n} nb={G.nb}, uniform rows "
             f"{info.get('n_uniform')}, apply err {err.max():.2e}")
        assert err.max() <= 1e-12
        G.close()


def test_irregular_rejections(apc):
    mask = l_mask(2)
    xyz = filtered(beam_halo(3000, seed=3), mask)
    bad = np.concatenate([xyz, np.array([[0.9], [0.9], [0.5]])], axis=1)
    with pytest.raises(apc.ApcError) as e:
        apc.Cloud(cuda(bad), order=2, c=0.35, max_depth=5, mask=mask)
    assert e.value.code == apc.APC_EDOMAIN
    for kw in (dict(periodic=1), dict(kernel=1), dict(max_depth=1)):
        args = dict(order=2, c=0.35, max_depth=5, mask=mask)
        args.update(kw)
        with pytest.raises(apc.ApcError) as e:
            apc.Cloud(cuda(xyz), **args)
        assert e.value.code == apc.APC_EINVAL
    with pytest.raises(apc.ApcError) as e:
        apc.Cloud(cuda(xyz), order=2, c=0.35, max_depth=5, mask=np.ones((4, 4, 4), bool))
    assert e.value.code == apc.APC_EINVAL
    with pytest.raises(apc.ApcError) as e:
        apc.Batch([cuda(xyz), cuda(xyz)], order=2, max_depth=5, mask=mask)
    assert e.value.code == apc.APC_EINVAL
    x, v = cuda(xyz), torch.zeros_like(cuda(xyz))
    with pytest.raises(apc.ApcError) as e:
        apc.step(x, v, 1e-3, 1e-2, order=2, c=0.35, max_depth=5, mask=mask)
    assert e.value.code == apc.APC_EINVAL
