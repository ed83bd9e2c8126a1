"""Fourth-order GFD (k = 4) on the GPU against the FP64 oracle.

Both sides fit with Householder QR in FP64 (the GPU: one wavefront per node),
so the bars are rounding-order bounds: operator rows within 1e-9 of the row's
|diag| (kappa(W V0) eps with kappa up to ~1e5 for 34-unknown stencils), the
node cloud, stencils and the order-2 fallback decisions bit-exact, Krylov
solutions within kappa (tol_gpu + tol_oracle).
"""
import sys

import numpy as np
import pytest

from workloads import beam_halo, uniform_lattice_points

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

K4A = dict(order=4, c=0.05, max_depth=5)   # 20,000 particles: 9,332 nodes, 185 order-2 rows
K4B = dict(order=4, c=0.05, max_depth=6)   # 50,000 particles: 16,234 nodes, 281 order-2 rows


def note(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def apc():
    from paper_1603_04039_amd import apcloud
    apcloud.load_library()
    assert torch.cuda.is_available()
    return apcloud


def gcloud(apc, xyz, **kw):
    return apc.Cloud(torch.from_numpy(np.ascontiguousarray(xyz)).cuda(), **kw)


@pytest.fixture(scope="module", params=["A", "B"])
def pair(request, apc, oracle_mod):
    if request.param == "A":
        xyz, kw = beam_halo(20000, seed=31), K4A
    else:
        xyz, kw = beam_halo(50000, seed=32), K4B
    note(f"k = 4 cloud {request.param}: oracle and GPU builds")
    O = oracle_mod.OracleCloud(xyz, **kw)
    G = gcloud(apc, xyz, precision=apc.APC_FP64, **kw)
    G.assemble_gfd()
    torch.cuda.synchronize()
    return xyz, O, G


def test_k4_structure_bit_exact(pair):
    xyz, O, G = pair
    note(f"k = 4 structure: n={O.n}")
    assert (G.n, G.nb, G.nnz, G.n_opened) == (O.n, O.nb, O.nnz, O.n_opened)
    a, b = O.nodes(), G.nodes()
    for k in ("perm", "code", "level", "first", "count", "bowner", "bface", "st_off", "st_idx"):
        np.testing.assert_array_equal(a[k].astype(np.int64), b[k].astype(np.int64), err_msg=k)
    np.testing.assert_array_equal(O.node_orders(), G.node_orders())
    note(f"order-2 fallback rows: {int((G.node_orders() == 2).sum())}")


def test_k4_operator_rows(pair):
    xyz, O, G = pair
    w_g, d_g = G.operator()
    w_o, d_o = O.assemble()
    m = np.diff(O.nodes()["st_off"])
    err = np.max(np.abs(w_g - w_o) / np.repeat(np.abs(d_o), m))
    derr = np.max(np.abs(d_g - d_o) / np.abs(d_o))
    note(f"k = 4 rows: max |w_gpu - w_oracle| / |diag| = {err:.2e}, diag {derr:.2e}")
    assert err <= 1e-9 and derr <= 1e-9


def test_k4_quartic_exactness(apc, pair):
    """Order-4 rows are exact on quartics, order-2 rows on quadratics (GPU alone)."""
    xyz, O, G = pair
    rng = np.random.default_rng(5)
    pos = G.positions()
    orders = G.node_orders()
    for deg, sel in ((4, orders == 4), (2, orders == 2)):
        if not sel.any():
            continue
        c = rng.standard_normal(5)
        x, y, z = pos
        if deg == 4:
            f = c[0] * x ** 4 + c[1] * x ** 2 * y * z + c[2] * y ** 3 * z + c[3] * z ** 4 + c[4] * x * y
            lap = (12 * c[0] * x ** 2 + 2 * c[1] * y * z + 6 * c[2] * y * z + 12 * c[3] * z ** 2)
        else:
            f = c[0] * x ** 2 + c[1] * y * z + c[2] * z ** 2 + c[3] * x
            lap = 2 * c[0] + 2 * c[2] + 0 * x
        got = G.apply_operator(torch.from_numpy(f).cuda()).cpu().numpy()[sel]
        want = lap[:G.n][sel]
        assert np.abs(got - want).max() <= 1e-7 * max(1.0, np.abs(want).max()), deg


def test_k4_deposit_and_solve(apc, pair):
    xyz, O, G = pair
    rho_M, rho_t, std = G.deposit(tol=1e-13, maxit=4000)
    rM_o = O.deposit()
    np.testing.assert_allclose(rho_M.cpu().numpy(), rM_o, rtol=1e-13)
    rt_o, sto = O.density_solve(rM_o, tol=1e-13, maxit=4000)
    d = np.abs(rho_t.cpu().numpy() - rt_o).max() / np.abs(rt_o).max()
    note(f"k = 4 density: rel diff {d:.2e}, iters gpu {std['iters']} oracle {sto['iters']}")
    assert d <= 1e-10
    # Poisson solve of the oracle's right-hand side on both sides
    rhs = torch.from_numpy(np.ascontiguousarray(rt_o[:O.n])).cuda()
    phi, st = G.solve(rhs, tol=1e-12, maxit=20000)
    phi_o, sto = O.poisson_solve(rt_o[:O.n], tol=1e-12, maxit=20000, precond=1)
    d = np.abs(phi.cpu().numpy() - phi_o).max() / np.abs(phi_o).max()
    note(f"k = 4 Poisson: rel diff {d:.2e}, iters gpu {st['iters']} oracle {sto['iters']}")
    assert st["status"] == 0 and d <= 1e-7


def test_k4_derivatives_and_interpolation(apc, pair):
    xyz, O, G = pair
    rng = np.random.default_rng(8)
    phi = rng.standard_normal(O.n + O.nb)
    D_o = O.node_derivs(phi)
    D_g = G.node_derivs(torch.from_numpy(phi).cuda()).cpu().numpy()
    assert D_g.shape == D_o.shape == (O.n, 34)
    scale = np.abs(D_o).max(axis=0) + 1e-300
    err = (np.abs(D_g - D_o) / scale).max()
    note(f"k = 4 derivatives: max err / column scale = {err:.2e}")
    assert err <= 1e-9
    pp_o, gp_o = O.interpolate(phi)
    pp_g, gp_g = G.interpolate_force(torch.from_numpy(phi).cuda())
    np.testing.assert_allclose(pp_g.cpu().numpy(), pp_o, rtol=0, atol=1e-10 * np.abs(pp_o).max())
    np.testing.assert_allclose(gp_g.cpu().numpy(), gp_o, rtol=0, atol=1e-9 * np.abs(gp_o).max())


def test_k4_mixed_weights(apc, oracle_mod):
    """Mixed precision keeps the FP64 fit and stores FP32 weights."""
    xyz = beam_halo(20000, seed=31)
    O = oracle_mod.OracleCloud(xyz, **K4A)
    G = gcloud(apc, xyz, precision=apc.APC_MIXED, **K4A)
    G.assemble_gfd()
    w_g, _ = G.operator()
    w_o, d_o = O.assemble()
    m = np.diff(O.nodes()["st_off"])
    err = np.max(np.abs(w_g - w_o) / np.repeat(np.abs(d_o), m))
    note(f"k = 4 mixed: max |w32 - w64| / |diag| = {err:.2e}")
    assert err <= 1e-6
    _, rho_t, _ = G.deposit(tol=1e-10, maxit=4000)
    phi, st = G.solve(rho_t[:G.n].contiguous(), tol=1e-8)
    assert st["status"] == 0 and st["rel_resid_true"] <= 1e-8
    G.close()


def test_k4_lattice_stencils(apc, oracle_mod):
    """Uniform lattice: interior order-4 stencils of 56 nodes, same on both sides."""
    xyz = uniform_lattice_points(4)
    O = oracle_mod.OracleCloud(xyz, order=4, c=1e-3, max_depth=4)
    G = gcloud(apc, xyz, order=4, c=1e-3, max_depth=4)
    a, b = O.nodes(), G.nodes()
    np.testing.assert_array_equal(a["st_off"], b["st_off"])
    np.testing.assert_array_equal(a["st_idx"], b["st_idx"])
    assert np.diff(b["st_off"]).max() == 56
    G.close()


def test_k4_batch_rejected(apc):
    """Batches carry k = 2 operators only."""
    xyz = beam_halo(20000, seed=31)
    with pytest.raises(apc.ApcError):
        apc.Batch([torch.from_numpy(xyz).cuda()], **K4A)
