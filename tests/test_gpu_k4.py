"""Fourth-order GFD (k = 4) on the GPU against the FP64 oracle.

Both sides fit with Householder QR in FP64 (the GPU: one wavefront per node),
so operator rows, density rows, derivatives and interpolated values agree to
1e-12 relative; the node cloud, stencils, the order-2 fallback decisions and the
density-row orders bit-exact; Krylov solutions, both sides at 1e-13, within
kappa_2 (1e-13 + 1e-13) with kappa_2 estimated from the oracle's operator, and
at most 1e-10 (Poisson) or 1e-12 (density).
"""
import math
import sys

import numpy as np
import pytest

from linalg_bounds import interior_matrix, kappa2, moment_row, row_ok, solve_bar
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
    assert err <= 1e-12 and derr <= 1e-12


SHELL56 = np.repeat(np.arange(1, 6), [6, 12, 8, 6, 24])  # r^2 (cells) of entry j


def uniform56_rows(nd, orders, D):
    """Rows (order 4) whose stencil is the uniform 56-node lattice stencil of their
    own level: the entry j of the (r^2, index) order lies at a lattice offset of
    one cell spacing with r^2 = SHELL56[j] (host classification from the node
    arrays)."""
    off, idx, lv, crd = nd["st_off"], nd["st_idx"], nd["level"], nd["ixyz"].astype(np.int64)
    rows = np.flatnonzero((np.diff(off) == 56) & (orders == 4))
    if rows.size == 0:
        return rows
    nb = idx[off[rows][:, None] + np.arange(56)[None, :]]
    sp = (1 << (D - lv[rows] + 1)).astype(np.int64)[:, None]
    r2 = np.zeros(nb.shape, np.int64)
    good = np.ones(nb.shape, bool)
    for d in range(3):
        dd = np.abs(crd[d][nb] - crd[d][rows][:, None])
        good &= (dd == 0) | (dd == sp) | (dd == 2 * sp)
        r2 += (dd // sp) ** 2
    good &= r2 == SHELL56[None, :]
    return rows[good.all(axis=1)]


def test_k4_uniform_rows(apc, pair):
    """Rows with the uniform 56-node stencil share shell constants and the SpMV
    reads no weights for them: the GPU flags exactly the rows a host
    classification finds, their CSR rows (written from the constants) are within
    1e-12 of the oracle's fits (test_k4_operator_rows), and the operator apply
    equals the oracle's row by row within 1e-12 of |d_i| max|f|, on the uniform
    rows and on the others."""
    xyz, O, G = pair
    nd = G.nodes()
    uni = uniform56_rows(nd, G.node_orders(), G.max_depth)
    info = G.operator_info()
    note(f"k = 4 uniform 56-node rows: {info['n_uniform']} of {G.n} (host {uni.size})")
    assert info["n_uniform"] == uni.size > 0
    assert info["nnz_general"] == G.nnz - 56 * uni.size
    rng = np.random.default_rng(12)
    f = rng.standard_normal(G.n + G.nb)
    got = G.apply_operator(torch.from_numpy(f).cuda()).cpu().numpy()
    want = O.apply_laplacian(f)
    _, d_o = O.assemble()
    err = np.abs(got - want) / (np.abs(d_o) * np.abs(f).max())
    mask = np.zeros(G.n, bool)
    mask[uni] = True
    note(f"k = 4 apply: max err uniform rows {err[mask].max():.2e}, "
         f"other rows {err[~mask].max():.2e}")
    assert err.max() <= 1e-12


def test_k4_density_rows(pair):
    """Density rows (eq. density_linear_system) with the stability rule: row
    orders (4, 2 for the order-2 row of the same stencil, 0 for the identity)
    equal to the oracle's, rows within 1e-12, every row within
    sum_j |b_ij| <= 0.5 b_ii."""
    xyz, O, G = pair
    bw_g, bd_g, ord_g = G.density_operator()
    bw_o, bd_o = O.density_rows()
    np.testing.assert_array_equal(ord_g, O.density_orders())
    err = max(np.abs(bw_g - bw_o).max(), np.abs(bd_g - bd_o).max())
    note(f"k = 4 density rows: orders {np.bincount(ord_g, minlength=5).tolist()}, "
         f"max diff {err:.2e}")
    assert err <= 1e-12
    off = O.nodes()["st_off"]
    assert np.all(np.add.reduceat(np.abs(bw_g), off[:-1]) <= 0.5 * bd_g * (1 + 1e-12))


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
    nd = O.nodes()
    rho_M, rho_t, std = G.deposit(tol=1e-13, maxit=4000)
    rM_o = O.deposit()
    np.testing.assert_allclose(rho_M.cpu().numpy(), rM_o, rtol=1e-13)
    rt_o, sto = O.density_solve(rM_o, tol=1e-13, maxit=4000)
    bw, bd = O.density_rows()
    kB = kappa2(interior_matrix(nd["st_off"], nd["st_idx"], bw, bd, O.n), direct=False)
    d = np.linalg.norm(rho_t.cpu().numpy() - rt_o) / np.linalg.norm(rt_o)
    note(f"k = 4 density: rel diff {d:.2e}, iters gpu {std['iters']} oracle {sto['iters']}, "
         f"kappa_B {kB:.2f}")
    assert std["status"] == 0 and std["iters"] <= 12
    assert d <= solve_bar(kB, 1e-13, 1e-13, cap=1e-12)
    # Poisson solve of the oracle's right-hand side on both sides
    w, dg = O.assemble()
    kL = kappa2(interior_matrix(nd["st_off"], nd["st_idx"], w, dg, O.n))
    rhs = torch.from_numpy(np.ascontiguousarray(rt_o[:O.n])).cuda()
    phi, st = G.solve(rhs, tol=1e-13, maxit=20000)
    phi_o, sto = O.poisson_solve(rt_o[:O.n], tol=1e-13, maxit=20000, precond=1)
    d = np.linalg.norm(phi.cpu().numpy() - phi_o) / np.linalg.norm(phi_o)
    note(f"k = 4 Poisson: rel diff {d:.2e}, iters gpu {st['iters']} oracle {sto['iters']}, "
         f"kappa_L {kL:.3e}")
    assert st["status"] == 0 and sto["status"] == 0
    assert d <= solve_bar(kL, 1e-13, 1e-13, cap=1e-10)


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
    assert err <= 1e-12
    pp_o, gp_o = O.interpolate(phi)
    pp_g, gp_g = G.interpolate_force(torch.from_numpy(phi).cuda())
    e_pp = np.abs(pp_g.cpu().numpy() - pp_o).max() / np.abs(pp_o).max()
    e_gp = np.abs(gp_g.cpu().numpy() - gp_o).max() / np.abs(gp_o).max()
    note(f"k = 4 interpolation: phi {e_pp:.2e}, grad {e_gp:.2e} (relative to the max)")
    assert e_pp <= 1e-12 and e_gp <= 1e-12


def test_k4_mixed_weights(apc, oracle_mod):
    """Mixed precision keeps the FP64 fit and stores FP32 weights; with the FP64
    reference residual requested, the mixed solve's residual on the FP64 rows
    equals that of the oracle's operator applied to its potential."""
    xyz = beam_halo(20000, seed=31)
    O = oracle_mod.OracleCloud(xyz, **K4A)
    G = gcloud(apc, xyz, precision=apc.APC_MIXED, **K4A)
    G.set_diagnostics(apc.APC_DIAG_FP64_RESIDUAL)
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
    rt = rho_t.cpu().numpy()[:O.n]
    want = np.linalg.norm(O.apply_laplacian(phi.cpu().numpy()) - rt) / np.linalg.norm(rt)
    note(f"k = 4 mixed: own residual {st['rel_resid_true']:.2e}, FP64 reference "
         f"{st['rel_resid_fp64ref']:.2e}, oracle operator {want:.2e}")
    assert abs(st["rel_resid_fp64ref"] - want) <= 1e-3 * want
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
    # the nodes two or more cells from every face have the uniform 56-node
    # stencil: 12^3 of the 16^3 lattice
    G.assemble_gfd()
    uni = uniform56_rows(b, G.node_orders(), 4)
    assert G.operator_info()["n_uniform"] == uni.size == 12 ** 3
    # complete 4 x 4 x 4 blocks of uniform rows: origins at 4 and 8 per axis
    assert G.operator_boxes() == 8
    w_g, d_g = G.operator()
    w_o, d_o = O.assemble()
    m = np.diff(a["st_off"])
    assert np.max(np.abs(w_g - w_o) / np.repeat(np.abs(d_o), m)) <= 1e-12
    bw_g, bd_g, ord_g = G.density_operator()
    bw_o, bd_o = O.density_rows()
    np.testing.assert_array_equal(ord_g, O.density_orders())
    assert max(np.abs(bw_g - bw_o).max(), np.abs(bd_g - bd_o).max()) <= 1e-12
    f = np.random.default_rng(13).standard_normal(G.n + G.nb)
    got = G.apply_operator(torch.from_numpy(f).cuda()).cpu().numpy()
    err = np.abs(got - O.apply_laplacian(f)) / (np.abs(d_o) * np.abs(f).max())
    note(f"k = 4 lattice: {uni.size} uniform rows, density row order "
         f"{int(ord_g[uni[0]])}, apply max err {err.max():.2e}")
    assert err.max() <= 1e-12
    G.close()


def test_k4_batch_rejected(apc):
    """Batches carry k = 2 operators only."""
    xyz = beam_halo(20000, seed=31)
    with pytest.raises(apc.ApcError):
        apc.Batch([torch.from_numpy(xyz).cuda()], **K4A)


# ---------------------------------------------------------------- full size
@pytest.mark.slow
@pytest.mark.timeout(900)
def test_k4_full_size_sampled(apc, oracle_mod):
    """beam_halo_1e8_k4 at full size (1e8 particles, ~8.8e6 nodes), mixed precision
    with the learned M, as the bench runs it.  The oracle cannot build a cloud
    this size, so it checks sampled outputs one node at a time: operator rows
    (the oracle's WLS fit on the GPU's stencil, at the row's order; stencil
    selection is bit-exact at the smaller sizes above), the deposit, and the
    Taylor interpolation of sampled particles from the GPU potential.  The solve
    must reach the 1e-8 true residual with the learned M and no fallback."""
    from paper_1603_04039_amd import learned as lrn
    from workloads import CONFIGS
    cfg = CONFIGS["beam_halo_1e8_k4"]
    note("k = 4 full size: generating 1e8 particles")
    xyz = beam_halo(cfg["N"], seed=cfg["seed"], sigma=cfg["sigma"], halo_frac=cfg["halo_frac"])
    kw = dict(order=4, c=cfg["c"], max_depth=cfg["max_depth"])
    note("k = 4 full size: GPU build and assembly")
    G = gcloud(apc, xyz, precision=apc.APC_MIXED, **kw)
    G.assemble_gfd()
    n, nb, N = G.n, G.nb, G.N
    nd = G.nodes()
    off, idx, lev = nd["st_off"], nd["st_idx"], nd["level"]
    pos = G.lo[:, None] + G.unit * nd["ixyz"].astype(np.float64)
    orders = G.node_orders()
    note(f"k = 4 full size: n={n} nb={nb} nnz={G.nnz} order-2 rows={int((orders == 2).sum())}")
    assert int(nd["count"].astype(np.int64).sum()) == N
    assert np.all(np.diff(off) >= np.where(orders == 4, 35, 10))
    w, d = G.operator()
    rng = np.random.default_rng(11)
    sample = rng.choice(n, 400, replace=False)
    worst = 0.0
    for i in sample:
        nbr = idx[off[i]:off[i + 1]]
        X, h, ratio = oracle_mod.wls_fit(int(orders[i]), (pos[:, nbr] - pos[:, [i]]).T)
        assert ratio >= 1e-6
        wl = (X[3] + X[6] + X[8]) / h ** 2
        err = np.abs(w[off[i]:off[i + 1]] - wl).max() / abs(d[i])
        worst = max(worst, err)
        assert abs(d[i] + wl.sum()) <= 1e-6 * abs(d[i])
    note(f"k = 4 full size: 400 sampled rows, max |w_gpu - w_oracle| / |diag| = {worst:.2e}")
    assert worst <= 1e-6  # FP32 weights of the FP64 fit
    del w
    note("k = 4 full size: deposit")
    rho_M, rho_t, std = G.deposit(tol=1e-10, maxit=20000)
    note(f"k = 4 full size: density solve {std['iters']} iterations, "
         f"true residual {std['rel_resid_true']:.2e}")
    assert std["status"] == 0 and std["iters"] <= 20
    rM = rho_M.cpu().numpy()
    hc = G.L / 2.0 ** lev[sample]
    np.testing.assert_allclose(rM[sample], nd["count"][sample] / N / hc ** 3, rtol=1e-13)
    # the oracle's density rows (its fit on the GPU's stencil, the stability rule
    # replayed) applied to the GPU's rho~ give rho_M to the solve tolerance plus the
    # FP32 rounding of the stored rows
    bw, bd, dord = G.density_operator()
    rt = rho_t.cpu().numpy()
    al4, al2 = oracle_mod.monomials(4), oracle_mod.monomials(2)
    nrm = np.linalg.norm(rM[:n])
    worst = 0.0
    for i in sample:
        nbr = idx[off[i]:off[i + 1]]
        dl = (pos[:, nbr] - pos[:, [i]]).T
        hci = G.L / 2.0 ** int(lev[i])
        ko = int(orders[i])
        X, h, _ = oracle_mod.wls_fit(ko, dl)
        b = moment_row(X, hci, h, al4 if ko == 4 else al2)
        if ko == 4 and not row_ok(b):
            X2, h2, _ = oracle_mod.wls_fit(2, dl)
            b = moment_row(X2, hci, h2, al2)
            want = 2 if row_ok(b) else 0
        else:
            want = ko if row_ok(b) else 0
        assert dord[i] == want, i
        if want == 0:
            b = np.zeros_like(b)
        assert np.abs(bw[off[i]:off[i + 1]] - b).max() <= 1e-6 * max(np.abs(b).max(), 1e-300) \
            or want == 0
        diff = rt[nbr] - rt[i]
        r = rt[i] + b @ diff - rM[i]
        bar = 1e-10 * nrm + 1e-7 * (np.abs(b) @ np.abs(diff))
        worst = max(worst, abs(r) / bar)
        assert abs(r) <= bar, i
    note(f"k = 4 full size: 400 sampled density rows (orders "
         f"{np.bincount(dord, minlength=5).tolist()} over all rows): max residual / bar = {worst:.2e}")
    note("k = 4 full size: learned M install and solve")
    P = torch.from_numpy(np.load(lrn.params_path(4))).cuda()
    G.set_learned_precond(P, lrn.probes(G, seed=0))
    phi, st = G.solve(rho_t[:n].contiguous(), tol=1e-8, maxit=20000,
                      precond=apc.APC_PRECOND_LEARNED)
    note(f"k = 4 full size: {st['iters']} iterations, true residual {st['rel_resid_true']:.2e}")
    assert st["status"] == 0 and st["rel_resid_true"] <= 1e-8
    assert st["precond_used"] == apc.APC_PRECOND_LEARNED
    # the oracle's Poisson rows applied to the GPU's phi (zero on the boundary) give
    # rho~ to the solve tolerance plus the FP32 rounding of the stored weights
    ph = phi.cpu().numpy()
    rtn = np.linalg.norm(rt[:n])
    worst = 0.0
    for i in sample:
        nbr = idx[off[i]:off[i + 1]]
        X, h, _ = oracle_mod.wls_fit(int(orders[i]), (pos[:, nbr] - pos[:, [i]]).T)
        wl = (X[3] + X[6] + X[8]) / h ** 2
        diff = ph[nbr] - ph[i]
        r = wl @ diff - rt[i]
        bar = 1e-8 * rtn + 1e-7 * (np.abs(wl) @ np.abs(diff))
        worst = max(worst, abs(r) / bar)
        assert abs(r) <= bar, i
    note(f"k = 4 full size: 400 sampled Poisson rows: max residual / bar = {worst:.2e}")
    note("k = 4 full size: interpolation of sampled particles")
    phi_p, grad_p = G.interpolate_force(phi)
    pp, gp = phi_p.cpu().numpy(), grad_p.cpu().numpy()
    alphas = oracle_mod.monomials(4)
    fact = np.array([np.prod([math.factorial(int(e)) for e in a]) for a in alphas], dtype=float)
    perm, first, count = nd["perm"], nd["first"], nd["count"]
    occupied = sample[count[sample] > 0][:200]
    assert occupied.size >= 50
    for i in occupied:
        p = int(perm[first[i]])
        nbr = idx[off[i]:off[i + 1]]
        X, h, _ = oracle_mod.wls_fit(int(orders[i]), (pos[:, nbr] - pos[:, [i]]).T)
        a = alphas[:X.shape[0]]
        df = ph[nbr] - ph[i]
        hk = h ** a.sum(axis=1)
        D = X @ df / hk
        Dm = np.abs(X) @ np.abs(df) / hk  # magnitude behind each derivative
        dl = xyz[:, p] - pos[:, i]
        mono = np.prod(dl[None, :] ** a, axis=1) / fact[:len(a)]
        # the value and the gradient of the Taylor polynomial at the particle; bars
        # relative to the magnitudes that enter them (kappa eps of the two fits)
        assert abs(pp[p] - (ph[i] + D @ mono)) <= 1e-9 * (abs(ph[i]) + Dm @ np.abs(mono)), i
        for c in range(3):
            ok = a[:, c] > 0
            da = a[ok].copy()
            da[:, c] -= 1
            dm = a[ok, c] * np.prod(dl[None, :] ** da, axis=1) / fact[:len(a)][ok]
            assert abs(gp[c, p] - D[ok] @ dm) <= 1e-9 * (Dm[ok] @ np.abs(dm)), (i, c)
    G.close()
