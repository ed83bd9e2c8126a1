"""Learned preconditioner on the GPU (via the C ABI) against the FP64 oracle.

Bars: training data within FP32 rounding of the oracle's FP64 values; FP32
gradients within 1e-4 (relative to the largest gradient entry of each layer) of
the oracle's FP64 back-propagation on the same FP32 inputs; BF16 inference
within the bound that follows from 8-bit mantissas (below); learned solves meet
the same true-residual tolerance as Jacobi ones.
"""
import sys

import numpy as np
import pytest

from workloads import beam_halo

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


@pytest.fixture(scope="module")
def lrn(apc):
    from paper_1603_04039_amd import learned
    return learned


SMALL = dict(order=2, c=0.45, max_depth=5)


@pytest.fixture(scope="module")
def small(apc, oracle_mod):
    note("small cloud (3000 particles, seed 21) on GPU and oracle")
    xyz = beam_halo(3000, seed=21)
    O = oracle_mod.OracleCloud(xyz, **SMALL)
    G = apc.Cloud(torch.from_numpy(xyz).cuda(), precision=apc.APC_FP64, **SMALL)
    G.assemble_gfd()
    torch.cuda.synchronize()
    assert (G.n, G.nb, G.nnz) == (O.n, O.nb, O.nnz)
    return O, G


def probes(n_tot, K, seed):
    return np.random.default_rng(seed).standard_normal((K, n_tot))


def test_learn_data_parity(small):
    note("learn_data parity (FP64 operator, K = 8 probes)")
    O, G = small
    Z = probes(O.n + O.nb, 8, 31)
    f_o, q_o = O.learn_data(Z)
    f_g, q_g = G.learn_data(torch.from_numpy(Z).cuda())
    f_g = f_g.cpu().numpy().astype(np.float64)
    q_g = q_g.cpu().numpy().astype(np.float64)
    # one FP32 rounding of an FP64 value (the FP64 parts agree to ~1e-13)
    np.testing.assert_allclose(f_g, f_o, rtol=2 ** -23, atol=1e-30)
    scale = np.abs(q_o).max(axis=1, keepdims=True)
    assert np.all(np.abs(q_g - q_o) <= 2 ** -23 * np.abs(q_o) + 1e-12 * scale)


def test_learn_data_features_mixed(apc, oracle_mod):
    """Mixed precision: the weight features come from the FP32 weights."""
    note("learn_data features, mixed precision")
    xyz = beam_halo(3000, seed=22)
    O = oracle_mod.OracleCloud(xyz, **SMALL)
    G = apc.Cloud(torch.from_numpy(xyz).cuda(), precision=apc.APC_MIXED, **SMALL)
    G.assemble_gfd()
    f_o, _ = O.learn_data()
    f_g, _ = G.learn_data()
    f_g = f_g.cpu().numpy().astype(np.float64)
    # FP32 fit (refit in FP64 when ill-conditioned) then an FP32 rounding: the
    # mixed-mode weight bar (1e-4 of the row's largest weight) carries over
    scale = np.abs(f_o[:, :40]).max(axis=1, keepdims=True)
    assert np.all(np.abs(f_g[:, :40] - f_o[:, :40]) <= 1e-4 * scale)
    np.testing.assert_allclose(f_g[:, 40:], f_o[:, 40:], rtol=2 ** -23, atol=0)
    G.close()


def _oracle_inputs(small, K=8, seed=41):
    """FP32 copies of the oracle's training data (inputs of both sides)."""
    O, _ = small
    f, q = O.learn_data(probes(O.n + O.nb, K, seed))
    return f.astype(np.float32), q.astype(np.float32)


@pytest.mark.parametrize("B", [1, 300, 1000])
def test_mlp_loss_grad_parity(apc, oracle_mod, small, B):
    note(f"mlp loss/grad parity B={B}")
    f32, q32 = _oracle_inputs(small)
    rng = np.random.default_rng(100 + B)
    P = (0.15 * rng.standard_normal(apc.MLP_NPARAM)).astype(np.float32)
    rows = rng.integers(0, f32.shape[0], size=B).astype(np.int32)
    L_o, g_o = oracle_mod.mlp_loss_grad(P.astype(np.float64), f32.astype(np.float64),
                                        q32.astype(np.float64), rows)
    L_g, g_g = apc.mlp_loss_grad(torch.from_numpy(P).cuda(), torch.from_numpy(f32).cuda(),
                                 torch.from_numpy(q32).cuda(), torch.from_numpy(rows).cuda())
    torch.cuda.synchronize()
    g_g = g_g.cpu().numpy().astype(np.float64)
    assert float(L_g.item()) == pytest.approx(L_o, rel=1e-4)
    IN, H, O = apc.MLP_IN, apc.MLP_HID, apc.MLP_OUT
    bounds = np.cumsum([0, IN * H, H, H * H, H, H * O, O])
    for a, b in zip(bounds[:-1], bounds[1:]):
        err = np.abs(g_g[a:b] - g_o[a:b]).max()
        assert err <= 1e-4 * max(np.abs(g_o[a:b]).max(), 1e-30), (a, b, err)


def test_adam_step(apc):
    note("adam step")
    rng = np.random.default_rng(3)
    n = apc.MLP_NPARAM
    P, m, v, g = [rng.standard_normal(n).astype(np.float32) for _ in range(4)]
    v = np.abs(v)
    dev = [torch.from_numpy(x.copy()).cuda() for x in (P, m, v, g)]
    step, lr = 7, 3e-3
    apc.mlp_adam(dev[0], dev[1], dev[2], dev[3], step, lr)
    torch.cuda.synchronize()
    P64, m64, v64, g64 = [x.astype(np.float64) for x in (P, m, v, g)]
    m1 = 0.9 * m64 + 0.1 * g64
    v1 = 0.999 * v64 + 0.001 * g64 ** 2
    P1 = P64 - lr * (m1 / (1 - 0.9 ** step)) / (np.sqrt(v1 / (1 - 0.999 ** step)) + 1e-8)
    np.testing.assert_allclose(dev[1].cpu().numpy(), m1, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(dev[2].cpu().numpy(), v1, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(dev[0].cpu().numpy(), P1, rtol=1e-6, atol=1e-6)


def test_inference_fp32_and_bf16(apc, lrn, oracle_mod, small):
    """FP32 inference within 1e-5 of the oracle's FP64 forward on the same FP32
    inputs.  BF16: features, weights and hidden activations are rounded to 8-bit
    mantissas (relative error <= 2^-9 per rounding, two rounded operands per
    product, three layers) and accumulated in FP32, so an output's error is at
    most about 6 * 2^-9 ~ 1.2% of the magnitude behind it, which the forward of
    the network with |W|, |b| on |x| bounds from above.  The bar is 2% of it."""
    note("inference FP32 / BF16 MFMA vs oracle forward")
    O, G = small
    rng = np.random.default_rng(12)
    P = lrn.init_params(5).cpu().numpy()
    n3 = apc.MLP_HID * apc.MLP_OUT + apc.MLP_OUT
    P[-n3:] = (0.2 * rng.standard_normal(n3)).astype(np.float32)
    f_o, _ = O.learn_data()
    f32 = f_o.astype(np.float32)
    o_ref = oracle_mod.mlp_forward(P.astype(np.float64), f32.astype(np.float64))
    mag = oracle_mod.mlp_forward(np.abs(P.astype(np.float64)), np.abs(f32.astype(np.float64)))
    Pd = torch.from_numpy(P).cuda()
    fd = torch.from_numpy(f32).cuda()
    o32 = G.mlp_infer(Pd, fd, bf16=False).cpu().numpy().astype(np.float64)
    o16 = G.mlp_infer(Pd, fd, bf16=True).cpu().numpy().astype(np.float64)
    assert np.all(np.abs(o32 - o_ref) <= 1e-5 * mag + 1e-7)
    err = np.abs(o16 - o_ref)
    note(f"bf16 max err / magnitude = {(err / mag).max():.4g}")
    assert np.all(err <= 0.02 * mag)
    # the BF16 path really rounds (not the FP32 kernel by another name)
    assert np.abs(o16 - o32).max() > 0.0


def _m_times(O, md, mw, f):
    nd = O.nodes()
    off, idx = nd["st_off"], nd["st_idx"]
    rows = np.repeat(np.arange(O.n), np.diff(off))
    out = md * f[:O.n]
    np.add.at(out, rows, mw * f[np.minimum(idx, O.n + O.nb - 1)] * (idx < O.n))
    return out


def _m_bound(O, oracle_mod, P, f, d, frac):
    """frac times the magnitude of each row of M f: the forward of the network
    with |W|, |b| on |x| bounds |o| and the BF16 error of o from above."""
    feat, _ = O.learn_data()
    mag = oracle_mod.mlp_forward(np.abs(P.astype(np.float64)),
                                 np.abs(feat.astype(np.float32).astype(np.float64)))
    nd = O.nodes()
    off, idx = nd["st_off"], nd["st_idx"]
    rows = np.repeat(np.arange(O.n), np.diff(off))
    pos = np.arange(off[-1]) - np.repeat(off[:-1], np.diff(off)) + 1
    tot = (mag[:, 0] + 1.0) * np.abs(f[:O.n])
    # M holds the first 40 stencil entries of a row (fourth-order rows are longer)
    np.add.at(tot, rows, np.where((idx < O.n) & (pos <= 40), mag[rows, np.minimum(pos, 40)], 0.0)
              * np.abs(f[np.minimum(idx, O.n + O.nb - 1)]))
    return frac * tot / np.abs(d)


def test_apply_precond(apc, lrn, oracle_mod, small):
    """M f of the installed learned M against the oracle's rows of M.  Uniform
    2-ring rows take the output of their level's first such row; their features
    are identical, so the oracle's per-row outputs agree.  Bar: the BF16
    inference bound (2% of the magnitude forward) through the row sum; with the
    safeguard 3% (alpha is computed from the BF16 outputs on the GPU and from FP64
    ones in the oracle).  Jacobi: f_i / d_i."""
    note("apply_precond: Jacobi and learned M vs oracle")
    O, G = small
    n, nt = O.n, O.n + O.nb
    rng = np.random.default_rng(17)
    f = rng.standard_normal(nt)
    fd = torch.from_numpy(f).cuda()
    _, d = O.assemble()
    outj = G.apply_precond(fd, apc.APC_PRECOND_JACOBI).cpu().numpy()
    np.testing.assert_allclose(outj, f[:n] / d, rtol=1e-14)
    np.testing.assert_array_equal(G.apply_precond(fd, apc.APC_PRECOND_NONE).cpu().numpy(), f[:n])
    P = lrn.init_params(3).cpu().numpy()
    n3 = apc.MLP_HID * apc.MLP_OUT + apc.MLP_OUT
    P[-n3:] = (0.05 * rng.standard_normal(n3)).astype(np.float32)
    Pd = torch.from_numpy(P).cuda()
    G.set_learned_precond(Pd)
    got = G.apply_precond(fd, apc.APC_PRECOND_LEARNED).cpu().numpy()
    md, mw = O.learned_m(P)
    err = np.abs(got - _m_times(O, md, mw, f))
    assert np.all(err <= _m_bound(O, oracle_mod, P, f, d, 0.02))
    # the install computes the features itself from the sliced layout: they must
    # be the ones apc_learn_data writes, so M agrees with the BF16 inference on
    # those features up to FP32 storage
    fg, _ = G.learn_data()
    o16 = G.mlp_infer(Pd, fg, bf16=True).cpu().numpy().astype(np.float64)
    nd = O.nodes()
    off, idx = nd["st_off"], nd["st_idx"]
    for i in range(n):
        J = [i] + list(idx[off[i]:off[i + 1]])
        live = np.array([j < n for j in J])
        Jc = np.array([j if j < n else 0 for j in J])
        mt = o16[i, :len(J)].copy()
        mt[0] += 1.0
        terms = np.where(live, mt * f[Jc], 0.0) / d[i]
        assert abs(got[i] - terms.sum()) <= 1e-5 * np.abs(terms).sum(), i
    # safeguard with probes
    Z = rng.standard_normal((8, nt))
    G.set_learned_precond(Pd, torch.from_numpy(Z).cuda())
    got_s = G.apply_precond(fd, apc.APC_PRECOND_LEARNED).cpu().numpy()
    md_s, mw_s = O.learned_m(P, Z)
    err = np.abs(got_s - _m_times(O, md_s, mw_s, f))
    assert np.all(err <= _m_bound(O, oracle_mod, P, f, d, 0.03))
    assert np.abs(got_s - got).max() > 0.0  # the safeguard changed rows


def test_learned_training_and_solve(apc, lrn):
    """A short training run on 20 clouds lowers the loss below Jacobi's; the
    installed M solves a held-out cloud to the same tolerance as Jacobi and to
    the same solution."""
    note("learned: data of 20 clouds")
    feat, quad = lrn.training_data(seeds=range(4000, 4020), K=32)
    P0 = lrn.init_params(0)
    l0 = lrn.full_loss(P0, feat, quad)
    note("learned: 600 Adam steps")
    P, hist = lrn.train(feat, quad, steps=600, batch=2048, lr=2e-3)
    l1 = lrn.full_loss(P, feat, quad)
    note(f"loss {l0:.5f} -> {l1:.5f}")
    assert l1 < 0.9 * l0
    cloud = lrn.make_cloud(5000)
    _, rho_t, _ = cloud.deposit(tol=1e-10, maxit=4000)
    b = rho_t[:cloud.n].contiguous()
    phi_j, st_j = cloud.solve(b, tol=1e-10, precond=apc.APC_PRECOND_JACOBI)
    cloud.set_learned_precond(P, lrn.probes(cloud, seed=1))
    phi_l, st_l = cloud.solve(b, tol=1e-10, precond=apc.APC_PRECOND_LEARNED)
    note(f"jacobi {st_j['iters']} it, learned {st_l['iters']} it")
    assert st_j["status"] == 0 and st_l["status"] == 0
    assert st_l["iters"] < st_j["iters"]
    assert st_l["precond_used"] == apc.APC_PRECOND_LEARNED
    assert st_l["rel_resid_true"] <= 1e-10
    d = (phi_l - phi_j)[:cloud.n].abs().max().item()
    assert d <= 1e-6 * phi_j[:cloud.n].abs().max().item()
    cloud.close()


def test_learned_fallback_to_jacobi(apc, lrn):
    """A network whose output is o = -e_0 makes M = 0 (singular): the learned
    iteration breaks down, the solve falls back to Jacobi and still converges."""
    note("learned: singular M falls back to Jacobi")
    P = np.zeros(apc.MLP_NPARAM, dtype=np.float32)
    P[-apc.MLP_OUT] = -1.0
    cloud = lrn.make_cloud(5001)
    _, rho_t, _ = cloud.deposit(tol=1e-10, maxit=4000)
    cloud.set_learned_precond(torch.from_numpy(P).cuda())
    phi, st = cloud.solve(rho_t[:cloud.n].contiguous(), tol=1e-8,
                          precond=apc.APC_PRECOND_LEARNED)
    assert st["status"] == 0
    assert st["precond_used"] == apc.APC_PRECOND_JACOBI
    assert st["rel_resid_true"] <= 1e-8
    cloud.close()


def test_learned_requires_install(apc, lrn):
    note("learned: solve without install is rejected")
    cloud = lrn.make_cloud(5002)
    b = torch.ones(cloud.n, dtype=torch.float64, device="cuda")
    with pytest.raises(apc.ApcError):
        cloud.solve(b, precond=apc.APC_PRECOND_LEARNED)
    P = lrn.init_params(0)
    cloud.set_learned_precond(P)
    cloud.assemble_gfd()  # re-assembly drops M
    with pytest.raises(apc.ApcError):
        cloud.solve(b, precond=apc.APC_PRECOND_LEARNED)
    cloud.close()


def test_learned_gain_held_out(apc, lrn):
    """Training on the 200 seeded clouds of the small beam recipe (seeds 4000..4199),
    evaluation on 20 held-out seeds (5000..5019): the learned M needs fewer
    iterations and less solve time than Jacobi to reach 1e-8, without fallback."""
    note("learned: training on 200 clouds")
    feat, quad = lrn.training_data()
    P, _ = lrn.train(feat, quad, steps=3000, batch=4096, lr=2e-3)
    del feat, quad
    note("learned: 20 held-out clouds")
    s = lrn.summarize(lrn.evaluate(P))
    note(f"held-out: {s}")
    assert s["fallbacks"] == 0
    assert s["iter_ratio"] >= 1.4
    assert s["time_ratio"] >= 1.2


# ---------------------------------------------------------------- k = 4
K4 = dict(order=4, c=0.05, max_depth=5)
# held-out bars (measured on MI355X: 2.89x fewer iterations, 1.99x less solve time)
K4_ITER_RATIO = 2.0
K4_TIME_RATIO = 1.4


@pytest.fixture(scope="module")
def small4(apc, oracle_mod):
    note("k = 4 cloud (20,000 particles, seed 31) on GPU and oracle")
    xyz = beam_halo(20000, seed=31)
    O = oracle_mod.OracleCloud(xyz, **K4)
    G = apc.Cloud(torch.from_numpy(xyz).cuda(), precision=apc.APC_FP64, **K4)
    G.assemble_gfd()
    torch.cuda.synchronize()
    assert (G.n, G.nb, G.nnz) == (O.n, O.nb, O.nnz)
    assert np.diff(O.nodes()["st_off"]).max() > 40  # rows longer than M's pattern
    return O, G


def test_k4_learn_data_parity(small4):
    """Fourth-order rows: the first 40 stencil entries make the features and M's
    pattern, on both sides."""
    note("k = 4 learn_data parity (FP64 operator, K = 8 probes)")
    O, G = small4
    Z = probes(O.n + O.nb, 8, 32)
    f_o, q_o = O.learn_data(Z)
    f_g, q_g = G.learn_data(torch.from_numpy(Z).cuda())
    f_g = f_g.cpu().numpy().astype(np.float64)
    q_g = q_g.cpu().numpy().astype(np.float64)
    # the FP64 rows of the two QR fits agree to ~1e-13 of |diag| (k = 4 parity),
    # then one FP32 rounding
    np.testing.assert_allclose(f_g, f_o, rtol=2 ** -23, atol=1e-11)
    scale = np.abs(q_o).max(axis=1, keepdims=True)
    assert np.all(np.abs(q_g - q_o) <= 2 ** -23 * np.abs(q_o) + 1e-11 * scale)


def test_k4_apply_precond(apc, lrn, oracle_mod, small4):
    """The installed M of a fourth-order cloud against the oracle's rows of M
    (every row general, first 40 stencil entries), with and without the
    safeguard; bars as for k = 2."""
    note("k = 4 apply_precond: learned M vs oracle")
    O, G = small4
    n, nt = O.n, O.n + O.nb
    rng = np.random.default_rng(18)
    f = rng.standard_normal(nt)
    fd = torch.from_numpy(f).cuda()
    _, d = O.assemble()
    P = lrn.init_params(4).cpu().numpy()
    n3 = apc.MLP_HID * apc.MLP_OUT + apc.MLP_OUT
    P[-n3:] = (0.05 * rng.standard_normal(n3)).astype(np.float32)
    Pd = torch.from_numpy(P).cuda()
    G.set_learned_precond(Pd)
    got = G.apply_precond(fd, apc.APC_PRECOND_LEARNED).cpu().numpy()
    md, mw = O.learned_m(P)
    err = np.abs(got - _m_times(O, md, mw, f))
    assert np.all(err <= _m_bound(O, oracle_mod, P, f, d, 0.02))
    Z = rng.standard_normal((8, nt))
    G.set_learned_precond(Pd, torch.from_numpy(Z).cuda())
    got_s = G.apply_precond(fd, apc.APC_PRECOND_LEARNED).cpu().numpy()
    md_s, mw_s = O.learned_m(P, Z)
    err = np.abs(got_s - _m_times(O, md_s, mw_s, f))
    assert np.all(err <= _m_bound(O, oracle_mod, P, f, d, 0.03))
    assert np.abs(got_s - got).max() > 0.0


@pytest.mark.timeout(600)
def test_k4_learned_gain_held_out(apc, lrn):
    """Training on 200 seeded clouds of the anisotropic recipe at k = 4 (seeds
    6000..6199), evaluation on 20 held-out seeds (7000..7019): fewer iterations
    and less solve time than Jacobi to reach 1e-8, without fallback."""
    rec = lrn.RECIPES[4]
    note("k = 4 learned: training on 200 clouds")
    feat, quad = lrn.training_data(rec["train"], workload=rec["workload"], log=note)
    note(f"k = 4 learned: {feat.shape[0]} rows, 3000 Adam steps")
    P, _ = lrn.train(feat, quad, steps=3000, batch=4096, lr=2e-3, log=note, log_every=1000)
    del feat, quad
    note("k = 4 learned: 20 held-out clouds")
    s = lrn.summarize(lrn.evaluate(P, rec["held_out"], workload=rec["workload"]))
    note(f"k = 4 held-out: {s}")
    assert s["fallbacks"] == 0
    assert s["iter_ratio"] >= K4_ITER_RATIO
    assert s["time_ratio"] >= K4_TIME_RATIO

