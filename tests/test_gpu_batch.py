"""Batches of clouds on the GPU (via the C ABI).

A batch must give every cloud what a single-cloud call gives it: node counts
equal, the deposit and the interpolation (same kernels on the same rows)
bit-exact, Krylov solutions within the solve tolerance times the conditioning
(the per-cloud dot products are summed in a different order than in the
single-cloud solver, so iterates agree to rounding, not bit for bit).  HIP
graph replays must equal the eager launches exactly, also with other work
between replays.  One small cloud is checked against the FP64 oracle directly.
"""
import sys

import numpy as np
import pytest

from workloads import BATCH, batch_specs, beam_halo

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SMALL = dict(order=2, c=0.35, max_depth=6)


def note(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def apc():
    from paper_1603_04039_amd import apcloud
    apcloud.load_library()
    assert torch.cuda.is_available()
    return apcloud


def small_specs():
    # the many-cloud recipe with particle counts scaled down (fast, still uneven)
    out = []
    for sp in batch_specs(count=6):
        out.append(dict(sp, N=max(2000, sp["N"] // 40)))
    return out


def cloud_points(sp):
    return beam_halo(sp["N"], seed=sp["seed"], sigma=sp["sigma"], halo_frac=sp["halo_frac"])


@pytest.fixture(scope="module")
def small_batch(apc):
    specs = small_specs()
    pts = [cloud_points(sp) for sp in specs]
    note(f"small batch: N = {[p.shape[1] for p in pts]}")
    xs = [torch.from_numpy(p).cuda() for p in pts]
    B = apc.Batch(xs, precision=apc.APC_MIXED, **SMALL)
    B.assemble_gfd()
    singles = []
    for x in xs:
        c = apc.Cloud(x, precision=apc.APC_MIXED, **SMALL)
        c.assemble_gfd()
        singles.append(c)
    torch.cuda.synchronize()
    return B, singles, xs, pts


def test_batch_sizes(small_batch):
    note("batch sizes vs single clouds")
    B, singles, _, _ = small_batch
    assert B.count == len(singles)
    for c, S in enumerate(singles):
        assert (B.cloud_N[c], B.cloud_n[c], B.cloud_nb[c]) == (S.N, S.n, S.nb)
    assert B.n == sum(S.n for S in singles) and B.nb == sum(S.nb for S in singles)


def test_batch_deposit_matches_single(apc, small_batch):
    note("batch deposit vs single-cloud deposit")
    B, singles, _, _ = small_batch
    rho_M, rho_t, st = B.deposit(tol=1e-12, maxit=4000)
    assert all(s["status"] == 0 for s in st)
    for c, S in enumerate(singles):
        rM, rt, st1 = S.deposit(tol=1e-12, maxit=4000)
        idx = torch.from_numpy(B.node_index(c)).cuda()
        assert torch.equal(rho_M[idx], rM)  # same kernel, same rows: bit-exact
        d = (rho_t[idx] - rt).abs().max().item()
        assert d <= 1e-9 * rt.abs().max().item()
        # the density system is well conditioned: same iteration count within 1
        assert abs(st[c]["iters"] - st1["iters"]) <= 1


@pytest.mark.parametrize("precond", ["jacobi", "none"])
def test_batch_solve_matches_single(apc, small_batch, precond):
    note(f"batch Poisson solve vs single clouds ({precond})")
    B, singles, _, _ = small_batch
    pc = apc.APC_PRECOND_JACOBI if precond == "jacobi" else apc.APC_PRECOND_NONE
    _, rho_t, _ = B.deposit(tol=1e-12, maxit=4000)
    phi, st = B.solve(rho_t, tol=1e-10, maxit=20000, precond=pc)
    for c, S in enumerate(singles):
        idx = torch.from_numpy(B.node_index(c)).cuda()
        rt = rho_t[idx][:S.n].contiguous()
        phi1, st1 = S.solve(rt, tol=1e-10, maxit=20000, precond=pc)
        assert st[c]["status"] == 0 and st1["status"] == 0
        assert st[c]["rel_resid_true"] <= 1e-10
        d = (phi[idx] - phi1).abs().max().item()
        note(f"cloud {c}: n={S.n} iters batch {st[c]['iters']} single {st1['iters']} diff {d:.2e}")
        assert d <= 1e-6 * phi1.abs().max().item()
        assert abs(st[c]["iters"] - st1["iters"]) <= max(3, st1["iters"] // 10)


def test_batch_learned_matches_single(apc, small_batch):
    """The learned preconditioner installed on the batch (one install over the
    union, probes Z) against each cloud's own install with the same probes (its
    columns of Z): the per-cloud solves agree as the Jacobi ones do, and the
    learned solves take fewer iterations than Jacobi."""
    from paper_1603_04039_amd import learned
    note("batch learned preconditioner vs single clouds")
    B, singles, _, _ = small_batch
    _, rho_t, _ = B.deposit(tol=1e-12, maxit=4000)
    with pytest.raises(apc.ApcError) as e:
        B.solve(rho_t, tol=1e-10, precond=apc.APC_PRECOND_LEARNED)
    assert e.value.code == apc.APC_EINVAL
    params = torch.from_numpy(np.load(learned.params_path(2))).cuda()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(11)
    Z = torch.randn((learned.SAFEGUARD_PROBES, B.n + B.nb), dtype=torch.float64, device="cuda",
                    generator=gen)
    B.set_learned_precond(params, Z)
    phi, st = B.solve(rho_t, tol=1e-10, maxit=20000, precond=apc.APC_PRECOND_LEARNED)
    _, stj = B.solve(rho_t, tol=1e-10, maxit=20000, precond=apc.APC_PRECOND_JACOBI)
    it_l = it_j = 0
    for c, S in enumerate(singles):
        idx = torch.from_numpy(B.node_index(c)).cuda()
        S.set_learned_precond(params, Z[:, idx].contiguous())
        rt = rho_t[idx][:S.n].contiguous()
        phi1, st1 = S.solve(rt, tol=1e-10, maxit=20000, precond=apc.APC_PRECOND_LEARNED)
        assert st[c]["status"] == 0 and st1["status"] == 0
        assert st[c]["precond_used"] == apc.APC_PRECOND_LEARNED
        assert st[c]["rel_resid_true"] <= 1e-10
        d = (phi[idx] - phi1).abs().max().item()
        note(f"cloud {c}: n={S.n} iters batch {st[c]['iters']} single {st1['iters']} "
             f"(Jacobi {stj[c]['iters']}) diff {d:.2e}")
        assert d <= 1e-6 * phi1.abs().max().item()
        assert abs(st[c]["iters"] - st1["iters"]) <= max(3, st1["iters"] // 10)
        it_l += st[c]["iters"]
        it_j += stj[c]["iters"]
    assert it_l < it_j
    # the pipeline graph with the learned M: replays equal the separate entry points
    bufs, sd0, sp0, used0 = B.pipeline(tol_density=1e-10, tol=1e-10,
                                       precond=apc.APC_PRECOND_LEARNED)
    ref = [b.clone() for b in bufs]
    for _ in range(2):
        out, sd, sp, used = B.pipeline(tol_density=1e-10, tol=1e-10,
                                       precond=apc.APC_PRECOND_LEARNED, out=bufs)
        assert used and all(x["status"] == 0 for x in sd + sp)
        assert all(x["precond_used"] == apc.APC_PRECOND_LEARNED for x in sp)
        for a, b in zip(out, ref):
            assert torch.equal(a, b)


def test_batch_interpolation_bit_exact(apc, small_batch):
    note("batch interpolation vs single clouds on the same phi")
    B, singles, _, _ = small_batch
    _, rho_t, _ = B.deposit(tol=1e-12, maxit=4000)
    phi, _ = B.solve(rho_t, tol=1e-10)
    phi_p, grad_p = B.interpolate_force(phi)
    for c, S in enumerate(singles):
        idx = torch.from_numpy(B.node_index(c)).cuda()
        pp, gp = S.interpolate_force(phi[idx].contiguous())
        a, b = int(B.pbase[c]), int(B.pbase[c] + B.cloud_N[c])
        assert torch.equal(phi_p[a:b], pp)
        assert torch.equal(grad_p[:, a:b], gp)


def test_batch_graph_replays_equal_eager(apc, small_batch):
    """Graph replays against eager launches, with eager work of the program
    between replays; every replay must give the eager result bit for bit."""
    note("batch graph replays vs eager")
    B, singles, _, _ = small_batch
    _, rho_t, _ = B.deposit(tol=1e-12, maxit=4000)
    B.configure(use_graph=0, chunk=8)
    phi_e, st_e = B.solve(rho_t, tol=1e-10)
    B.configure(use_graph=1, chunk=8)
    for rep in range(4):
        phi_g, st_g = B.solve(rho_t, tol=1e-10)
        assert torch.equal(phi_g, phi_e), rep
        assert [s["iters"] for s in st_g] == [s["iters"] for s in st_e]
        # unrelated eager work between replays
        singles[rep % len(singles)].apply_operator(
            torch.rand(singles[rep % len(singles)].n + singles[rep % len(singles)].nb,
                       dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
    # another chunk length re-records the graph
    B.configure(chunk=4)
    phi_4, _ = B.solve(rho_t, tol=1e-10)
    B.configure(use_graph=0)
    phi_4e, _ = B.solve(rho_t, tol=1e-10)
    assert torch.equal(phi_4, phi_4e)
    B.configure(use_graph=1, chunk=8)


def test_batch_pipeline_graph(apc, small_batch):
    """The whole field solve of the batch (assembly, deposit and density solve,
    Poisson solve, interpolation) as one graph replay: the first call runs the
    separate entry points and sets the iteration budgets, later calls replay the
    graph and give the same outputs and iteration counts bit for bit, also with
    other work of the program between replays; a tighter tolerance records a new
    graph (or falls back once to the separate entry points and enlarges the
    budgets) and still converges."""
    note("batch pipeline graph vs the separate entry points")
    B, singles, _, _ = small_batch
    pc = apc.APC_PRECOND_JACOBI
    out, sd0, sp0, used = B.pipeline(tol_density=1e-12, tol=1e-10, precond=pc)
    assert not used
    assert all(s["status"] == 0 for s in sd0 + sp0)
    ref = [t.clone() for t in out]
    # the separate entry points themselves give the same values
    _, rho_t, _ = B.deposit(tol=1e-12, maxit=20000)
    phi, _ = B.solve(rho_t, tol=1e-10, precond=pc)
    assert torch.equal(rho_t, ref[0]) and torch.equal(phi, ref[1])
    for rep in range(3):
        out2, sd, sp, used = B.pipeline(tol_density=1e-12, tol=1e-10, precond=pc, out=out)
        assert used, rep
        for a, b in zip(out2, ref):
            assert torch.equal(a, b), rep
        assert [s["iters"] for s in sd] == [s["iters"] for s in sd0]
        assert [s["iters"] for s in sp] == [s["iters"] for s in sp0]
        assert all(s["status"] == 0 for s in sd + sp)
        S = singles[rep % len(singles)]
        S.apply_operator(torch.rand(S.n + S.nb, dtype=torch.float64, device="cuda"))
        torch.cuda.synchronize()
    used_any = False
    for k in range(3):
        out3, sd, sp, used = B.pipeline(tol_density=1e-12, tol=1e-12, precond=pc, out=out)
        assert all(s["status"] == 0 for s in sd + sp)
        assert all(s["rel_resid_true"] <= 1e-12 for s in sp)
        note(f"  tol 1e-12 call {k}: graph {used}, iters {[s['iters'] for s in sp]}")
        used_any = used_any or used
    assert used_any


def test_batch_tune(apc, small_batch):
    note("batch autotuner")
    B, _, _, _ = small_batch
    div, chunk = B.tune(tol=1e-8)
    assert div in (1, 2, 4, 8) and chunk in (4, 8, 16, 32)
    assert B.info["chunk"] == chunk
    _, rho_t, _ = B.deposit(tol=1e-12, maxit=4000)
    phi, st = B.solve(rho_t, tol=1e-8)
    assert all(s["status"] == 0 for s in st)


def test_batch_noconv_reported(apc, small_batch):
    note("batch: maxit = 2 reports non-convergence per cloud")
    B, _, _, _ = small_batch
    _, rho_t, _ = B.deposit(tol=1e-12, maxit=4000)
    phi, st = B.solve(rho_t, tol=1e-12, maxit=2)
    assert all(s["status"] == apc.APC_ENOCONV for s in st)
    assert all(s["rc"] == apc.APC_ENOCONV for s in st)
    assert all(s["iters"] <= 2 + 8 for s in st)  # stops within one replay of maxit


def test_batch_vs_oracle(apc, oracle_mod):
    """Two clouds, the smaller one checked against the oracle's FP64 solve."""
    note("batch of 2 vs oracle")
    p1 = beam_halo(4000, seed=71)
    p2 = beam_halo(12000, seed=72)
    B = apc.Batch([torch.from_numpy(p1).cuda(), torch.from_numpy(p2).cuda()],
                  precision=apc.APC_FP64, **SMALL)
    B.assemble_gfd()
    _, rho_t, _ = B.deposit(tol=1e-12, maxit=4000)
    O = oracle_mod.OracleCloud(p1, **SMALL)
    assert (O.n, O.nb) == (B.cloud_n[0], B.cloud_nb[0])
    rt_o = O.density_solve(O.deposit(), tol=1e-13, maxit=4000)[0]
    idx = torch.from_numpy(B.node_index(0)).cuda()
    rt_g = rho_t[idx].cpu().numpy()
    np.testing.assert_allclose(rt_g, rt_o, rtol=0, atol=1e-9 * np.abs(rt_o).max())
    # the Poisson solve of cloud 0 from the oracle's own right-hand side
    rho_in = rho_t.clone()
    rho_in[idx] = torch.from_numpy(rt_o).cuda()
    phi, st = B.solve(rho_in, tol=1e-12)
    assert st[0]["status"] == 0 and st[1]["status"] == 0
    phi_o, _ = O.poisson_solve(rt_o[:O.n], tol=1e-13, maxit=20000, precond=1)
    np.testing.assert_allclose(phi[idx].cpu().numpy(), phi_o, rtol=0,
                               atol=1e-7 * np.abs(phi_o).max())
    B.close()


@pytest.mark.slow
def test_batch64_full(apc):
    """The 64-cloud recipe at full size: every cloud converges to 1e-8, and the
    smallest and largest clouds agree with single-cloud solves."""
    specs = batch_specs(master_seed=BATCH["master_seed"], count=BATCH["count"])
    pts = [cloud_points(sp) for sp in specs]
    note(f"batch64: N total {sum(p.shape[1] for p in pts)}")
    kw = dict(order=BATCH["order"], c=BATCH["c"], max_depth=BATCH["max_depth"],
              precision=apc.APC_MIXED)
    xs = [torch.from_numpy(p).cuda() for p in pts]
    B = apc.Batch(xs, **kw)
    B.assemble_gfd()
    _, rho_t, std = B.deposit(tol=1e-10, maxit=4000)
    assert all(s["status"] == 0 for s in std)
    phi, st = B.solve(rho_t, tol=1e-8)
    assert all(s["status"] == 0 and s["rel_resid_true"] <= 1e-8 for s in st)
    note(f"batch64: n total {B.n}, iters {min(s['iters'] for s in st)}..{max(s['iters'] for s in st)}")
    for c in (int(np.argmin(B.cloud_n)), int(np.argmax(B.cloud_n))):
        S = apc.Cloud(xs[c], **kw)
        S.assemble_gfd()
        idx = torch.from_numpy(B.node_index(c)).cuda()
        phi1, st1 = S.solve(rho_t[idx][:S.n].contiguous(), tol=1e-8)
        d = (phi[idx] - phi1).abs().max().item()
        assert d <= 1e-4 * phi1.abs().max().item()
        S.close()
    B.close()
