"""Vlasov-Poisson time loop (GPU, via the C ABI) against the oracle.

* apc_push: leapfrog kick-drift with specular walls, bit for bit against the
  oracle's push on the same inputs (ragged sizes, a non-unit domain, particles
  that cross several walls in one step);
* apc_step: one whole step (build, assemble, deposit, solve, interpolate, push)
  against the oracle's verbs chained on the same particles: the node cloud's sizes
  exactly, the field at the particles within the end-to-end chain's bar, and the
  pushed state bit for bit against the oracle's push fed the step's own field;
* the single-test-particle trajectory of the self-force test (Sec. 5): a sharp
  Gaussian cloud crossing cell boundaries for several steps, GPU and oracle each
  advancing their own state; clouds equal in size every step, trajectories
  within the Krylov tolerances.
"""
import sys

import numpy as np
import pytest

from workloads import beam_halo, gaussian_blob

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

P1 = dict(order=2, c=0.35, max_depth=6)


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


@pytest.mark.parametrize("N", [0, 1, 63, 100_003])
def test_push_bit_exact(apc, oracle_mod, N):
    note(f"push parity N={N}")
    lo, L = (-0.5, 0.25, 1.0), 1.5
    rng = np.random.default_rng(N + 7)
    x = np.array(lo)[:, None] + L * rng.random((3, N))
    v = rng.standard_normal((3, N))
    v[:, : N // 3] *= 8 * L  # these cross one or several walls
    g = rng.standard_normal((3, N))
    if N > 4:
        x[0, 0], x[1, 1], x[2, 2] = lo[0], lo[1] + L, lo[2]  # on a face
    kick, dt = 0.0125, 0.7
    xg, vg = cuda(x), cuda(v)
    apc.push(xg, vg, cuda(g), kick, dt, lo=lo, L=L)
    torch.cuda.synchronize()
    xo, vo = oracle_mod.push(x, v, g, kick, dt, lo, L)
    np.testing.assert_array_equal(bits(xg.cpu().numpy()), bits(xo))
    np.testing.assert_array_equal(bits(vg.cpu().numpy()), bits(vo))
    if N:
        xs = xg.cpu().numpy()
        for d in range(3):
            assert xs[d].min() >= lo[d] and xs[d].max() <= lo[d] + L


def test_push_rejects_bad_arguments(apc):
    x = torch.zeros((3, 4), dtype=torch.float64, device="cuda")
    for kick, dt, L in [(float("nan"), 1.0, 1.0), (1.0, float("inf"), 1.0), (1.0, 1.0, 0.0)]:
        with pytest.raises(apc.ApcError) as e:
            apc.push(x, x.clone(), x.clone(), kick, dt, L=L)
        assert e.value.code == apc.APC_EINVAL


def oracle_step(oracle_mod, x, v, kick, dt, tol_density, tol, params):
    """The oracle's verbs chained in the order of one time step."""
    O = oracle_mod.OracleCloud(x, **params)
    rt, _ = O.density_solve(O.deposit(), tol=tol_density, maxit=20000)
    phi, _ = O.poisson_solve(rt[:O.n], tol=tol, maxit=20000, precond=1)
    pp, gp = O.interpolate(phi)
    x1, v1 = oracle_mod.push(x, v, gp, kick, dt, O.lo, O.L)
    return O, pp, gp, x1, v1


def test_step_against_oracle_chain(apc, oracle_mod):
    note("one time step, beam_halo_1e5 (seed 1)")
    x = beam_halo(100_000, seed=1)
    v = 0.1 * np.random.default_rng(2).standard_normal(x.shape)
    kick, dt = 2e-3, 1e-2
    xg, vg = cuda(x), cuda(v)
    pp, gp, st = apc.step(xg, vg, kick, dt, tol_density=1e-13, tol=1e-12, **P1)
    torch.cuda.synchronize()
    note(f"  n={st['n']} iters={st['iters']} density_iters={st['density_iters']} ms={st['ms']}")
    assert st["rc"] == apc.APC_OK and st["status"] == apc.APC_OK
    assert st["rel_resid_true"] <= 1e-12
    O, pp_o, gp_o, _, _ = oracle_step(oracle_mod, x, v, kick, dt, 1e-13, 1e-12, P1)
    assert (st["n"], st["nb"], st["nnz"]) == (O.n, O.nb, O.nnz)
    pp, gp = pp.cpu().numpy(), gp.cpu().numpy()
    assert np.linalg.norm(pp - pp_o) <= 1e-8 * np.linalg.norm(pp_o)
    assert np.linalg.norm(gp - gp_o) <= 1e-7 * np.linalg.norm(gp_o)
    # the push inside the step is the oracle's push of the step's own field
    x1, v1 = oracle_mod.push(x, v, gp, kick, dt)
    np.testing.assert_array_equal(bits(xg.cpu().numpy()), bits(x1))
    np.testing.assert_array_equal(bits(vg.cpu().numpy()), bits(v1))
    assert all(t >= 0.0 for t in st["ms"].values())


def test_step_rejects_learned_and_bad_input(apc):
    x = cuda(beam_halo(1000, seed=3))
    v = torch.zeros_like(x)
    with pytest.raises(apc.ApcError) as e:
        apc.step(x, v, 1e-3, 1e-3, precond=apc.APC_PRECOND_LEARNED, **P1)
    assert e.value.code == apc.APC_EINVAL
    x_bad = x.clone()
    x_bad[0, 5] = 1.5  # outside the unit cube: the build rejects it, nothing moves
    v0 = v.clone()
    with pytest.raises(apc.ApcError) as e:
        apc.step(x_bad, v, 1e-3, 1e-3, **P1)
    assert e.value.code == apc.APC_EDOMAIN
    assert torch.equal(v, v0)


def test_single_particle_trajectory(apc, oracle_mod):
    """A sharp Gaussian test particle (20,000 points, sigma 0.03) moving along x
    through cell boundaries of the cloud that refines towards it, 8 steps."""
    prm = dict(order=2, c=0.35, max_depth=7)
    x, v = gaussian_blob(20_000, seed=5)
    kick, dt, K = 1e-4, 1e-2, 8
    xg, vg = cuda(x), cuda(v)
    xo, vo = x.copy(), v.copy()
    for k in range(K):
        note(f"trajectory step {k}")
        _, gp, st = apc.step(xg, vg, kick, dt, tol_density=1e-13, tol=1e-11, **prm)
        O, _, gp_o, xo, vo = oracle_step(oracle_mod, xo, vo, kick, dt, 1e-13, 1e-11, prm)
        assert st["status"] == apc.APC_OK
        assert (st["n"], st["nb"], st["nnz"]) == (O.n, O.nb, O.nnz)
        g = gp.cpu().numpy()
        assert np.linalg.norm(g - gp_o) <= 1e-6 * np.linalg.norm(gp_o)
    xs, vs = xg.cpu().numpy(), vg.cpu().numpy()
    # each step's field differs by ~1e-9 relative; positions by far less
    assert np.max(np.abs(xs - xo)) <= 1e-10
    assert np.max(np.abs(vs - vo)) <= 1e-8
    # the centroid moved with the blob's velocity (the self-force is small)
    drift = xs.mean(axis=1) - x.mean(axis=1)
    np.testing.assert_allclose(drift, K * dt * v.mean(axis=1), atol=1e-4)


def test_step_order4_against_oracle_chain(apc, oracle_mod):
    """One fourth-order time step (20,000 particles, 9,332 nodes), FP64, against the
    oracle's verbs chained: cloud sizes exact, the field within the fourth-order
    chain's bar, the push bit for bit given the step's field."""
    note("one fourth-order time step")
    prm = dict(order=4, c=0.05, max_depth=5)
    x = beam_halo(20_000, seed=31)
    v = 0.1 * np.random.default_rng(5).standard_normal(x.shape)
    kick, dt = 1e-3, 1e-2
    xg, vg = cuda(x), cuda(v)
    pp, gp, st = apc.step(xg, vg, kick, dt, tol_density=1e-13, tol=1e-12, maxit=20000,
                          precision=apc.APC_FP64, **prm)
    torch.cuda.synchronize()
    note(f"  n={st['n']} iters={st['iters']} density_iters={st['density_iters']}")
    assert st["status"] == apc.APC_OK
    O, pp_o, gp_o, _, _ = oracle_step(oracle_mod, x, v, kick, dt, 1e-13, 1e-12, prm)
    assert (st["n"], st["nb"], st["nnz"]) == (O.n, O.nb, O.nnz)
    pp, gp = pp.cpu().numpy(), gp.cpu().numpy()
    assert np.linalg.norm(pp - pp_o) <= 1e-7 * np.linalg.norm(pp_o)
    assert np.linalg.norm(gp - gp_o) <= 1e-6 * np.linalg.norm(gp_o)
    x1, v1 = oracle_mod.push(x, v, gp, kick, dt)
    np.testing.assert_array_equal(bits(xg.cpu().numpy()), bits(x1))
    np.testing.assert_array_equal(bits(vg.cpu().numpy()), bits(v1))
