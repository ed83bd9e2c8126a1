"""Neighbour staging of the operator kernels (GPU, via the C ABI).

A 64-row slice of the sliced layout can gather its distinct neighbour columns
once into LDS and read every entry from there.  That is a change of data path
only: the operator apply, the learned M apply, the density solve and the Poisson
solves must agree bit for bit between clouds built with staging off
(stage_cap = -1), on for every slice (0, the default) and on for part of the
slices (a cap between).  The parity tests against the oracle run with the
default, so these tests also carry the oracle parity over to the direct path.
"""
import sys

import numpy as np
import pytest

from workloads import CONFIGS, beam_halo, uniform_lattice_points

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


def bits(t):
    return t.detach().cpu().numpy().view(np.uint64)


LATTICE5 = dict(order=2, c=1e-3, max_depth=5)  # a uniform 32^3 grid: nearly all rows uniform
# the same grid at fourth order: 216 boxed slices (complete 4 x 4 x 4 blocks of
# uniform rows), which run from their box staged (tile >= 512) or unstaged
LATTICE5_K4 = dict(order=4, c=1e-3, max_depth=5)


@pytest.mark.parametrize("workload", ["beam_halo_1e5", "beam_halo_k4_3e4", "lattice5",
                                      "lattice5_k4"])
@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_staging_changes_no_result(apc, workload, precision):
    from paper_1603_04039_amd import learned
    cfg = {"lattice5": LATTICE5, "lattice5_k4": LATTICE5_K4}.get(workload) or CONFIGS[workload]
    prec = apc.APC_FP64 if precision == "fp64" else apc.APC_MIXED
    note(f"staging: {workload} {precision}")
    if workload.startswith("lattice5"):
        xyz = uniform_lattice_points(5)
    else:
        xyz = beam_halo(cfg["N"], seed=cfg["seed"], sigma=cfg["sigma"], halo_frac=cfg["halo_frac"])
    xyz_d = torch.from_numpy(xyz).cuda()
    prm = dict(order=cfg["order"], c=cfg["c"], max_depth=cfg["max_depth"], precision=prec)

    def build(cap):
        cl = apc.Cloud(xyz_d, stage_cap=cap, **prm)
        cl.assemble_gfd()
        return cl

    full = build(0)
    if workload == "lattice5_k4":
        assert full.operator_boxes() == 216  # 4 x 4 x 4 blocks with origins 4 .. 24
    info = full.operator_info(staged=True)
    assert info["staged_slices"] > 0 and 0 < info["stage_tile"] <= 1008
    assert info["staged_distinct"] <= info["staged_entries"]
    # a cap at the mean distinct count leaves part of the slices on the direct path
    mid_cap = int(info["staged_distinct"] // info["staged_slices"])
    clouds = {"full": full, "off": build(-1), "part": build(mid_cap)}
    part = clouds["part"].operator_info(staged=True)
    assert 0 < part["staged_slices"] <= info["staged_slices"]
    if not workload.startswith("lattice5"):  # the lattice's slices may all sit at the mean
        assert part["staged_slices"] < info["staged_slices"]
    assert part["stage_tile"] <= mid_cap
    assert clouds["off"].operator_info(staged=True)["staged_slices"] == 0
    note(f"  slices staged: {info['staged_slices']} (default), {part['staged_slices']} "
         f"(cap {mid_cap}); tile {info['stage_tile']} doubles")

    gen = torch.Generator(device="cuda")
    gen.manual_seed(3)
    f = torch.rand(full.n + full.nb, dtype=torch.float64, device="cuda", generator=gen)
    params, _ = learned_params(apc, learned, cfg["order"])
    out = {}
    for name, cl in clouds.items():
        r = {"apply": cl.apply_operator(f)}
        _, rho_t, _ = cl.deposit(tol=1e-10, maxit=20000)
        r["rho_t"] = rho_t
        b = rho_t[:cl.n].contiguous()
        r["phi_jacobi"], _ = cl.solve(b, tol=1e-8, precond=apc.APC_PRECOND_JACOBI)
        cl.set_learned_precond(params, learned.probes(cl))
        r["m_apply"] = cl.apply_precond(f, apc.APC_PRECOND_LEARNED)
        r["phi_learned"], _ = cl.solve(b, tol=1e-8, precond=apc.APC_PRECOND_LEARNED)
        torch.cuda.synchronize()
        out[name] = {k: bits(v) for k, v in r.items()}
    for name in ("off", "part"):
        for k in out["full"]:
            np.testing.assert_array_equal(out[name][k], out["full"][k],
                                          err_msg=f"{k}: {name} vs full staging")
    for cl in clouds.values():
        cl.close()


def learned_params(apc, learned, order):
    P = np.load(learned.params_path(order))
    assert P.size == apc.MLP_NPARAM
    return torch.from_numpy(P).cuda(), order
