"""The tiers of the order-2 stencil search (GPU, via the C ABI).

Rings of up to 63 candidates are searched by one wavefront per node and rings of
up to 255 by one block per node, both in LDS; the rest, and every order-4 ring,
by one thread per node.  The tiers only change where the search runs: clouds built
with every ring per thread (ring_lds = -1), with the wavefront tier only (1) and
with both LDS tiers (0, the default) must agree bit for bit in every array of the
node cloud.  The default is the one the oracle parity tests check.
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


CASES = {
    "beam_halo_1e5": (lambda: beam_halo(100_000, seed=1), dict(order=2, c=0.35, max_depth=6)),
    "beam_halo_1e5_deep": (lambda: beam_halo(100_000, seed=2, sigma=(0.02, 0.05, 0.1)),
                           dict(order=2, c=0.05, max_depth=10)),
    "beam_halo_k4_3e4": (lambda: beam_halo(CONFIGS["beam_halo_k4_3e4"]["N"],
                                           seed=CONFIGS["beam_halo_k4_3e4"]["seed"],
                                           sigma=CONFIGS["beam_halo_k4_3e4"]["sigma"],
                                           halo_frac=CONFIGS["beam_halo_k4_3e4"]["halo_frac"]),
                         dict(order=4, c=CONFIGS["beam_halo_k4_3e4"]["c"],
                              max_depth=CONFIGS["beam_halo_k4_3e4"]["max_depth"])),
    "lattice5": (lambda: uniform_lattice_points(5), dict(order=2, c=1e-3, max_depth=5)),
}


@pytest.mark.parametrize("case", list(CASES))
def test_ring_search_tiers_agree(apc, case):
    gen, kw = CASES[case]
    xyz = torch.from_numpy(gen()).cuda()
    out = {}
    for mode in (0, 1, -1):
        note(f"ring search tiers: {case} ring_lds={mode}")
        cl = apc.Cloud(xyz, ring_lds=mode, **kw)
        out[mode] = (cl.n, cl.nb, cl.nnz, cl.nodes(), cl.node_orders())
        cl.close()
    n0, nb0, nnz0, nodes0, ord0 = out[0]
    note(f"  n={n0} nnz={nnz0}")
    for mode in (1, -1):
        n, nb, nnz, nodes, ords = out[mode]
        assert (n, nb, nnz) == (n0, nb0, nnz0)
        for k, v in nodes0.items():
            np.testing.assert_array_equal(nodes[k], v, err_msg=f"{k}: ring_lds={mode}")
        np.testing.assert_array_equal(ords, ord0)


def test_ring_lds_rejects_bad_value(apc):
    xyz = torch.from_numpy(uniform_lattice_points(2)).cuda()
    with pytest.raises(apc.ApcError) as e:
        apc.Cloud(xyz, ring_lds=2, order=2, c=1.0, max_depth=3)
    assert e.value.code == apc.APC_EINVAL


def _deep_points():
    """2,000 copies of one point and 5 uniform points: with c = 1e-3 the point's
    cell is opened down to level 16, while most of the domain stays coarse, so
    candidate rings of coarse nodes span squared distances of 2^32 integer units
    and more (the integer unit is 2^-(max_depth+1) of the domain)."""
    rng = np.random.default_rng(16)
    pt = np.tile(np.array([[0.3], [0.7], [0.55]]), (1, 2000))
    return np.ascontiguousarray(np.concatenate([pt, rng.random((3, 5))], axis=1))


@pytest.mark.parametrize("mode", [0, -1])
def test_deep_tree_max_depth_16(apc, oracle_mod, mode):
    """max_depth 16: the node cloud and the stencils (every ring per thread with
    mode -1) equal the oracle's bit for bit, with candidate squared distances at
    and above 2^32."""
    xyz = _deep_points()
    kw = dict(order=2, c=1e-3, max_depth=16)
    note(f"deep tree: max_depth 16, ring_lds={mode}")
    O = oracle_mod.OracleCloud(xyz, **kw)
    cl = apc.Cloud(torch.from_numpy(xyz).cuda(), ring_lds=mode, **kw)
    nd_o, nd_g = O.nodes(), cl.nodes()
    assert (cl.n, cl.nb, cl.nnz) == (O.n, O.nb, O.nnz)
    assert int(nd_g["level"].max()) == 16
    for k in ("code", "level", "first", "count", "bowner", "bface", "st_off", "st_idx"):
        np.testing.assert_array_equal(nd_o[k].astype(np.int64), nd_g[k].astype(np.int64),
                                      err_msg=k)
    crd = nd_g["ixyz"].astype(np.int64)
    rows = np.repeat(np.arange(cl.n), np.diff(nd_g["st_off"]))
    r2 = ((crd[:, nd_g["st_idx"]] - crd[:, rows]) ** 2).sum(0)
    note(f"  n={cl.n} max stencil r^2 = 2^{np.log2(r2.max()):.1f}")
    assert r2.max() >= 2 ** 32
    cl.close()


@pytest.mark.parametrize("case", ["order2", "order4"])
def test_ring_first_cap_rerun(apc, oracle_mod, case):
    """The per-thread stencil search first runs with a ring capacity per node and
    reruns nodes whose ring is larger with the full capacity.  A first-pass
    capacity below the uniform ring (24 candidates at order 2, 62 at order 4)
    sends almost every node through the rerun; the stencils must still equal the
    oracle's bit for bit."""
    if case == "order2":
        xyz, kw, cap = beam_halo(100_000, seed=1), dict(order=2, c=0.35, max_depth=6), 16
    else:
        xyz, kw, cap = beam_halo(20_000, seed=31), dict(order=4, c=0.05, max_depth=5), 48
    note(f"ring first-pass capacity {cap}: {case}")
    O = oracle_mod.OracleCloud(xyz, **kw)
    cl = apc.Cloud(torch.from_numpy(xyz).cuda(), ring_lds=-1, ring_first_cap=cap, **kw)
    nd_o, nd_g = O.nodes(), cl.nodes()
    assert (cl.n, cl.nb, cl.nnz) == (O.n, O.nb, O.nnz)
    for k in ("st_off", "st_idx", "code", "level"):
        np.testing.assert_array_equal(nd_o[k].astype(np.int64), nd_g[k].astype(np.int64),
                                      err_msg=k)
    np.testing.assert_array_equal(O.node_orders(), cl.node_orders())
    cl.close()
    with pytest.raises(apc.ApcError) as e:
        apc.Cloud(torch.from_numpy(xyz).cuda(), ring_first_cap=-1, **kw)
    assert e.value.code == apc.APC_EINVAL
