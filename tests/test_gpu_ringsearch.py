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
