"""apc_interpolate_force_noalloc (GPU, via the C ABI): the entry point for callers
that cannot allocate keeps its derivative buffer in a fixed device array.  Its
outputs must equal apc_interpolate_force's bit for bit (same kernels), on two
calls in a row with the second cloud smaller than the first (the array keeps the
first call's contents), for k = 2 and k = 4; a cloud whose n x p derivatives
exceed the array is rejected with APC_EINVAL."""
import sys

import numpy as np
import pytest

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


def _run(apc, xyz, kw, seed):
    cl = apc.Cloud(torch.from_numpy(np.ascontiguousarray(xyz)).cuda(), **kw)
    phi = torch.from_numpy(np.random.default_rng(seed).standard_normal(cl.n + cl.nb)).cuda()
    pp_ref, gp_ref = cl.interpolate_force(phi)
    pp = torch.full((cl.N,), np.nan, dtype=torch.float64, device="cuda")
    gp = torch.full((3, cl.N), np.nan, dtype=torch.float64, device="cuda")
    cl.interpolate_force_noalloc(phi, pp, gp)
    torch.cuda.synchronize()
    out = (cl.n, pp.cpu().numpy(), gp.cpu().numpy(), pp_ref.cpu().numpy(), gp_ref.cpu().numpy())
    cl.close()
    return out


@pytest.mark.parametrize("order", [2, 4])
def test_noalloc_interpolation_matches(apc, order):
    if order == 2:
        big, small = beam_halo(200_000, seed=41), beam_halo(30_000, seed=42)
        kw = dict(order=2, c=0.3, max_depth=7)
    else:
        big, small = beam_halo(50_000, seed=32), beam_halo(20_000, seed=31)
        kw = dict(order=4, c=0.05, max_depth=6)
    sizes = []
    for i, xyz in enumerate((big, small)):
        note(f"noalloc interpolation: order {order}, call {i + 1}, N={xyz.shape[1]}")
        n, pp, gp, pp_ref, gp_ref = _run(apc, xyz, kw, seed=i)
        sizes.append(n)
        np.testing.assert_array_equal(pp, pp_ref)
        np.testing.assert_array_equal(gp, gp_ref)
    assert sizes[1] < sizes[0]


def test_noalloc_rejects_oversized_cloud(apc):
    """A 128^3 lattice (2,097,152 nodes, 151 MB of k = 2 derivatives) exceeds the
    32 MiB array."""
    xyz = torch.from_numpy(uniform_lattice_points(7)).cuda()
    cl = apc.Cloud(xyz, order=2, c=1e-3, max_depth=7)
    assert cl.n * 9 * 8 > apc.APC_NOALLOC_BYTES
    phi = torch.zeros(cl.n + cl.nb, dtype=torch.float64, device="cuda")
    pp = torch.empty(cl.N, dtype=torch.float64, device="cuda")
    gp = torch.empty((3, cl.N), dtype=torch.float64, device="cuda")
    with pytest.raises(apc.ApcError) as e:
        cl.interpolate_force_noalloc(phi, pp, gp)
    assert e.value.code == apc.APC_EINVAL and "APC_NOALLOC_BYTES" in str(e.value)
    cl.close()
