"""The paper's 3-D beam-with-halo benchmark (Sec. 5.2, Table 3D_ap_cloud) on the GPU.

1e6 particles of the beam (workloads.paper_beam_3d) in Omega = [-1, 1]^3, the
benchmark solution (oracle/beam_exact.py, pinned on the CPU) as Dirichlet data on
the boundary nodes, and the root-mean-square errors of phi and phi_x at the
particles against it, for clouds of about the sizes in the paper's table:

* the whole GPU chain reproduces the oracle's errors on the same particles (both
  discretise identically, so the errors agree to the solver tolerances);
* the errors fall as the cloud is refined, and phi_x stays within a factor 2 of the
  paper's table at the same node count (log-log interpolation of its rows);
  phi within a factor 4 (at 3.7e3 nodes our phi error is 3.3x the table's; from
  1.4e4 nodes on they agree within 1.6x);
* the mixed mode (FP32 weights) gives the same errors.
The errors are printed as a table.
"""
import os
import sys

import numpy as np
import pytest

from workloads import BEAM3D, paper_beam_3d

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "beam3d_sec5_2.txt")
PRM = dict(order=2, max_depth=10, lo=BEAM3D["lo"], L=BEAM3D["L"])
CS = (1.0, 0.3, 0.15, 0.1)


def note(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def table_rows():
    rows = []
    for line in open(GOLDEN):
        f = line.split()
        if f and f[0] == "row":
            rows.append(tuple(float(x) for x in f[1:]))
    return np.array(rows)


def paper_at(n, col):
    """log-log interpolation (or end-segment extrapolation) of a table column at n."""
    t = table_rows()
    ln, le = np.log(t[:, 0]), np.log(t[:, col])
    k = int(np.clip(np.searchsorted(ln, np.log(n)) - 1, 0, len(ln) - 2))
    s = (le[k + 1] - le[k]) / (ln[k + 1] - ln[k])
    return float(np.exp(le[k] + s * (np.log(n) - ln[k])))


@pytest.fixture(scope="module")
def apc():
    from paper_1603_04039_amd import apcloud
    apcloud.load_library()
    assert torch.cuda.is_available()
    return apcloud


@pytest.fixture(scope="module")
def beam():
    from oracle import beam_exact as B
    xyz = paper_beam_3d(1_000_000, seed=1)
    return xyz, B, B.potential(xyz), B.gradient(xyz)


def gpu_errors(apc, beam, c, precision):
    xyz, B, phi_ex, grad_ex = beam
    cl = apc.Cloud(torch.from_numpy(xyz).cuda(), c=c, precision=precision, **PRM)
    cl.assemble_gfd()
    g = B.potential(cl.positions()[:, cl.n:])
    _, rho_t, _ = cl.deposit(tol=1e-12, maxit=20000)
    phi, st = cl.solve(rho_t[:cl.n].contiguous(), torch.from_numpy(g).cuda(), tol=1e-10)
    pp, gp = cl.interpolate_force(phi)
    torch.cuda.synchronize()
    assert st["status"] == 0
    pp, gp = pp.cpu().numpy(), gp.cpu().numpy()
    n = cl.n
    cl.close()
    e_phi = float(np.sqrt(np.mean((pp - phi_ex) ** 2)))
    e_x = float(np.sqrt(np.mean((gp[0] - grad_ex[0]) ** 2)))
    return n, e_phi, e_x


def test_beam_errors_match_oracle(apc, oracle_mod, beam):
    xyz, B, phi_ex, grad_ex = beam
    for c in (1.0, 0.3):
        note(f"beam3d c={c}: GPU vs oracle errors")
        n, e_phi, e_x = gpu_errors(apc, beam, c, apc.APC_FP64)
        O = oracle_mod.OracleCloud(xyz, c=c, **PRM)
        assert O.n == n
        g = B.potential(O.positions()[:, O.n:])
        rt, _ = O.density_solve(O.deposit(), tol=1e-12)
        phi, _ = O.poisson_solve(rt[:O.n], g, tol=1e-10, precond=1)
        pp, gp = O.interpolate(phi)
        o_phi = float(np.sqrt(np.mean((pp - phi_ex) ** 2)))
        o_x = float(np.sqrt(np.mean((gp[0] - grad_ex[0]) ** 2)))
        note(f"  n={n}: phi {e_phi:.4g} (oracle {o_phi:.4g}), phi_x {e_x:.4g} (oracle {o_x:.4g})")
        assert e_phi == pytest.approx(o_phi, rel=1e-3)
        assert e_x == pytest.approx(o_x, rel=1e-3)


def test_beam_convergence_against_table(apc, beam):
    rows = []
    for c in CS:
        note(f"beam3d c={c}")
        n, e_phi, e_x = gpu_errors(apc, beam, c, apc.APC_FP64)
        _, m_phi, m_x = gpu_errors(apc, beam, c, apc.APC_MIXED)
        rows.append((n, e_phi, e_x, paper_at(n, 2), paper_at(n, 3), m_phi, m_x))
    note("     n   err phi  (paper)   err phi_x  (paper)   mixed: phi, phi_x")
    for n, e_phi, e_x, p_phi, p_x, m_phi, m_x in rows:
        note(f"{n:6d}  {e_phi:8.4g} ({p_phi:7.3g})  {e_x:8.4g} ({p_x:7.3g})   {m_phi:.4g}, {m_x:.4g}")
    ns = [r[0] for r in rows]
    assert ns == sorted(ns) and ns[0] > 1000 and ns[-1] > 40_000
    for k in range(1, len(rows)):
        assert rows[k][1] < rows[k - 1][1] and rows[k][2] < rows[k - 1][2]
    for n, e_phi, e_x, p_phi, p_x, m_phi, m_x in rows:
        assert 0.5 * p_x <= e_x <= 2.0 * p_x
        assert 0.25 * p_phi <= e_phi <= 4.0 * p_phi
        # FP32 weights change the operator by ~1e-7 relative: far below the
        # discretisation error at these sizes
        assert m_phi == pytest.approx(e_phi, rel=5e-2) and m_x == pytest.approx(e_x, rel=5e-2)
