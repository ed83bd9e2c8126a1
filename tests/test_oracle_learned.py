"""Pins of the oracle's learned-preconditioner data and gradients (CPU only).

The learned preconditioner is not part of the paper's method: row i of M has
the pattern {i} + the stencil of row i, m_i = (e_0 + o_i) / d_i, and the
per-row loss is the left approximate-inverse residual ||m_i^T A - e_i^T||^2
estimated from probe vectors.  Expected values here come from a dense matrix
built out of the assembled rows, from the zero row sums of the operator
(Sec. 3.2: a constant has zero Laplacian) and from central differences; none
re-calls the routine under test to make them.
"""
import numpy as np
import pytest

from workloads import beam_halo


@pytest.fixture(scope="module")
def small_cloud(oracle_mod):
    xyz = beam_halo(3000, seed=21)
    return oracle_mod.OracleCloud(xyz, order=2, c=0.45, max_depth=5)


def _dense_interior(C):
    w, d = C.assemble()
    nd = C.nodes()
    off, idx = nd["st_off"], nd["st_idx"]
    A = np.diag(d)
    for i in range(C.n):
        for e in range(off[i], off[i + 1]):
            if idx[e] < C.n:
                A[i, idx[e]] += w[e]
    return A, w, d, off, idx


NOUT, NQ = 41, 41 * 42 // 2 + 41 + 1


def test_features_row_sums(oracle_mod, small_cloud):
    """The operator's rows sum to zero (the fit reproduces constants exactly), so
    the 40 weight features of a row sum to -d_i/|d_i| = 1 in magnitude.  The
    structural features, counted here from the node list: level differences to
    the first 6 stencil nodes (2:1 balance keeps face neighbours within one
    level), the stencil size m / 40, the boundary fraction of the stencil."""
    C = small_cloud
    feat, _ = C.learn_data()
    nd = C.nodes()
    off, idx, lev = nd["st_off"], nd["st_idx"], nd["level"]
    m = np.diff(off)
    assert m.max() <= 40
    np.testing.assert_allclose(np.abs(feat[:, :40].sum(axis=1)), 1.0, atol=1e-10)
    for i in range(C.n):
        nbrs = idx[off[i]:off[i + 1]]
        for k in range(6):
            v = nbrs[k]
            assert feat[i, 40 + k] == (lev[v] - lev[i] if v < C.n else 0)
        assert feat[i, 47] == pytest.approx(np.mean(nbrs >= C.n), abs=1e-15)
        assert np.all(feat[i, m[i]:40] == 0.0)
    np.testing.assert_array_equal(feat[:, 46], m / 40.0)
    assert feat[:, 47].max() > 0.0 and np.all(np.abs(feat[:, 40:46]) <= 2)


def test_quadratic_data_with_identity_probes(oracle_mod, small_cloud):
    """With the n unit vectors as probes, the per-row quadratic equals
    ||m_i^T A - e_i^T||^2 / n exactly, for any m_i on the pattern."""
    C = small_cloud
    n, ntot = C.n, C.n + C.nb
    Z = np.zeros((n, ntot))
    Z[np.arange(n), np.arange(n)] = 1.0
    feat, quad = C.learn_data(Z)
    A, w, d, off, idx = _dense_interior(C)
    rng = np.random.default_rng(5)
    for i in rng.choice(n, size=25, replace=False):
        J = [i] + list(idx[off[i]:off[i + 1]])
        o = np.zeros(NOUT)
        o[:len(J)] = 0.3 * rng.standard_normal(len(J))
        mt = o.copy()
        mt[0] += 1.0
        mvec = np.zeros(n)
        for p, j in enumerate(J):
            if j < n:
                mvec[j] += mt[p] / d[i]
        r = mvec @ A
        r[i] -= 1.0
        expect = r @ r / n
        Q, bq, cq = unpack(quad[i])
        got = mt @ Q @ mt - 2 * bq @ mt + cq
        assert got == pytest.approx(expect, rel=1e-10, abs=1e-14)
        # entries beyond the row's stencil do not enter the loss
        mt2 = mt.copy()
        mt2[len(J):] = rng.standard_normal(NOUT - len(J))
        assert mt2 @ Q @ mt2 - 2 * bq @ mt2 + cq == pytest.approx(got, rel=1e-12)


def unpack(q):
    Q = np.zeros((NOUT, NOUT))
    t = 0
    for p in range(NOUT):
        for s in range(p + 1):
            Q[p, s] = Q[s, p] = q[t]
            t += 1
    return Q, q[t:t + NOUT], q[t + NOUT]


def test_mlp_gradient_central_differences(oracle_mod):
    """The FP64 back-propagation agrees with central differences of the loss."""
    rng = np.random.default_rng(9)
    P = 0.2 * rng.standard_normal(oracle_mod.MLP_NPARAM)
    nrow = 12
    feat = rng.standard_normal((nrow, 48))
    # per-row quadratic data of a positive semi-definite Q (from random u)
    quad = np.zeros((nrow, NQ))
    nqq = NOUT * (NOUT + 1) // 2
    for r in range(nrow):
        U = rng.standard_normal((NOUT, 5))
        z = rng.standard_normal(5)
        Q = U @ U.T / 5
        quad[r, :nqq] = [Q[p, s] for p in range(NOUT) for s in range(p + 1)]
        quad[r, nqq:nqq + NOUT] = U @ z / 5
        quad[r, -1] = z @ z / 5
    rows = np.array([3, 0, 7, 7, 11, 5], dtype=np.int32)
    L0, g = oracle_mod.mlp_loss_grad(P, feat, quad, rows)
    idx = rng.choice(P.size, size=120, replace=False)
    # always include the output layer and the first-layer biases
    idx = np.unique(np.concatenate([idx, np.arange(P.size - NOUT, P.size), [48 * 64 + 3]]))
    eps = 1e-6
    for k in idx:
        Pp = P.copy()
        Pm = P.copy()
        Pp[k] += eps
        Pm[k] -= eps
        fd = (oracle_mod.mlp_loss_grad(Pp, feat, quad, rows)[0]
              - oracle_mod.mlp_loss_grad(Pm, feat, quad, rows)[0]) / (2 * eps)
        assert g[k] == pytest.approx(fd, rel=1e-6, abs=1e-8 * max(1.0, abs(L0)))


def test_mlp_zero_network_is_jacobi(oracle_mod):
    """All-zero parameters give o = 0, i.e. Jacobi: the loss is the mean of
    Q_00 - 2 b_0 + c and the gradient reaches only the output bias."""
    rng = np.random.default_rng(3)
    feat = rng.standard_normal((4, 48))
    quad = rng.standard_normal((4, NQ))
    rows = np.arange(4, dtype=np.int32)
    L, g = oracle_mod.mlp_loss_grad(np.zeros(oracle_mod.MLP_NPARAM), feat, quad, rows)
    nqq = NOUT * (NOUT + 1) // 2
    assert L == pytest.approx(np.mean(quad[:, 0] - 2 * quad[:, nqq] + quad[:, -1]), rel=1e-14)
    assert np.all(g[:-NOUT] == 0.0)
    # dL/db3_p = mean over rows of 2 (Q e_0 - b)_p; Q_p0 sits at p (p + 1) / 2
    Qe0 = np.stack([quad[:, p * (p + 1) // 2] for p in range(NOUT)], axis=1)
    np.testing.assert_allclose(g[-NOUT:], np.mean(2 * (Qe0 - quad[:, nqq:nqq + NOUT]), axis=0),
                               rtol=1e-12)


def test_mlp_forward_identity_layers(oracle_mod):
    """Layout pin: with W1 = [I_48 | 0], W2 = I_64 and zero hidden biases, a
    non-negative input passes both ReLU layers unchanged, so o = W3[:48]^T x + b3."""
    rng = np.random.default_rng(4)
    IN, H, O = 48, 64, NOUT
    W1 = np.zeros((IN, H))
    W1[np.arange(IN), np.arange(IN)] = 1.0
    W2 = np.eye(H)
    W3 = rng.standard_normal((H, O))
    b3 = rng.standard_normal(O)
    P = np.concatenate([W1.ravel(), np.zeros(H), W2.ravel(), np.zeros(H), W3.ravel(), b3])
    x = np.abs(rng.standard_normal((5, IN)))
    np.testing.assert_allclose(oracle_mod.mlp_forward(P, x), x @ W3[:IN] + b3, rtol=1e-13)
    # a negative first-layer pre-activation is cut by the ReLU
    x2 = x.copy()
    x2[:, 0] = -1.0
    np.testing.assert_allclose(oracle_mod.mlp_forward(P, x2), x2[:, 1:] @ W3[1:IN] + b3,
                               rtol=1e-13)


def test_mlp_loss_consistent_with_forward(oracle_mod):
    """The loss of the gradient routine equals the quadratic of the rows evaluated
    at the forward output."""
    rng = np.random.default_rng(8)
    P = 0.1 * rng.standard_normal(oracle_mod.MLP_NPARAM)
    feat = rng.standard_normal((6, 48))
    quad = rng.standard_normal((6, NQ))
    rows = np.array([5, 1, 1, 0], dtype=np.int32)
    L, _ = oracle_mod.mlp_loss_grad(P, feat, quad, rows)
    o = oracle_mod.mlp_forward(P, feat)
    tot = 0.0
    for r in rows:
        m = o[r].copy()
        m[0] += 1.0
        Q, bq, cq = unpack(quad[r])
        tot += m @ Q @ m - 2 * bq @ m + cq
    assert L == pytest.approx(tot / rows.size, rel=1e-12)


def _probe_losses(C, w, d, off, idx, Z, mdiag, mw):
    """Per-row probe estimate sum_k (m_i^T A z_k - z_ki)^2, with A z computed here."""
    n = C.n
    import scipy.sparse as sp
    rows = np.repeat(np.arange(n), np.diff(off))
    keep = idx < n
    A = sp.csr_matrix((np.concatenate([d, w[keep]]),
                       (np.concatenate([np.arange(n), rows[keep]]),
                        np.concatenate([np.arange(n), idx[keep]]))), shape=(n, n))
    M = sp.csr_matrix((np.concatenate([mdiag, mw[keep]]),
                       (np.concatenate([np.arange(n), rows[keep]]),
                        np.concatenate([np.arange(n), idx[keep]]))), shape=(n, n))
    Zi = Z[:, :n].T
    R = M @ (A @ Zi) - Zi
    return (R * R).sum(axis=1)


def test_learned_m_zero_network_is_jacobi(oracle_mod, small_cloud):
    C = small_cloud
    _, d = C.assemble()
    Z = np.random.default_rng(2).standard_normal((4, C.n + C.nb))
    for z in (None, Z):
        md, mw = C.learned_m(np.zeros(oracle_mod.MLP_NPARAM), z)
        np.testing.assert_allclose(md, 1.0 / d, rtol=1e-15)
        assert np.all(mw == 0.0)


def test_learned_m_safeguard_minimises_probe_loss(oracle_mod, small_cloud):
    """The safeguarded row is the best point of the segment from the Jacobi row to
    the network's row under the probe loss: never worse than either end."""
    C = small_cloud
    w, d = C.assemble()
    nd = C.nodes()
    off, idx = nd["st_off"], nd["st_idx"]
    rng = np.random.default_rng(6)
    P = 0.3 * rng.standard_normal(oracle_mod.MLP_NPARAM)
    Z = rng.standard_normal((6, C.n + C.nb))
    md0, mw0 = C.learned_m(P)
    md1, mw1 = C.learned_m(P, Z)
    Lj = _probe_losses(C, w, d, off, idx, Z, 1.0 / d, np.zeros_like(w))
    L0 = _probe_losses(C, w, d, off, idx, Z, md0, mw0)
    L1 = _probe_losses(C, w, d, off, idx, Z, md1, mw1)
    tol = 1e-9 * (Lj + L0)
    assert np.all(L1 <= np.minimum(Lj, L0) + tol)
    # with random weights most rows are pulled back, some all the way to Jacobi
    changed = np.abs(md1 - md0) > 1e-12 * np.abs(md0)
    assert changed.mean() > 0.5
    # every row lies on the segment: m1 - j = alpha (m0 - j) with one alpha per row
    for i in np.where(changed)[0][:50]:
        a = (md1[i] - 1.0 / d[i]) / (md0[i] - 1.0 / d[i])
        assert -1e-12 <= a <= 1.0 + 1e-12
        np.testing.assert_allclose(mw1[off[i]:off[i + 1]], a * mw0[off[i]:off[i + 1]],
                                   rtol=1e-12, atol=1e-300)


def test_learned_m_uniform_rows(oracle_mod):
    """On a uniform lattice the interior rows two cells away from the boundary
    have the uniform 2-ring stencil and identical features: the network gives
    them all the same scaled row.  The safeguard treats them like every other
    row: each moves along its own segment towards the Jacobi row, never worse
    than either end under its probe loss."""
    from workloads import uniform_lattice_points
    C = oracle_mod.OracleCloud(uniform_lattice_points(4), order=2, c=1e-3, max_depth=4)
    rng = np.random.default_rng(7)
    P = 0.3 * rng.standard_normal(oracle_mod.MLP_NPARAM)
    Z = rng.standard_normal((4, C.n + C.nb))
    md0, mw0 = C.learned_m(P)
    md1, mw1 = C.learned_m(P, Z)
    ix = C.coords()[:, :C.n]
    sp = 2  # cell size of level 4 in units of 2^-(max_depth+1)
    lo, hi = ix.min(axis=1), ix.max(axis=1)
    inner = np.all((ix >= lo[:, None] + 2 * sp) & (ix <= hi[:, None] - 2 * sp), axis=0)
    assert inner.sum() == 12 ** 3  # nodes 2..13 of 0..15 along each axis
    w, d = C.assemble()
    scaled = md0[inner] * d[inner]
    np.testing.assert_allclose(scaled, scaled[0], rtol=1e-12)
    nd = C.nodes()
    off, idx = nd["st_off"], nd["st_idx"]
    Lj = _probe_losses(C, w, d, off, idx, Z, 1.0 / d, np.zeros_like(w))
    L0 = _probe_losses(C, w, d, off, idx, Z, md0, mw0)
    L1 = _probe_losses(C, w, d, off, idx, Z, md1, mw1)
    assert np.all(L1[inner] <= np.minimum(Lj, L0)[inner] + 1e-9 * (Lj + L0)[inner])
    a = (md1 - 1.0 / d) / (md0 - 1.0 / d)
    assert np.all((a[inner] >= -1e-12) & (a[inner] <= 1.0 + 1e-12))
    assert np.unique(np.round(a[inner], 12)).size > 1  # alpha is per row


# ---------------------------------------------------------------- k = 4
@pytest.fixture(scope="module")
def small_cloud4(oracle_mod):
    xyz = beam_halo(3000, seed=21)
    C = oracle_mod.OracleCloud(xyz, order=4, c=0.05, max_depth=4)
    assert np.diff(C.nodes()["st_off"]).max() > 40
    return C


def test_k4_features_first_40_weights(oracle_mod, small_cloud4):
    """Fourth-order rows hold up to 56 stencil nodes; the weight features are the
    first 40 (the nearest) over |d_i|, the size feature is m / 40 (> 1 here)."""
    C = small_cloud4
    feat, _ = C.learn_data()
    w, d = C.assemble()
    off = C.nodes()["st_off"]
    m = np.diff(off)
    for i in range(C.n):
        k = min(m[i], 40)
        np.testing.assert_allclose(feat[i, :k], w[off[i]:off[i] + k] / abs(d[i]), rtol=1e-15)
        assert np.all(feat[i, k:40] == 0.0)
    np.testing.assert_array_equal(feat[:, 46], m / 40.0)
    assert feat[:, 46].max() > 1.0


def test_k4_quadratic_data_with_identity_probes(oracle_mod, small_cloud4):
    """With the n unit vectors as probes, the per-row quadratic of a fourth-order
    row equals ||m_i^T A - e_i^T||^2 / n exactly for m_i on {i} and the first 40
    stencil nodes; stencil nodes beyond the 40th are not part of M."""
    C = small_cloud4
    n, ntot = C.n, C.n + C.nb
    Z = np.zeros((n, ntot))
    Z[np.arange(n), np.arange(n)] = 1.0
    _, quad = C.learn_data(Z)
    A, w, d, off, idx = _dense_interior(C)
    rng = np.random.default_rng(8)
    long_rows = np.where(np.diff(off) > 40)[0]
    for i in rng.choice(long_rows, size=20, replace=False):
        J = [i] + list(idx[off[i]:off[i] + 40])
        mt = 0.3 * rng.standard_normal(NOUT)
        mt[0] += 1.0
        mvec = np.zeros(n)
        for p, j in enumerate(J):
            if j < n:
                mvec[j] += mt[p] / d[i]
        r = mvec @ A
        r[i] -= 1.0
        Q, bq, cq = unpack(quad[i])
        assert mt @ Q @ mt - 2 * bq @ mt + cq == pytest.approx(r @ r / n, rel=1e-10, abs=1e-14)


def test_k4_learned_m_pattern_and_safeguard(oracle_mod, small_cloud4):
    """Rows of M carry weights on their first 40 stencil nodes only, and the
    safeguard is never worse than either end of its segment (every fourth-order
    row is safeguarded)."""
    C = small_cloud4
    w, d = C.assemble()
    nd = C.nodes()
    off, idx = nd["st_off"], nd["st_idx"]
    rng = np.random.default_rng(9)
    P = 0.3 * rng.standard_normal(oracle_mod.MLP_NPARAM)
    Z = rng.standard_normal((6, C.n + C.nb))
    md0, mw0 = C.learned_m(P)
    pos = np.arange(off[-1]) - np.repeat(off[:-1], np.diff(off))
    assert np.all(mw0[pos >= 40] == 0.0)
    assert np.any(mw0[(pos < 40) & (idx < C.n)] != 0.0)
    md1, mw1 = C.learned_m(P, Z)
    Lj = _probe_losses(C, w, d, off, idx, Z, 1.0 / d, np.zeros_like(w))
    L0 = _probe_losses(C, w, d, off, idx, Z, md0, mw0)
    L1 = _probe_losses(C, w, d, off, idx, Z, md1, mw1)
    assert np.all(L1 <= np.minimum(Lj, L0) + 1e-9 * (Lj + L0))
    assert (np.abs(md1 - md0) > 1e-12 * np.abs(md0)).mean() > 0.5
