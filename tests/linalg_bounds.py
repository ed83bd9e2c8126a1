"""Error bounds for the GPU-vs-oracle solve comparisons (test infrastructure).

For A x = b solved on two sides to relative residuals t1 and t2,
||x1 - x2|| / ||x|| <= kappa_2(A) (t1 + t2).  kappa_2 is estimated here from the
oracle's assembled rows with scipy: power iteration on A^T A for ||A||_2 and on
A^-T A^-1 (through a sparse LU) for ||A^-1||_2.  Power iteration approaches each
norm from below, so the bars built on it carry a safety factor of 2.
"""
import math

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl


def interior_matrix(off, idx, w, diag, n):
    """CSR matrix of the interior rows/columns: diag_i on the diagonal, w_ij at
    interior columns j (boundary columns belong to the right-hand side)."""
    m = np.diff(off)
    rows = np.repeat(np.arange(n), m)
    keep = idx < n
    A = sp.csr_matrix((w[keep], (rows[keep], idx[keep])), shape=(n, n))
    return (A + sp.diags(diag)).tocsr()


def kappa2(A, iters=30, seed=0, direct=True):
    """2-norm condition estimate of the sparse matrix A.  direct=False solves with
    A by BiCGSTAB instead of a sparse LU (for well-conditioned A, such as a
    diagonally dominant density operator)."""
    rng = np.random.default_rng(seed)
    n = A.shape[0]
    x = rng.standard_normal(n)
    s = 1.0
    for _ in range(iters):
        y = A.T @ (A @ x)
        s = np.linalg.norm(y)
        x = y / s
    smax = math.sqrt(s)
    if direct:
        lu = spl.splu(A.tocsc())
        solve = lu.solve
        solve_t = lambda v: lu.solve(v, trans="T")
    else:
        At = A.T.tocsr()

        def _it(M, v):
            out, info = spl.bicgstab(M, v, rtol=1e-12, atol=0.0, maxiter=2000)
            assert info == 0
            return out
        solve = lambda v: _it(A, v)
        solve_t = lambda v: _it(At, v)
    x = rng.standard_normal(n)
    for _ in range(iters):
        y = solve_t(solve(x))
        s = np.linalg.norm(y)
        x = y / s
    smin = 1.0 / math.sqrt(s)
    return smax / smin


def solve_bar(kappa, t1, t2, cap=None):
    """Relative 2-norm bar for the difference of two solutions."""
    bar = 2.0 * kappa * (t1 + t2)
    return bar if cap is None else min(bar, cap)


def moment_row(X, hc, hp, al):
    """Density row b = sum_alpha a_alpha X_alpha / h^|alpha| with the NGP cell
    moments a_alpha = prod_d (hc/2)^a_d / ((a_d + 1) a_d!) for even alpha, 0 else
    (eq. density_apcloud with the cell's characteristic function)."""
    b = np.zeros(X.shape[1])
    for i, a in enumerate(np.asarray(al).tolist()):
        if any(e % 2 for e in a):
            continue
        mom = np.prod([(hc / 2) ** e / ((e + 1) * math.factorial(e)) for e in a])
        b += mom / hp ** sum(a) * X[i]
    return b


def row_ok(b, theta=0.5):
    """Density-row stability bound sum_j |b_j| <= theta (1 - sum_j b_j)."""
    return np.abs(b).sum() <= theta * (1.0 - b.sum())
