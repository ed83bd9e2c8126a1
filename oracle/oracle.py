"""ctypes binding of the C oracle (oracle/apc_oracle.c, and oracle/apc_oracle2d.c for the
two-dimensional variant).  Test infrastructure only."""
from __future__ import annotations

import ctypes as ct
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "apc_oracle.c")
_SRC2 = os.path.join(_HERE, "apc_oracle2d.c")
_LIB = os.path.join(_HERE, "libapc_oracle.so")
_lib = None

ERRORS = {0: "ok", -1: "invalid argument", -2: "out of memory", -4: "particle outside domain",
          -5: "no acceptable stencil", 1: "not converged"}


def build_oracle_lib() -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off",
           "-o", _LIB, _SRC, _SRC2, "-lm"]
    subprocess.run(cmd, check=True)
    return _LIB


class _Params(ct.Structure):
    _fields_ = [("lo", ct.c_double * 3), ("L", ct.c_double), ("order", ct.c_int),
                ("c", ct.c_double), ("max_depth", ct.c_int), ("ring_min", ct.c_int),
                ("ring_max", ct.c_int), ("m_cap", ct.c_int), ("poisson_c", ct.c_double),
                ("criterion_pow", ct.c_int), ("tau_dom", ct.c_double), ("periodic", ct.c_int),
                ("kernel", ct.c_int), ("mask_level", ct.c_int), ("mask", ct.c_void_p)]


class _Stats(ct.Structure):
    _fields_ = [("iters", ct.c_int), ("status", ct.c_int), ("rel_resid", ct.c_double),
                ("rel_resid_true", ct.c_double)]


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < max(os.path.getmtime(_SRC),
                                                                 os.path.getmtime(_SRC2)):
        build_oracle_lib()
    lib = ct.CDLL(_LIB)
    P = ct.c_void_p
    lib.apco_build_cloud.argtypes = [ct.POINTER(_Params), P, ct.c_int64, ct.POINTER(ct.c_void_p)]
    lib.apco_destroy.argtypes = [P]
    lib.apco_destroy.restype = None
    lib.apco_info.argtypes = [P] + [ct.POINTER(ct.c_int64)] * 5
    lib.apco_get_nodes.argtypes = [P] * 11
    lib.apco_node_coords.argtypes = [P, P]
    lib.apco_node_orders.argtypes = [P, P]
    lib.apco_density_orders.argtypes = [P, P]
    lib.apco_get_cells.argtypes = [P] * 5
    lib.apco_ring1.argtypes = [P, P, P, ct.c_int64]
    lib.apco_wls_fit.argtypes = [ct.c_int, ct.c_int, P, P, P, P]
    lib.apco_assemble.argtypes = [P, P, P]
    lib.apco_density_rows.argtypes = [P, P, P]
    lib.apco_deposit.argtypes = [P, P, P]
    lib.apco_deposit_xyz.argtypes = [P, P, P, P]
    lib.apco_kernel_moment.argtypes = [ct.c_int, ct.c_int, ct.c_double, ct.c_double]
    lib.apco_kernel_moment.restype = ct.c_double
    lib.apco_density_solve.argtypes = [P, P, P, ct.c_double, ct.c_int, ct.c_int,
                                       ct.POINTER(_Stats)]
    lib.apco_poisson_solve.argtypes = [P, P, P, P, ct.c_double, ct.c_int, ct.c_int,
                                       ct.POINTER(_Stats)]
    lib.apco_poisson_lu.argtypes = [P, P, P, P]
    lib.apco_bicgstab_rows.argtypes = [P, P, P, P, P, ct.c_double, ct.c_int, ct.c_int,
                                       ct.POINTER(_Stats)]
    lib.apco_apply_laplacian.argtypes = [P, P, P]
    lib.apco_node_derivs.argtypes = [P, P, P]
    lib.apco_interpolate.argtypes = [P, P, P, P, P]
    lib.apco_num_unknowns.argtypes = [ct.c_int]
    lib.apco_monomials.argtypes = [ct.c_int, P]
    lib.apco_thresholds.argtypes = [ct.POINTER(_Params), P]
    lib.apco_learn_data.argtypes = [P, P, ct.c_int, P, P]
    lib.apco_mlp_loss_grad.argtypes = [P, P, P, P, ct.c_int, P, P]
    lib.apco_mlp_forward.argtypes = [P, P, ct.c_int64, P]
    lib.apco_learned_m.argtypes = [P, P, P, ct.c_int, P, P]
    lib.apco2_build_cloud.argtypes = [ct.POINTER(_Params), P, ct.c_int64, ct.POINTER(ct.c_void_p)]
    lib.apco2_destroy.argtypes = [P]
    lib.apco2_destroy.restype = None
    lib.apco2_info.argtypes = [P] + [ct.POINTER(ct.c_int64)] * 4
    lib.apco2_get_nodes.argtypes = [P] * 10
    lib.apco2_node_coords.argtypes = [P, P]
    lib.apco2_ring1.argtypes = [P, P, P, ct.c_int64]
    lib.apco2_assemble.argtypes = [P, P, P]
    lib.apco2_density_rows.argtypes = [P, P, P, P]
    lib.apco2_deposit.argtypes = [P, P, P]
    lib.apco2_density_solve.argtypes = [P, P, P, ct.c_double, ct.c_int, ct.POINTER(_Stats)]
    lib.apco2_poisson_solve.argtypes = [P, P, P, P, ct.c_double, ct.c_int, ct.c_int,
                                        ct.POINTER(_Stats)]
    lib.apco2_node_derivs.argtypes = [P, P, P]
    lib.apco2_interpolate.argtypes = [P, P, P, P, P]
    lib.apco_push.argtypes = [ct.POINTER(_Params), ct.c_int64, P, P, P, ct.c_double,
                              ct.c_double]
    _lib = lib
    return lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ct.c_void_p)


def _check(rc, what):
    if rc < 0:
        raise RuntimeError(f"oracle {what}: {ERRORS.get(rc, rc)} ({rc})")
    return rc


def make_params(order=2, c=0.35, max_depth=6, lo=(0.0, 0.0, 0.0), L=1.0, ring_min=None,
                ring_max=5, m_cap=None, poisson_c=1.0, criterion_pow=0, tau_dom=0.0, periodic=0,
                kernel=0, mask=None):
    """mask: None, or a (s, s, s) boolean array over the cells of the uniform grid of
    level log2(s), indexed [ix, iy, iz]; True excludes the cell from Omega."""
    P = _Params()
    P.lo[:] = lo
    P.L = L
    P.order = order
    P.c = c
    P.max_depth = max_depth
    P.ring_min = ring_min if ring_min is not None else (2 if order == 2 else 3)
    P.ring_max = ring_max
    P.m_cap = m_cap if m_cap is not None else (40 if order == 2 else 56)
    P.poisson_c = poisson_c
    P.criterion_pow = criterion_pow
    P.tau_dom = tau_dom
    P.periodic = int(periodic)
    P.kernel = int(kernel)
    if mask is not None:
        m = np.asarray(mask).astype(np.uint8)
        s = m.shape[0]
        ml = int(s).bit_length() - 1
        assert m.shape == (s, s, s) and (1 << ml) == s
        flat = np.ascontiguousarray(m.transpose(2, 1, 0)).ravel()  # x fastest
        P.mask_level = ml
        P.mask = flat.ctypes.data
        P._mask_ref = flat  # kept alive with the parameters
    return P


KERNEL_NGP, KERNEL_CIC, KERNEL_TSC = 0, 1, 2


def kernel_moment(kernel, k, tlo=-np.inf, thi=np.inf):
    """1-D moment of a charge-assignment kernel over [tlo, thi] (apco_kernel_moment)."""
    return _load().apco_kernel_moment(int(kernel), int(k), float(tlo), float(thi))


def push(xyz, vel, grad, kick, dt, lo=(0.0, 0.0, 0.0), L=1.0, periodic=0):
    """Leapfrog kick-drift push with specular walls, or wrap-around on a periodic
    domain (apco_push).  xyz, vel: 3 x N float64, updated copies are returned;
    grad: 3 x N."""
    x = np.array(xyz, dtype=np.float64, order="C", copy=True)
    v = np.array(vel, dtype=np.float64, order="C", copy=True)
    g = np.ascontiguousarray(grad, dtype=np.float64)
    assert x.shape == v.shape == g.shape and x.shape[0] == 3
    P = make_params(lo=lo, L=L, periodic=periodic)
    _check(_load().apco_push(ct.byref(P), x.shape[1], _ptr(x), _ptr(v), _ptr(g), kick, dt),
           "push")
    return x, v


def num_unknowns(order: int) -> int:
    return _load().apco_num_unknowns(order)


def monomials(order: int) -> np.ndarray:
    p = num_unknowns(order)
    a = np.zeros((p, 3), dtype=np.int32)
    _check(_load().apco_monomials(order, _ptr(a)), "monomials")
    return a


def thresholds(**kw) -> np.ndarray:
    P = make_params(**kw)
    T = np.zeros(P.max_depth + 1)
    _load().apco_thresholds(ct.byref(P), _ptr(T))
    return T


MLP_OUT = 41
LEARN_QUAD = MLP_OUT * (MLP_OUT + 1) // 2 + MLP_OUT + 1
MLP_NPARAM = 48 * 64 + 64 + 64 * 64 + 64 + 64 * MLP_OUT + MLP_OUT


def mlp_loss_grad(params, feat, quad, rows):
    """FP64 mean loss and gradient of the learned-preconditioner network."""
    P = np.ascontiguousarray(params, dtype=np.float64)
    f = np.ascontiguousarray(feat, dtype=np.float64)
    q = np.ascontiguousarray(quad, dtype=np.float64)
    r = np.ascontiguousarray(rows, dtype=np.int32)
    assert P.size == MLP_NPARAM
    g = np.zeros(MLP_NPARAM)
    loss = np.zeros(1)
    _check(_load().apco_mlp_loss_grad(_ptr(P), _ptr(f), _ptr(q), _ptr(r), r.size, _ptr(loss),
                                      _ptr(g)), "mlp_loss_grad")
    return loss[0], g


def mlp_forward(params, feat):
    """FP64 network output (nrow x 41) of the learned-preconditioner network."""
    P = np.ascontiguousarray(params, dtype=np.float64)
    f = np.ascontiguousarray(feat, dtype=np.float64)
    assert P.size == MLP_NPARAM and f.shape[1] == 48
    out = np.zeros((f.shape[0], MLP_OUT))
    _check(_load().apco_mlp_forward(_ptr(P), _ptr(f), f.shape[0], _ptr(out)), "mlp_forward")
    return out


def wls_fit(order: int, delta: np.ndarray):
    """X (p x m), h, R-diagonal ratio for an explicit stencil delta (m x 3)."""
    d = np.ascontiguousarray(delta, dtype=np.float64)
    m = d.shape[0]
    p = num_unknowns(order)
    X = np.zeros((p, m))
    h = ct.c_double()
    r = ct.c_double()
    _check(_load().apco_wls_fit(order, m, _ptr(d), _ptr(X), ct.byref(h), ct.byref(r)), "wls_fit")
    return X, h.value, r.value


class OracleCloud:
    """An oracle node cloud built from particles (3 x N float64)."""

    def __init__(self, xyz: np.ndarray, **params):
        self.lib = _load()
        self.params = make_params(**params)
        self.xyz = np.ascontiguousarray(xyz, dtype=np.float64)
        assert self.xyz.ndim == 2 and self.xyz.shape[0] == 3
        self.N = self.xyz.shape[1]
        h = ct.c_void_p()
        _check(self.lib.apco_build_cloud(ct.byref(self.params), _ptr(self.xyz), self.N,
                                         ct.byref(h)), "build_cloud")
        self.h = h
        v = [ct.c_int64() for _ in range(5)]
        self.lib.apco_info(self.h, *[ct.byref(x) for x in v])
        self.n, self.nb, self.nnz, self.n_opened, self.ncells = [x.value for x in v]
        self.order = self.params.order
        self.p = num_unknowns(self.order)
        self.L = self.params.L
        self.lo = np.array(self.params.lo[:])
        self.max_depth = self.params.max_depth
        self.unit = self.L / 2.0 ** (self.max_depth + 1)

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.apco_destroy(self.h)
            self.h = None

    def nodes(self):
        n, nb, nnz = self.n, self.nb, self.nnz
        out = dict(perm=np.zeros(self.N, np.int64), code=np.zeros(n, np.uint64),
                   level=np.zeros(n, np.int32), first=np.zeros(n, np.int64),
                   count=np.zeros(n, np.int64), bowner=np.zeros(nb, np.int32),
                   bface=np.zeros(nb, np.int32), st_off=np.zeros(n + 1, np.int32),
                   st_idx=np.zeros(nnz, np.int32), st_ring=np.zeros(n, np.int32))
        self.lib.apco_get_nodes(self.h, *[_ptr(out[k]) for k in
                                          ["perm", "code", "level", "first", "count", "bowner",
                                           "bface", "st_off", "st_idx", "st_ring"]])
        return out

    def node_orders(self) -> np.ndarray:
        o = np.zeros(self.n, np.int8)
        _check(self.lib.apco_node_orders(self.h, _ptr(o)), "node_orders")
        return o

    def density_orders(self) -> np.ndarray:
        o = np.zeros(self.n, np.int8)
        _check(self.lib.apco_density_orders(self.h, _ptr(o)), "density_orders")
        return o

    def coords(self) -> np.ndarray:
        a = np.zeros((3, self.n + self.nb), np.int32)
        self.lib.apco_node_coords(self.h, _ptr(a))
        return a

    def positions(self) -> np.ndarray:
        return self.lo[:, None] + self.unit * self.coords().astype(np.float64)

    def cells(self):
        nc = self.ncells
        lv = np.zeros(nc, np.int32)
        ijk = np.zeros((nc, 3), np.int32)
        cnt = np.zeros(nc, np.int64)
        op = np.zeros(nc, np.int32)
        self.lib.apco_get_cells(self.h, _ptr(lv), _ptr(ijk), _ptr(cnt), _ptr(op))
        return dict(level=lv, ijk=ijk, count=cnt, opened=op)

    def ring1(self):
        off = np.zeros(self.n + 1, np.int32)
        idx = np.zeros(24 * self.n + 6, np.int32)
        _check(self.lib.apco_ring1(self.h, _ptr(off), _ptr(idx), idx.size), "ring1")
        return off, idx[: off[-1]].copy()

    def assemble(self):
        w = np.zeros(self.nnz)
        d = np.zeros(self.n)
        _check(self.lib.apco_assemble(self.h, _ptr(w), _ptr(d)), "assemble")
        return w, d

    def density_rows(self):
        w = np.zeros(self.nnz)
        d = np.zeros(self.n)
        _check(self.lib.apco_density_rows(self.h, _ptr(w), _ptr(d)), "density_rows")
        return w, d

    def deposit(self, q=None):
        r = np.zeros(self.n + self.nb)
        qq = None if q is None else np.ascontiguousarray(q, dtype=np.float64)
        _check(self.lib.apco_deposit_xyz(self.h, _ptr(self.xyz), _ptr(qq), _ptr(r)), "deposit")
        return r

    def density_solve(self, rho_M, tol=1e-12, maxit=10000, precond=0):
        rho_M = np.ascontiguousarray(rho_M, dtype=np.float64)
        out = np.zeros(self.n + self.nb)
        st = _Stats()
        _check(self.lib.apco_density_solve(self.h, _ptr(rho_M), _ptr(out), tol, maxit, precond,
                                           ct.byref(st)), "density_solve")
        return out, dict(iters=st.iters, status=st.status, rel_resid=st.rel_resid,
                         rel_resid_true=st.rel_resid_true)

    def poisson_solve(self, rho_t, g=None, tol=1e-12, maxit=20000, precond=1):
        rho_t = np.ascontiguousarray(rho_t, dtype=np.float64)
        gg = None if g is None else np.ascontiguousarray(g, dtype=np.float64)
        out = np.zeros(self.n + self.nb)
        st = _Stats()
        _check(self.lib.apco_poisson_solve(self.h, _ptr(rho_t), _ptr(gg), _ptr(out), tol, maxit,
                                           precond, ct.byref(st)), "poisson_solve")
        return out, dict(iters=st.iters, status=st.status, rel_resid=st.rel_resid,
                         rel_resid_true=st.rel_resid_true)

    def bicgstab_rows(self, w, diag, rhs, tol=1e-12, maxit=20000, precond=0):
        """The oracle's BiCGSTAB on rows assembled beforehand (no assembly inside)."""
        w = np.ascontiguousarray(w, dtype=np.float64)
        diag = np.ascontiguousarray(diag, dtype=np.float64)
        rhs = np.ascontiguousarray(rhs, dtype=np.float64)
        x = np.zeros(self.n)
        st = _Stats()
        _check(self.lib.apco_bicgstab_rows(self.h, _ptr(w), _ptr(diag), _ptr(rhs), _ptr(x), tol,
                                           maxit, precond, ct.byref(st)), "bicgstab_rows")
        return x, dict(iters=st.iters, status=st.status, rel_resid=st.rel_resid,
                       rel_resid_true=st.rel_resid_true)

    def poisson_lu(self, rho_t, g=None):
        rho_t = np.ascontiguousarray(rho_t, dtype=np.float64)
        gg = None if g is None else np.ascontiguousarray(g, dtype=np.float64)
        out = np.zeros(self.n + self.nb)
        _check(self.lib.apco_poisson_lu(self.h, _ptr(rho_t), _ptr(gg), _ptr(out)), "poisson_lu")
        return out

    def apply_laplacian(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros(self.n)
        _check(self.lib.apco_apply_laplacian(self.h, _ptr(f), _ptr(out)), "apply_laplacian")
        return out

    def node_derivs(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        out = np.zeros((self.n, self.p))
        _check(self.lib.apco_node_derivs(self.h, _ptr(f), _ptr(out)), "node_derivs")
        return out

    def learn_data(self, Z=None):
        """Features (n x 48) and, with probes Z (K x (n+nb)), quadratic data (n x 903)."""
        feat = np.zeros((self.n, 48))
        if Z is None:
            _check(self.lib.apco_learn_data(self.h, None, 0, _ptr(feat), None), "learn_data")
            return feat, None
        Z = np.ascontiguousarray(Z, dtype=np.float64)
        quad = np.zeros((self.n, LEARN_QUAD))
        _check(self.lib.apco_learn_data(self.h, _ptr(Z), Z.shape[0], _ptr(feat), _ptr(quad)),
               "learn_data")
        return feat, quad

    def learned_m(self, params, Z=None):
        """Rows of the learned M: diagonal (n) and weights aligned with the stencil."""
        P = np.ascontiguousarray(params, dtype=np.float64)
        assert P.size == MLP_NPARAM
        md = np.zeros(self.n)
        mw = np.zeros(self.nnz)
        if Z is None:
            _check(self.lib.apco_learned_m(self.h, _ptr(P), None, 0, _ptr(md), _ptr(mw)),
                   "learned_m")
        else:
            Z = np.ascontiguousarray(Z, dtype=np.float64)
            _check(self.lib.apco_learned_m(self.h, _ptr(P), _ptr(Z), Z.shape[0], _ptr(md),
                                           _ptr(mw)), "learned_m")
        return md, mw

    def interpolate(self, phi, xyz=None):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        xyz = self.xyz if xyz is None else np.ascontiguousarray(xyz, dtype=np.float64)
        pp = np.zeros(self.N)
        gp = np.zeros((3, self.N))
        _check(self.lib.apco_interpolate(self.h, _ptr(phi), _ptr(xyz), _ptr(pp), _ptr(gp)),
               "interpolate")
        return pp, gp


class OracleCloud2D:
    """A two-dimensional oracle node cloud (quadtree, k = 2) from particles (2 x N
    float64).  Parameters as for OracleCloud (lo and L of the square; m_cap
    defaults to 8, the paper's 8 neighbours in two dimensions)."""

    def __init__(self, xy: np.ndarray, **params):
        self.lib = _load()
        params.setdefault("m_cap", 8)
        params.setdefault("ring_min", 2)
        lo = params.pop("lo", (0.0, 0.0))
        self.params = make_params(lo=(lo[0], lo[1], 0.0), **params)
        self.xy = np.ascontiguousarray(xy, dtype=np.float64)
        assert self.xy.ndim == 2 and self.xy.shape[0] == 2
        self.N = self.xy.shape[1]
        h = ct.c_void_p()
        _check(self.lib.apco2_build_cloud(ct.byref(self.params), _ptr(self.xy), self.N,
                                          ct.byref(h)), "build_cloud_2d")
        self.h = h
        v = [ct.c_int64() for _ in range(4)]
        self.lib.apco2_info(self.h, *[ct.byref(x) for x in v])
        self.n, self.nb, self.nnz, self.n_opened = [x.value for x in v]
        self.L = self.params.L
        self.lo = np.array(self.params.lo[:2])
        self.max_depth = self.params.max_depth
        self.unit = self.L / 2.0 ** (self.max_depth + 1)

    def __del__(self):
        if getattr(self, "h", None):
            self.lib.apco2_destroy(self.h)
            self.h = None

    def nodes(self):
        n, nb, nnz = self.n, self.nb, self.nnz
        out = dict(perm=np.zeros(self.N, np.int64), code=np.zeros(n, np.uint64),
                   level=np.zeros(n, np.int32), first=np.zeros(n, np.int64),
                   count=np.zeros(n, np.int64), bowner=np.zeros(nb, np.int32),
                   bface=np.zeros(nb, np.int32), st_off=np.zeros(n + 1, np.int32),
                   st_idx=np.zeros(nnz, np.int32))
        self.lib.apco2_get_nodes(self.h, *[_ptr(out[k]) for k in
                                           ["perm", "code", "level", "first", "count", "bowner",
                                            "bface", "st_off", "st_idx"]])
        return out

    def coords(self):
        a = np.zeros((2, self.n + self.nb), np.int32)
        self.lib.apco2_node_coords(self.h, _ptr(a))
        return a

    def positions(self):
        return self.lo[:, None] + self.unit * self.coords().astype(np.float64)

    def ring1(self):
        off = np.zeros(self.n + 1, np.int32)
        idx = np.zeros(8 * self.n + 4, np.int32)
        _check(self.lib.apco2_ring1(self.h, _ptr(off), _ptr(idx), idx.size), "ring1_2d")
        return off, idx[: off[-1]].copy()

    def assemble(self):
        w, d = np.zeros(self.nnz), np.zeros(self.n)
        _check(self.lib.apco2_assemble(self.h, _ptr(w), _ptr(d)), "assemble_2d")
        return w, d

    def density_rows(self):
        w, d, o = np.zeros(self.nnz), np.zeros(self.n), np.zeros(self.n, np.int8)
        _check(self.lib.apco2_density_rows(self.h, _ptr(w), _ptr(d), _ptr(o)), "density_rows_2d")
        return w, d, o

    def deposit(self, q=None):
        r = np.zeros(self.n + self.nb)
        qq = None if q is None else np.ascontiguousarray(q, dtype=np.float64)
        _check(self.lib.apco2_deposit(self.h, _ptr(qq), _ptr(r)), "deposit_2d")
        return r

    def density_solve(self, rho_M, tol=1e-12, maxit=10000):
        rho_M = np.ascontiguousarray(rho_M, dtype=np.float64)
        out = np.zeros(self.n + self.nb)
        st = _Stats()
        _check(self.lib.apco2_density_solve(self.h, _ptr(rho_M), _ptr(out), tol, maxit,
                                            ct.byref(st)), "density_solve_2d")
        return out, dict(iters=st.iters, status=st.status, rel_resid=st.rel_resid,
                         rel_resid_true=st.rel_resid_true)

    def poisson_solve(self, rho_t, g=None, tol=1e-12, maxit=20000, precond=1):
        rho_t = np.ascontiguousarray(rho_t, dtype=np.float64)
        gg = None if g is None else np.ascontiguousarray(g, dtype=np.float64)
        out = np.zeros(self.n + self.nb)
        st = _Stats()
        _check(self.lib.apco2_poisson_solve(self.h, _ptr(rho_t), _ptr(gg), _ptr(out), tol, maxit,
                                            precond, ct.byref(st)), "poisson_solve_2d")
        return out, dict(iters=st.iters, status=st.status, rel_resid=st.rel_resid,
                         rel_resid_true=st.rel_resid_true)

    def apply_laplacian(self, f):
        """sum_j w_ij (f_j - f_i) over each row (f over all n + nb nodes)."""
        w, _ = self.assemble()
        nd = self.nodes()
        rows = np.repeat(np.arange(self.n), np.diff(nd["st_off"]))
        f = np.asarray(f, dtype=np.float64)
        return np.bincount(rows, weights=w * (f[nd["st_idx"]] - f[rows]), minlength=self.n)

    def node_derivs(self, f):
        f = np.ascontiguousarray(f, dtype=np.float64)
        D = np.zeros((self.n, 5))
        _check(self.lib.apco2_node_derivs(self.h, _ptr(f), _ptr(D)), "node_derivs_2d")
        return D

    def interpolate(self, phi, xy=None):
        phi = np.ascontiguousarray(phi, dtype=np.float64)
        xy = self.xy if xy is None else np.ascontiguousarray(xy, dtype=np.float64)
        pp, gp = np.zeros(self.N), np.zeros((2, self.N))
        _check(self.lib.apco2_interpolate(self.h, _ptr(phi), _ptr(xy), _ptr(pp), _ptr(gp)),
               "interpolate_2d")
        return pp, gp
