"""Thin ctypes binding of libapcloud.so (include/apcloud.h).

Argument marshalling only: every step runs in the HIP library.  Device buffers
are torch CUDA tensors (PyTorch-ROCm provides device memory and streams); the
calls receive their raw pointers and the current stream.  There is no CPU
fallback: without the built library every call raises.
"""
from __future__ import annotations

import ctypes as ct
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libapcloud.so")

APC_OK, APC_EINVAL, APC_ENOMEM, APC_EHIP, APC_EDOMAIN, APC_ESTENCIL = 0, -1, -2, -3, -4, -5
APC_ENOCONV = 1
APC_NOALLOC_BYTES = 32 << 20  # fixed derivative buffer of apc_interpolate_force_noalloc
APC_FP64, APC_MIXED, APC_MIXED_F32ACC = 0, 1, 2
APC_KERNEL_NGP, APC_KERNEL_CIC, APC_KERNEL_TSC = 0, 1, 2
APC_PRECOND_NONE, APC_PRECOND_JACOBI, APC_PRECOND_LEARNED = 0, 1, 2
APC_DIAG_KERNEL_TIMES, APC_DIAG_FP64_RESIDUAL = 1, 2
MLP_IN, MLP_HID, MLP_OUT = 48, 64, 41
MLP_NPARAM = MLP_IN * MLP_HID + MLP_HID + MLP_HID * MLP_HID + MLP_HID + MLP_HID * MLP_OUT + MLP_OUT
LEARN_QUAD = MLP_OUT * (MLP_OUT + 1) // 2 + MLP_OUT + 1

# every symbol declared in include/apcloud.h
EXPORTS = ["apc_default_params", "apc_build_cloud", "apc_cloud_info", "apc_get_nodes",
           "apc_assemble_gfd", "apc_get_operator", "apc_get_node_orders",
           "apc_get_density_operator", "apc_operator_info", "apc_operator_boxes", "apc_deposit",
           "apc_density_solve",
           "apc_solve", "apc_interpolate_force", "apc_interpolate_force_noalloc", "apc_node_derivs", "apc_apply_operator",
           "apc_learn_data", "apc_mlp_loss_grad", "apc_mlp_adam", "apc_mlp_infer",
           "apc_set_learned_precond", "apc_apply_precond", "apc_build_batch", "apc_batch_info",
           "apc_batch_configure", "apc_batch_tune", "apc_batch_assemble", "apc_batch_deposit",
           "apc_batch_solve", "apc_batch_set_learned_precond", "apc_batch_interpolate_force",
           "apc_batch_pipeline",
           "apc_batch_destroy", "apc_push",
           "apc_step", "apc_set_diagnostics", "apc_destroy", "apc_strerror", "apc_last_error",
           "apc2_build_cloud", "apc2_cloud_info", "apc2_get_nodes", "apc2_assemble",
           "apc2_get_operator", "apc2_deposit", "apc2_density_solve", "apc2_solve",
           "apc2_node_derivs", "apc2_interpolate_force", "apc2_destroy"]


class ApcError(RuntimeError):
    def __init__(self, code, what):
        self.code = code
        super().__init__(f"{what}: {_strerror(code)} ({code}) {_last_error()}")


class Params(ct.Structure):
    _fields_ = [("lo", ct.c_double * 3), ("L", ct.c_double), ("order", ct.c_int),
                ("c", ct.c_double), ("max_depth", ct.c_int), ("ring_min", ct.c_int),
                ("ring_max", ct.c_int), ("m_cap", ct.c_int), ("poisson_c", ct.c_double),
                ("precision", ct.c_int), ("stage_cap", ct.c_int), ("criterion_pow", ct.c_int),
                ("ring_lds", ct.c_int), ("ring_first_cap", ct.c_int), ("tau_dom", ct.c_double),
                ("periodic", ct.c_int), ("kernel", ct.c_int), ("mask_level", ct.c_int),
                ("mask", ct.c_void_p)]


class Stats(ct.Structure):
    _fields_ = [("iters", ct.c_int), ("restarts", ct.c_int), ("sweeps", ct.c_int),
                ("status", ct.c_int), ("rel_resid", ct.c_double),
                ("rel_resid_true", ct.c_double), ("n_fp64_rows", ct.c_int64), ("ms", ct.c_double),
                ("precond_used", ct.c_int), ("pad", ct.c_int), ("rel_resid_fp64ref", ct.c_double),
                ("spmv_ms", ct.c_double), ("spmv_launches", ct.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class StepStats(ct.Structure):
    _fields_ = [("n", ct.c_int64), ("nb", ct.c_int64), ("nnz", ct.c_int64),
                ("density_iters", ct.c_int), ("iters", ct.c_int), ("status", ct.c_int),
                ("pad", ct.c_int), ("rel_resid_true", ct.c_double), ("ms", ct.c_double * 6)]

    PHASES = ("build", "assemble", "deposit", "solve", "interpolate", "push")

    def as_dict(self):
        out = {k: getattr(self, k) for k, _ in self._fields_ if k not in ("pad", "ms")}
        out["ms"] = dict(zip(self.PHASES, self.ms[:]))
        return out


class BatchInfo(ct.Structure):
    _fields_ = [("count", ct.c_int64), ("N", ct.c_int64), ("n", ct.c_int64), ("nb", ct.c_int64),
                ("nnz", ct.c_int64), ("nsl", ct.c_int64), ("use_graph", ct.c_int),
                ("chunk", ct.c_int), ("spmv_blocks", ct.c_int), ("pad", ct.c_int)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libapcloud.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with paper_1603_04039_amd/build.py "
                          "(or __graft_entry__.build()); there is no fallback path")
    lib = ct.CDLL(path)
    P = ct.c_void_p
    I64 = ct.c_int64
    lib.apc_default_params.argtypes = [ct.POINTER(Params), ct.c_int]
    lib.apc_default_params.restype = None
    lib.apc_build_cloud.argtypes = [ct.POINTER(Params), P, I64, P, ct.POINTER(P)]
    lib.apc_cloud_info.argtypes = [P] + [ct.POINTER(I64)] * 4
    lib.apc_get_nodes.argtypes = [P] * 11
    lib.apc_assemble_gfd.argtypes = [P, P]
    lib.apc_get_operator.argtypes = [P, P, P]
    lib.apc_operator_info.argtypes = [P] + [ct.POINTER(I64)] * 5
    lib.apc_operator_boxes.argtypes = [P, ct.POINTER(I64)]
    lib.apc_get_node_orders.argtypes = [P, P]
    lib.apc_get_density_operator.argtypes = [P, P, P, P]
    lib.apc_deposit.argtypes = [P, P, P, P, ct.c_double, ct.c_int, ct.POINTER(Stats), P]
    lib.apc_density_solve.argtypes = [P, P, P, ct.c_double, ct.c_int, ct.POINTER(Stats), P]
    lib.apc_solve.argtypes = [P, P, P, P, ct.c_double, ct.c_int, ct.c_int, ct.POINTER(Stats), P]
    lib.apc_interpolate_force.argtypes = [P, P, P, P, P]
    lib.apc_interpolate_force_noalloc.argtypes = [P, P, P, P, P]
    lib.apc_node_derivs.argtypes = [P, P, P, P]
    lib.apc_apply_operator.argtypes = [P, P, P, P]
    lib.apc_learn_data.argtypes = [P, P, ct.c_int, P, P, P]
    lib.apc_mlp_loss_grad.argtypes = [P, P, P, P, ct.c_int, P, P, P]
    lib.apc_mlp_adam.argtypes = [P, P, P, P, ct.c_int, ct.c_float, P]
    lib.apc_mlp_infer.argtypes = [P, P, P, ct.c_int, P, P]
    lib.apc_set_learned_precond.argtypes = [P, P, P, ct.c_int, P]
    lib.apc_apply_precond.argtypes = [P, ct.c_int, P, P, P]
    lib.apc_build_batch.argtypes = [ct.POINTER(Params), ct.c_int, P, P, P, ct.POINTER(P)]
    lib.apc_batch_info.argtypes = [P, ct.POINTER(BatchInfo), P, P, P]
    lib.apc_batch_configure.argtypes = [P, ct.c_int, ct.c_int, ct.c_int]
    lib.apc_batch_tune.argtypes = [P, ct.c_double, ct.POINTER(ct.c_int), ct.POINTER(ct.c_int), P]
    lib.apc_batch_assemble.argtypes = [P, P]
    lib.apc_batch_deposit.argtypes = [P, P, P, P, ct.c_double, ct.c_int, P, P]
    lib.apc_batch_solve.argtypes = [P, P, P, P, ct.c_double, ct.c_int, ct.c_int, P, P]
    lib.apc_batch_set_learned_precond.argtypes = [P, P, P, ct.c_int, P]
    lib.apc_batch_interpolate_force.argtypes = [P, P, P, P, P]
    lib.apc_batch_pipeline.argtypes = [P, P, P, ct.c_double, ct.c_double, ct.c_int, ct.c_int,
                                       P, P, P, P, P, P, ct.POINTER(ct.c_int), P]
    lib.apc_batch_destroy.argtypes = [P]
    lib.apc_batch_destroy.restype = None
    lib.apc_push.argtypes = [ct.POINTER(Params), I64, P, P, P, ct.c_double, ct.c_double, P]
    lib.apc_step.argtypes = [ct.POINTER(Params), P, P, P, I64, ct.c_double, ct.c_double,
                             ct.c_double, ct.c_double, ct.c_int, ct.c_int, P, P,
                             ct.POINTER(StepStats), P]
    lib.apc_set_diagnostics.argtypes = [P, ct.c_int]
    lib.apc_destroy.argtypes = [P]
    lib.apc_destroy.restype = None
    lib.apc2_build_cloud.argtypes = [ct.POINTER(Params), P, I64, P, ct.POINTER(P)]
    lib.apc2_cloud_info.argtypes = [P] + [ct.POINTER(I64)] * 4
    lib.apc2_get_nodes.argtypes = [P] * 11
    lib.apc2_assemble.argtypes = [P, P]
    lib.apc2_get_operator.argtypes = [P] * 6
    lib.apc2_deposit.argtypes = [P, P, P, P]
    lib.apc2_density_solve.argtypes = [P, P, P, ct.c_double, ct.c_int, ct.POINTER(Stats), P]
    lib.apc2_solve.argtypes = [P, P, P, P, ct.c_double, ct.c_int, ct.c_int, ct.POINTER(Stats), P]
    lib.apc2_node_derivs.argtypes = [P, P, P, P]
    lib.apc2_interpolate_force.argtypes = [P, P, P, P, P]
    lib.apc2_destroy.argtypes = [P]
    lib.apc2_destroy.restype = None
    lib.apc_strerror.argtypes = [ct.c_int]
    lib.apc_strerror.restype = ct.c_char_p
    lib.apc_last_error.argtypes = []
    lib.apc_last_error.restype = ct.c_char_p
    _lib = lib
    return lib


def _strerror(code):
    return load_library().apc_strerror(code).decode()


def _last_error():
    return load_library().apc_last_error().decode()


def _check(rc, what):
    if rc < 0:
        raise ApcError(rc, what)
    return rc


def make_params(order=2, c=0.35, max_depth=6, lo=(0.0, 0.0, 0.0), L=1.0, ring_min=None,
                ring_max=5, m_cap=None, poisson_c=1.0, precision=APC_FP64,
                stage_cap=0, criterion_pow=0, ring_lds=0, ring_first_cap=0,
                tau_dom=0.0, periodic=0, kernel=0, mask=None) -> Params:
    p = Params()
    load_library().apc_default_params(ct.byref(p), order)
    p.lo[:] = lo
    p.L = L
    p.c = c
    p.max_depth = max_depth
    if ring_min is not None:
        p.ring_min = ring_min
    p.ring_max = ring_max
    if m_cap is not None:
        p.m_cap = m_cap
    p.poisson_c = poisson_c
    p.precision = precision
    p.stage_cap = stage_cap
    p.criterion_pow = criterion_pow
    p.ring_lds = ring_lds
    p.ring_first_cap = ring_first_cap
    p.tau_dom = tau_dom
    p.periodic = periodic
    p.kernel = kernel
    if mask is not None:
        # (s, s, s) boolean array over the level-log2(s) grid, indexed [ix, iy, iz];
        # True excludes the cell.  Handed over with x fastest.
        m = np.asarray(mask).astype(np.uint8)
        s = m.shape[0]
        ml = int(s).bit_length() - 1
        if m.shape != (s, s, s) or (1 << ml) != s:
            raise ValueError("mask must be a (2^l, 2^l, 2^l) array")
        flat = np.ascontiguousarray(m.transpose(2, 1, 0)).ravel()
        p.mask_level = ml
        p.mask = flat.ctypes.data
        p._mask_ref = flat  # alive as long as the parameters
    return p


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ct.c_void_p(s.cuda_stream)


def _dptr(t, dtype=None, numel=None):
    """Raw device pointer of a contiguous CUDA tensor (None passes NULL)."""
    if t is None:
        return None
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.is_contiguous()):
        raise ValueError("expected a contiguous CUDA tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"tensor too small: {t.numel()} < {numel}")
    return ct.c_void_p(t.data_ptr())


class Cloud:
    """A node cloud built on the GPU from particles xyz (3 x N float64 CUDA tensor)."""

    def __init__(self, xyz, stream=None, **params):
        import torch
        self.lib = load_library()
        self.params = make_params(**params)
        self.xyz = xyz
        assert xyz.dim() == 2 and xyz.shape[0] == 3
        self.N = xyz.shape[1]
        h = ct.c_void_p()
        _check(self.lib.apc_build_cloud(ct.byref(self.params), _dptr(xyz, torch.float64),
                                        self.N, _stream(stream), ct.byref(h)), "apc_build_cloud")
        self.h = h
        v = [ct.c_int64() for _ in range(4)]
        _check(self.lib.apc_cloud_info(self.h, *[ct.byref(x) for x in v]), "apc_cloud_info")
        self.n, self.nb, self.nnz, self.n_opened = [x.value for x in v]
        self.L = self.params.L
        self.lo = np.array(self.params.lo[:])
        self.max_depth = self.params.max_depth
        self.p = 9 if self.params.order == 2 else 34
        self.unit = self.L / 2.0 ** (self.max_depth + 1)
        self.assembled = False

    def close(self):
        if getattr(self, "h", None):
            self.lib.apc_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    # ---- structure (host copies)
    def nodes(self):
        n, nb, nnz = self.n, self.nb, self.nnz
        out = dict(perm=np.zeros(self.N, np.int32), code=np.zeros(n, np.uint64),
                   level=np.zeros(n, np.int32), first=np.zeros(n, np.int32),
                   count=np.zeros(n, np.int32), bowner=np.zeros(nb, np.int32),
                   bface=np.zeros(nb, np.int32), st_off=np.zeros(n + 1, np.int32),
                   st_idx=np.zeros(nnz, np.int32), ixyz=np.zeros((3, n + nb), np.int32))
        ptrs = [out[k].ctypes.data_as(ct.c_void_p) for k in
                ["perm", "code", "level", "first", "count", "bowner", "bface", "st_off",
                 "st_idx", "ixyz"]]
        _check(self.lib.apc_get_nodes(self.h, *ptrs), "apc_get_nodes")
        return out

    def node_orders(self):
        o = np.zeros(self.n, np.int8)
        _check(self.lib.apc_get_node_orders(self.h, o.ctypes.data_as(ct.c_void_p)),
               "apc_get_node_orders")
        return o

    def set_diagnostics(self, flags):
        """APC_DIAG_KERNEL_TIMES and/or APC_DIAG_FP64_RESIDUAL for the cloud's solves."""
        _check(self.lib.apc_set_diagnostics(self.h, flags), "apc_set_diagnostics")

    def density_operator(self):
        """Rows of the density operator B (bw aligned with the CSR, diagonal) and the
        order of each row (4, 2 or 0 for the identity row)."""
        bw = np.zeros(max(self.nnz, 1))
        bd = np.zeros(max(self.n, 1))
        o = np.zeros(max(self.n, 1), np.int8)
        _check(self.lib.apc_get_density_operator(self.h, bw.ctypes.data_as(ct.c_void_p),
                                                 bd.ctypes.data_as(ct.c_void_p),
                                                 o.ctypes.data_as(ct.c_void_p)),
               "apc_get_density_operator")
        return bw[:self.nnz], bd[:self.n], o[:self.n]

    def positions(self):
        return self.lo[:, None] + self.unit * self.nodes()["ixyz"].astype(np.float64)

    # ---- the hot path
    def assemble_gfd(self, stream=None):
        _check(self.lib.apc_assemble_gfd(self.h, _stream(stream)), "apc_assemble_gfd")
        self.assembled = True

    def operator(self):
        w = np.zeros(self.nnz)
        d = np.zeros(self.n)
        _check(self.lib.apc_get_operator(self.h, w.ctypes.data_as(ct.c_void_p),
                                         d.ctypes.data_as(ct.c_void_p)), "apc_get_operator")
        return w, d

    def operator_boxes(self):
        """Number of boxed slices (64-row 4 x 4 x 4 blocks of uniform k = 4 rows)."""
        v = ct.c_int64()
        _check(self.lib.apc_operator_boxes(self.h, ct.byref(v)), "apc_operator_boxes")
        return v.value

    def operator_info(self, m_entries=False, staged=False):
        v = [ct.c_int64() for _ in range(4)]
        st = (ct.c_int64 * 4)()
        refs = ([ct.byref(x) for x in v[:3]] + [ct.byref(v[3]) if m_entries else None]
                + [ct.cast(st, ct.POINTER(ct.c_int64)) if staged else None])
        _check(self.lib.apc_operator_info(self.h, *refs), "apc_operator_info")
        out = dict(n_uniform=v[0].value, nnz_general=v[1].value, sell_entries=v[2].value)
        if m_entries:
            out["m_entries"] = v[3].value
        if staged:
            out.update(staged_slices=st[0], staged_distinct=st[1], staged_entries=st[2],
                       stage_tile=st[3])
        return out

    def deposit(self, q=None, tol=1e-12, maxit=1000, stream=None, rho_M=None, rho_t=None):
        import torch
        nt = self.n + self.nb
        rho_M = rho_M if rho_M is not None else torch.empty(nt, dtype=torch.float64, device="cuda")
        rho_t = rho_t if rho_t is not None else torch.empty(nt, dtype=torch.float64, device="cuda")
        st = Stats()
        rc = _check(self.lib.apc_deposit(self.h, _dptr(q, torch.float64, self.N),
                                         _dptr(rho_M, torch.float64, nt),
                                         _dptr(rho_t, torch.float64, nt), tol, maxit,
                                         ct.byref(st), _stream(stream)), "apc_deposit")
        return rho_M, rho_t, dict(st.as_dict(), rc=rc)

    def density_solve(self, rho_M, tol=1e-12, maxit=1000, stream=None, rho_t=None):
        import torch
        nt = self.n + self.nb
        rho_t = rho_t if rho_t is not None else torch.empty(nt, dtype=torch.float64, device="cuda")
        st = Stats()
        rc = _check(self.lib.apc_density_solve(self.h, _dptr(rho_M, torch.float64, nt),
                                               _dptr(rho_t, torch.float64, nt), tol, maxit,
                                               ct.byref(st), _stream(stream)), "apc_density_solve")
        return rho_t, dict(st.as_dict(), rc=rc)

    def solve(self, rho_t, g=None, tol=1e-8, maxit=20000, precond=APC_PRECOND_JACOBI,
              stream=None, phi=None):
        import torch
        nt = self.n + self.nb
        phi = phi if phi is not None else torch.empty(nt, dtype=torch.float64, device="cuda")
        st = Stats()
        rc = _check(self.lib.apc_solve(self.h, _dptr(rho_t, torch.float64, self.n),
                                       _dptr(g, torch.float64, self.nb),
                                       _dptr(phi, torch.float64, nt), tol, maxit, precond,
                                       ct.byref(st), _stream(stream)), "apc_solve")
        return phi, dict(st.as_dict(), rc=rc)

    def interpolate_force(self, phi, stream=None, phi_p=None, grad_p=None):
        import torch
        phi_p = phi_p if phi_p is not None else torch.empty(self.N, dtype=torch.float64,
                                                            device="cuda")
        grad_p = grad_p if grad_p is not None else torch.empty((3, self.N), dtype=torch.float64,
                                                               device="cuda")
        _check(self.lib.apc_interpolate_force(self.h, _dptr(phi, torch.float64, self.n + self.nb),
                                              _dptr(phi_p, torch.float64, self.N),
                                              _dptr(grad_p, torch.float64, 3 * self.N),
                                              _stream(stream)), "apc_interpolate_force")
        return phi_p, grad_p

    def interpolate_force_noalloc(self, phi, phi_p, grad_p, stream=None):
        """apc_interpolate_force_noalloc into caller-owned outputs (no allocation in
        the library)."""
        import torch
        _check(self.lib.apc_interpolate_force_noalloc(
            self.h, _dptr(phi, torch.float64, self.n + self.nb),
            _dptr(phi_p, torch.float64, self.N), _dptr(grad_p, torch.float64, 3 * self.N),
            _stream(stream)), "apc_interpolate_force_noalloc")
        return phi_p, grad_p

    def node_derivs(self, f, stream=None):
        import torch
        D = torch.empty((self.n, self.p), dtype=torch.float64, device="cuda")
        _check(self.lib.apc_node_derivs(self.h, _dptr(f, torch.float64, self.n + self.nb),
                                        _dptr(D), _stream(stream)), "apc_node_derivs")
        return D

    # ---- learned preconditioner
    def learn_data(self, Z=None, stream=None):
        """Row features (n x 48 float32) and, with probes Z (K x (n+nb) float64),
        the per-row quadratic loss data (n x 903 float32)."""
        import torch
        nt = self.n + self.nb
        feat = torch.empty((self.n, MLP_IN), dtype=torch.float32, device="cuda")
        quad = None
        K = 0
        if Z is not None:
            assert Z.dim() == 2 and Z.shape[1] == nt
            K = Z.shape[0]
            quad = torch.empty((self.n, LEARN_QUAD), dtype=torch.float32, device="cuda")
        _check(self.lib.apc_learn_data(self.h, _dptr(Z, torch.float64), K, _dptr(feat),
                                       _dptr(quad), _stream(stream)), "apc_learn_data")
        return feat, quad

    def mlp_infer(self, params, feat, bf16=False, stream=None):
        import torch
        out = torch.empty((self.n, MLP_OUT), dtype=torch.float32, device="cuda")
        _check(self.lib.apc_mlp_infer(self.h, _dptr(params, torch.float32, MLP_NPARAM),
                                      _dptr(feat, torch.float32, self.n * MLP_IN), int(bf16),
                                      _dptr(out), _stream(stream)), "apc_mlp_infer")
        return out

    def set_learned_precond(self, params, Z=None, stream=None):
        """Install M from the network parameters; Z (K x (n+nb) float64 probes)
        enables the per-row safeguard towards Jacobi."""
        import torch
        K = 0
        if Z is not None:
            assert Z.dim() == 2 and Z.shape[1] == self.n + self.nb
            K = Z.shape[0]
        _check(self.lib.apc_set_learned_precond(self.h, _dptr(params, torch.float32, MLP_NPARAM),
                                                _dptr(Z, torch.float64), K, _stream(stream)),
               "apc_set_learned_precond")

    def apply_precond(self, f, precond=APC_PRECOND_LEARNED, stream=None):
        """out = M f over the interior rows (f: n+nb)."""
        import torch
        out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        _check(self.lib.apc_apply_precond(self.h, int(precond),
                                          _dptr(f, torch.float64, self.n + self.nb), _dptr(out),
                                          _stream(stream)), "apc_apply_precond")
        return out

    def apply_operator(self, f, stream=None):
        import torch
        out = torch.empty(self.n, dtype=torch.float64, device="cuda")
        _check(self.lib.apc_apply_operator(self.h, _dptr(f, torch.float64, self.n + self.nb),
                                           _dptr(out), _stream(stream)), "apc_apply_operator")
        return out


def _particles(t, N=None):
    import torch
    if not (isinstance(t, torch.Tensor) and t.dim() == 2 and t.shape[0] == 3):
        raise ValueError("expected a 3 x N tensor")
    if N is not None and t.shape[1] != N:
        raise ValueError(f"expected 3 x {N}, got {tuple(t.shape)}")
    return _dptr(t, torch.float64)


def push(xyz, vel, grad, kick, dt, stream=None, **params):
    """Leapfrog kick-drift push with specular walls (apc_push), in place on the
    3 x N float64 CUDA tensors xyz and vel; grad: 3 x N.  params: the domain
    (lo, L) as for Cloud."""
    p = make_params(**params)
    N = xyz.shape[1]
    _check(load_library().apc_push(ct.byref(p), N, _particles(xyz), _particles(vel, N),
                                   _particles(grad, N), kick, dt, _stream(stream)), "apc_push")
    return xyz, vel


def step(xyz, vel, kick, dt, q=None, tol_density=1e-12, tol=1e-8, maxit=20000,
         precond=APC_PRECOND_JACOBI, stream=None, phi_p=None, grad_p=None, **params):
    """One Vlasov-Poisson time step (apc_step): cloud from xyz, field, push of xyz
    and vel in place.  Returns (phi_p, grad_p, stats) -- the potential and its
    gradient at the positions the step started from."""
    import torch
    p = make_params(**params)
    N = xyz.shape[1]
    phi_p = phi_p if phi_p is not None else torch.empty(N, dtype=torch.float64, device="cuda")
    grad_p = grad_p if grad_p is not None else torch.empty((3, N), dtype=torch.float64,
                                                           device="cuda")
    st = StepStats()
    rc = _check(load_library().apc_step(ct.byref(p), _particles(xyz), _particles(vel, N),
                                        _dptr(q, torch.float64, N), N, kick, dt, tol_density,
                                        tol, maxit, precond, _dptr(phi_p, torch.float64, N),
                                        _particles(grad_p, N), ct.byref(st), _stream(stream)),
                "apc_step")
    return phi_p, grad_p, dict(st.as_dict(), rc=rc)


def mlp_loss_grad(params, feat, quad, rows, stream=None, grad=None, loss=None):
    """Mean loss over feat/quad rows[B] and its gradient (FP32 device tensors)."""
    import torch
    lib = load_library()
    grad = grad if grad is not None else torch.empty(MLP_NPARAM, dtype=torch.float32,
                                                     device="cuda")
    loss = loss if loss is not None else torch.empty(1, dtype=torch.float32, device="cuda")
    _check(lib.apc_mlp_loss_grad(_dptr(params, torch.float32, MLP_NPARAM),
                                 _dptr(feat, torch.float32), _dptr(quad, torch.float32),
                                 _dptr(rows, torch.int32), rows.numel(), _dptr(loss),
                                 _dptr(grad, torch.float32, MLP_NPARAM), _stream(stream)),
           "apc_mlp_loss_grad")
    return loss, grad


def mlp_adam(params, m, v, grad, step, lr, stream=None):
    import torch
    lib = load_library()
    f32 = torch.float32
    _check(lib.apc_mlp_adam(_dptr(params, f32, MLP_NPARAM), _dptr(m, f32, MLP_NPARAM),
                            _dptr(v, f32, MLP_NPARAM), _dptr(grad, f32, MLP_NPARAM), int(step),
                            float(lr), _stream(stream)), "apc_mlp_adam")


class Batch:
    """count clouds (list of 3 x N_c float64 CUDA tensors) built with one set of
    parameters and held as one union (see apc_build_batch)."""

    def __init__(self, xyz_list, stream=None, **params):
        import torch
        self.lib = load_library()
        self.params = make_params(**params)
        self.xyz = list(xyz_list)
        self.count = len(self.xyz)
        ptrs = (ct.c_void_p * self.count)(*[_dptr(x, torch.float64).value for x in self.xyz])
        Ns = (ct.c_int64 * self.count)(*[x.shape[1] for x in self.xyz])
        h = ct.c_void_p()
        _check(self.lib.apc_build_batch(ct.byref(self.params), self.count, ptrs, Ns,
                                        _stream(stream), ct.byref(h)), "apc_build_batch")
        self.h = h
        self.refresh()

    def refresh(self):
        info = BatchInfo()
        cN, cn, cnb = [np.zeros(self.count, np.int64) for _ in range(3)]
        _check(self.lib.apc_batch_info(self.h, ct.byref(info), cN.ctypes.data_as(ct.c_void_p),
                                       cn.ctypes.data_as(ct.c_void_p),
                                       cnb.ctypes.data_as(ct.c_void_p)), "apc_batch_info")
        self.info = {k: getattr(info, k) for k, _ in BatchInfo._fields_ if k != "pad"}
        self.N, self.n, self.nb = int(info.N), int(info.n), int(info.nb)
        self.cloud_N, self.cloud_n, self.cloud_nb = cN, cn, cnb
        self.pbase = np.concatenate([[0], np.cumsum(cN)[:-1]])
        self.ibase = np.concatenate([[0], np.cumsum(cn)[:-1]])
        self.bbase = np.concatenate([[0], np.cumsum(cnb)[:-1]])

    def node_index(self, c):
        """Batch positions of cloud c's n_c + nb_c nodes, in single-cloud order."""
        return np.concatenate([self.ibase[c] + np.arange(self.cloud_n[c]),
                               self.n + self.bbase[c] + np.arange(self.cloud_nb[c])])

    def close(self):
        if getattr(self, "h", None):
            self.lib.apc_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def configure(self, use_graph=-1, chunk=0, spmv_div=0):
        _check(self.lib.apc_batch_configure(self.h, int(use_graph), int(chunk), int(spmv_div)),
               "apc_batch_configure")
        self.refresh()

    def tune(self, tol=1e-8, stream=None):
        d, c = ct.c_int(), ct.c_int()
        _check(self.lib.apc_batch_tune(self.h, tol, ct.byref(d), ct.byref(c), _stream(stream)),
               "apc_batch_tune")
        self.refresh()
        return d.value, c.value

    def assemble_gfd(self, stream=None):
        _check(self.lib.apc_batch_assemble(self.h, _stream(stream)), "apc_batch_assemble")

    def _stats(self):
        return (Stats * self.count)()

    def deposit(self, q=None, tol=1e-12, maxit=1000, stream=None):
        import torch
        nt = self.n + self.nb
        rho_M = torch.empty(nt, dtype=torch.float64, device="cuda")
        rho_t = torch.empty(nt, dtype=torch.float64, device="cuda")
        st = self._stats()
        rc = _check(self.lib.apc_batch_deposit(self.h, _dptr(q, torch.float64, self.N),
                                               _dptr(rho_M), _dptr(rho_t), tol, maxit,
                                               ct.cast(st, ct.c_void_p), _stream(stream)),
                    "apc_batch_deposit")
        return rho_M, rho_t, [dict(x.as_dict(), rc=rc) for x in st]

    def solve(self, rho_t, g=None, tol=1e-8, maxit=20000, precond=APC_PRECOND_JACOBI,
              stream=None):
        import torch
        nt = self.n + self.nb
        phi = torch.empty(nt, dtype=torch.float64, device="cuda")
        st = self._stats()
        rc = _check(self.lib.apc_batch_solve(self.h, _dptr(rho_t, torch.float64, self.n),
                                             _dptr(g, torch.float64, self.nb), _dptr(phi), tol,
                                             maxit, precond, ct.cast(st, ct.c_void_p),
                                             _stream(stream)), "apc_batch_solve")
        return phi, [dict(x.as_dict(), rc=rc) for x in st]

    def set_learned_precond(self, params, Z=None, stream=None):
        """Install the learned M of every cloud on the union (second order); Z
        (K x (n_total + nb_total) float64 probes) enables the per-row safeguard."""
        import torch
        K = 0
        if Z is not None:
            assert Z.dim() == 2 and Z.shape[1] == self.n + self.nb
            K = Z.shape[0]
        _check(self.lib.apc_batch_set_learned_precond(
            self.h, _dptr(params, torch.float32, MLP_NPARAM), _dptr(Z, torch.float64), K,
            _stream(stream)), "apc_batch_set_learned_precond")

    def interpolate_force(self, phi, stream=None):
        import torch
        phi_p = torch.empty(self.N, dtype=torch.float64, device="cuda")
        grad_p = torch.empty((3, self.N), dtype=torch.float64, device="cuda")
        _check(self.lib.apc_batch_interpolate_force(
            self.h, _dptr(phi, torch.float64, self.n + self.nb), _dptr(phi_p), _dptr(grad_p),
            _stream(stream)), "apc_batch_interpolate_force")
        return phi_p, grad_p

    def pipeline(self, q=None, g=None, tol_density=1e-12, tol=1e-8, maxit=20000,
                 precond=APC_PRECOND_JACOBI, out=None, stream=None):
        """Assembly, deposit with the density solve, Poisson solve and interpolation of
        every cloud as one graph replay (apc_batch_pipeline).  out: the four output
        tensors (rho_t, phi, phi_p, grad_p) to reuse, so that the recorded graph is
        replayed (new buffers record it again).  Returns (rho_t, phi, phi_p, grad_p),
        the density and Poisson records, and whether the graph ran."""
        import torch
        nt = self.n + self.nb
        if out is None:
            out = (torch.empty(nt, dtype=torch.float64, device="cuda"),
                   torch.empty(nt, dtype=torch.float64, device="cuda"),
                   torch.empty(self.N, dtype=torch.float64, device="cuda"),
                   torch.empty((3, self.N), dtype=torch.float64, device="cuda"))
        rho_t, phi, phi_p, grad_p = out
        sd, sp = self._stats(), self._stats()
        used = ct.c_int()
        rc = _check(self.lib.apc_batch_pipeline(
            self.h, _dptr(q, torch.float64, self.N), _dptr(g, torch.float64, self.nb),
            tol_density, tol, maxit, precond, _dptr(rho_t, torch.float64, nt),
            _dptr(phi, torch.float64, nt), _dptr(phi_p, torch.float64, self.N),
            _dptr(grad_p, torch.float64, 3 * self.N), ct.cast(sd, ct.c_void_p),
            ct.cast(sp, ct.c_void_p), ct.byref(used), _stream(stream)), "apc_batch_pipeline")
        return (out, [dict(x.as_dict(), rc=rc) for x in sd], [dict(x.as_dict(), rc=rc) for x in sp],
                bool(used.value))


# C-ABI names as free functions
def build_cloud(xyz, stream=None, **params) -> Cloud:
    return Cloud(xyz, stream=stream, **params)


def assemble_gfd(cloud: Cloud, stream=None):
    return cloud.assemble_gfd(stream)


def deposit(cloud: Cloud, q=None, **kw):
    return cloud.deposit(q, **kw)


def solve(cloud: Cloud, rho_t, g=None, **kw):
    return cloud.solve(rho_t, g, **kw)


def interpolate_force(cloud: Cloud, phi, stream=None):
    return cloud.interpolate_force(phi, stream)


class Cloud2D:
    """A two-dimensional node cloud (quadtree, k = 2) built on the GPU from particles
    xy (2 x N float64 CUDA tensor).  params as for make_params (lo of the square as
    a pair; m_cap defaults to 8, the paper's 8 neighbours in two dimensions)."""

    def __init__(self, xy, stream=None, **params):
        import torch
        self.lib = load_library()
        params.setdefault("m_cap", 8)
        params.setdefault("ring_min", 2)
        lo = params.pop("lo", (0.0, 0.0))
        self.params = make_params(lo=(lo[0], lo[1], 0.0), **params)
        if not (isinstance(xy, torch.Tensor) and xy.dim() == 2 and xy.shape[0] == 2):
            raise ValueError("expected a 2 x N tensor")
        self.N = xy.shape[1]
        h = ct.c_void_p()
        _check(self.lib.apc2_build_cloud(ct.byref(self.params), _dptr(xy, torch.float64), self.N,
                                         _stream(stream), ct.byref(h)), "apc2_build_cloud")
        self.h = h
        v = [ct.c_int64() for _ in range(4)]
        self.lib.apc2_cloud_info(self.h, *[ct.byref(x) for x in v])
        self.n, self.nb, self.nnz, self.n_opened = [x.value for x in v]

    def close(self):
        if getattr(self, "h", None):
            self.lib.apc2_destroy(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def nodes(self):
        n, nb, nnz, N = self.n, self.nb, self.nnz, self.N
        out = dict(perm=np.zeros(N, np.int32), code=np.zeros(n, np.uint64),
                   level=np.zeros(n, np.int32), first=np.zeros(n, np.int32),
                   count=np.zeros(n, np.int32), bowner=np.zeros(nb, np.int32),
                   bface=np.zeros(nb, np.int32), st_off=np.zeros(n + 1, np.int32),
                   st_idx=np.zeros(nnz, np.int32), ixy=np.zeros((2, n + nb), np.int32))
        _check(self.lib.apc2_get_nodes(self.h, *[out[k].ctypes.data for k in
                                                 ["perm", "code", "level", "first", "count",
                                                  "bowner", "bface", "st_off", "st_idx", "ixy"]]),
               "apc2_get_nodes")
        return out

    def assemble(self, stream=None):
        _check(self.lib.apc2_assemble(self.h, _stream(stream)), "apc2_assemble")

    def operator(self):
        """(w, diag, bw, bdiag, order) on the host."""
        w, d = np.zeros(self.nnz), np.zeros(self.n)
        bw, bd, o = np.zeros(self.nnz), np.zeros(self.n), np.zeros(self.n, np.int8)
        _check(self.lib.apc2_get_operator(self.h, w.ctypes.data, d.ctypes.data, bw.ctypes.data,
                                          bd.ctypes.data, o.ctypes.data), "apc2_get_operator")
        return w, d, bw, bd, o

    def deposit(self, q=None, stream=None):
        import torch
        rho = torch.empty(self.n + self.nb, dtype=torch.float64, device="cuda")
        _check(self.lib.apc2_deposit(self.h, _dptr(q, torch.float64, self.N), _dptr(rho),
                                     _stream(stream)), "apc2_deposit")
        return rho

    def density_solve(self, rho_M, tol=1e-12, maxit=1000, stream=None):
        import torch
        out = torch.empty(self.n + self.nb, dtype=torch.float64, device="cuda")
        st = Stats()
        rc = _check(self.lib.apc2_density_solve(self.h, _dptr(rho_M, torch.float64, self.n + self.nb),
                                                _dptr(out), tol, maxit, ct.byref(st),
                                                _stream(stream)), "apc2_density_solve")
        return out, dict(st.as_dict(), rc=rc)

    def solve(self, rho_t, g=None, tol=1e-10, maxit=20000, precond=APC_PRECOND_JACOBI,
              stream=None):
        import torch
        phi = torch.empty(self.n + self.nb, dtype=torch.float64, device="cuda")
        st = Stats()
        rc = _check(self.lib.apc2_solve(self.h, _dptr(rho_t, torch.float64, self.n),
                                        _dptr(g, torch.float64, self.nb), _dptr(phi), tol, maxit,
                                        precond, ct.byref(st), _stream(stream)), "apc2_solve")
        return phi, dict(st.as_dict(), rc=rc)

    def node_derivs(self, f, stream=None):
        import torch
        D = torch.empty((self.n, 5), dtype=torch.float64, device="cuda")
        _check(self.lib.apc2_node_derivs(self.h, _dptr(f, torch.float64, self.n + self.nb),
                                         _dptr(D), _stream(stream)), "apc2_node_derivs")
        return D

    def interpolate_force(self, phi, stream=None):
        import torch
        pp = torch.empty(self.N, dtype=torch.float64, device="cuda")
        gp = torch.empty((2, self.N), dtype=torch.float64, device="cuda")
        _check(self.lib.apc2_interpolate_force(self.h, _dptr(phi, torch.float64, self.n + self.nb),
                                               _dptr(pp), _dptr(gp), _stream(stream)),
               "apc2_interpolate_force")
        return pp, gp

