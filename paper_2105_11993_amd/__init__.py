"""Python binding of libthm.so, the MI355X time-harmonic Maxwell solver.

Argument marshalling only: every step of assembly and solve runs in the HIP
library (include/thm.h).  PyTorch provides device memory and streams.  The
binding raises ImportError if the library has not been built; there is no
fallback path.

Functions keep the C names: thm_assemble, thm_gmres_solve, thm_ddm_solve,
thm_adjoint_grad, plus the lifecycle and kernel-level entry points.
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libthm.so")

THM_OK, THM_NOT_CONVERGED = 0, 1
THM_FP64, THM_FP32_IR = 0, 1
THM_DDM_GMRES, THM_DDM_JACOBI = 0, 1
THM_ORTH_CGS, THM_ORTH_CGS2 = 0, 1
THM_KRYLOV_COMPLEX, THM_KRYLOV_REAL = 0, 1
THM_PREC_BLOCK, THM_PREC_FULL = 0, 1
THM_IR_CLASSIC, THM_IR_GMRES = 0, 1

_d3 = ctypes.c_double * 3
_i3 = ctypes.c_int32 * 3


class ThmProblem(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("cells", _i3), ("box_lo", _d3), ("box_hi", _d3),
                ("degree", ctypes.c_int32), ("omega", ctypes.c_double), ("kappa", ctypes.c_double),
                ("mu", ctypes.POINTER(ctypes.c_double)), ("inc_faces", ctypes.c_uint32), ("inc_dir", _d3),
                ("inc_pol_re", _d3), ("inc_pol_im", _d3), ("subdomains", _i3),
                ("eps", ctypes.POINTER(ctypes.c_double)), ("transmission", ctypes.c_double * 2)]


class ThmSolveOpts(ctypes.Structure):
    _fields_ = [("restart", ctypes.c_int32), ("max_iter", ctypes.c_int32), ("rtol", ctypes.c_double),
                ("precision", ctypes.c_int32), ("orth", ctypes.c_int32), ("transpose", ctypes.c_int32),
                ("ddm_outer", ctypes.c_int32), ("inner_rtol", ctypes.c_double), ("max_outer", ctypes.c_int32),
                ("outer_restart", ctypes.c_int32), ("batched", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("ir_inner_rtol", ctypes.c_double), ("max_refine", ctypes.c_int32), ("krylov", ctypes.c_int32),
                ("relax_inner", ctypes.c_int32), ("precond", ctypes.c_int32), ("ir_mode", ctypes.c_int32)]


class ThmStats(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("iters", ctypes.c_int32), ("outer_iters", ctypes.c_int32),
                ("refinements", ctypes.c_int32), ("rel_residual", ctypes.c_double), ("setup_ms", ctypes.c_double),
                ("solve_ms", ctypes.c_double), ("fp64_fallback", ctypes.c_int32),
                ("precond_extra_bytes", ctypes.c_int64), ("gmres_ir", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class ThmInfo(ctypes.Structure):
    _fields_ = [("n_dofs", ctypes.c_int64), ("n_free", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("nnz_c", ctypes.c_int64), ("n_cells", ctypes.c_int64), ("n_subdomains", ctypes.c_int32),
                ("n_layers", ctypes.c_int32), ("factor_bytes", ctypes.c_int64), ("n_interface", ctypes.c_int64),
                ("spmv_variant", ctypes.c_int32), ("ddm_spmv_variant", ctypes.c_int32),
                ("ddm_spmv_groups", ctypes.c_int32)]


EXPORTS = ["thm_default_opts", "thm_assemble", "thm_gmres_solve", "thm_ddm_solve", "thm_adjoint_grad",
           "thm_system_info", "thm_system_set_mu", "thm_system_destroy", "thm_last_error", "thm_apply_operator",
           "thm_apply_precond", "thm_export_matrices", "thm_export_rhs", "thm_export_elements", "thm_time_spmv",
           "thm_time_precond", "thm_set_spmv_variant", "thm_apply_precond_full", "thm_time_spmv_batch",
           "thm_time_spmv_systems", "thm_system_release_workspaces", "thm_apply_precond_noalloc"]
THM_SPMV_SELL = 19
THM_SPMV_SELL_GROUP = 20
THM_SPMV_SELL_GROUP_IL = 29  # timing code of the grouped product on the member-interleaved copy
SPMV_VARIANTS = [21, 41, 81, 161, 321, 641, 24, 44, 84, 164, 324, THM_SPMV_SELL, THM_SPMV_SELL_GROUP]


def load_library(path=LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python paper_2105_11993_amd/build_lib.py`")
    lib = ctypes.CDLL(path)
    vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)
    sig = {
        "thm_default_opts": (None, [ctypes.POINTER(ThmSolveOpts)]),
        "thm_assemble": (i32, [ctypes.POINTER(ThmProblem), vp, ctypes.POINTER(vp)]),
        "thm_gmres_solve": (i32, [i32, ctypes.POINTER(vp), ctypes.POINTER(ThmSolveOpts), ctypes.POINTER(vp),
                                  ctypes.POINTER(ThmStats), vp]),
        "thm_ddm_solve": (i32, [vp, ctypes.POINTER(ThmSolveOpts), vp, ctypes.POINTER(ThmStats), vp]),
        "thm_adjoint_grad": (i32, [vp, vp, dp, dp, ctypes.POINTER(ThmSolveOpts), vp, dp, vp]),
        "thm_system_info": (i32, [vp, ctypes.POINTER(ThmInfo)]),
        "thm_system_set_mu": (i32, [vp, vp, vp]),
        "thm_system_destroy": (None, [vp]),
        "thm_system_release_workspaces": (i32, [vp]),
        "thm_last_error": (ctypes.c_char_p, []),
        "thm_apply_operator": (i32, [vp, i32, i32, vp, vp, vp]),
        "thm_apply_precond": (i32, [vp, i32, vp, vp, vp]),
        "thm_export_matrices": (i32, [vp, vp, vp, vp, vp, vp, vp]),
        "thm_export_rhs": (i32, [vp, vp, vp, vp]),
        "thm_export_elements": (i32, [vp, i64, i64, vp]),
        "thm_time_spmv": (i32, [vp, i32, i32, dp, dp, vp]),
        "thm_time_spmv_batch": (i32, [vp, i32, i32, i32, dp, dp, vp]),
        "thm_time_spmv_systems": (i32, [i32, ctypes.POINTER(vp), i32, i32, dp, dp, vp]),
        "thm_time_precond": (i32, [vp, i32, i32, dp, dp, ctypes.POINTER(i32), vp]),
        "thm_set_spmv_variant": (i32, [vp, i32, i32]),
        "thm_apply_precond_full": (i32, [vp, i32, i32, vp, vp, vp]),
        "thm_apply_precond_noalloc": (i32, [vp, i32, vp, vp, vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = load_library()


class ThmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"thm status {code}: {msg}")
        self.code = code


def _check(rc, allow_warning=False):
    if rc < 0 or (rc > 0 and not allow_warning):
        raise ThmError(rc, _lib.thm_last_error().decode())
    return rc


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def default_opts(**kw):
    o = ThmSolveOpts()
    _lib.thm_default_opts(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def make_problem(d):
    """ThmProblem from a workload dict (dim, n, p, omega, kappa, mu, inc_faces, inc_dir,
    inc_pol, lo, hi, subdomains, eps, transmission).  Returns (struct, keep-alive buffers)."""
    p = ThmProblem()
    dim = int(d["dim"])
    p.dim = dim
    n = list(d["n"]) + [1] * (3 - len(d["n"]))
    p.cells = _i3(*[int(v) for v in n[:3]])
    lo = list(d.get("lo", (0.0, 0.0, 0.0))) + [0.0] * 3
    hi = list(d.get("hi", (1.0, 1.0, 1.0))) + [1.0] * 3
    p.box_lo = _d3(*[float(v) for v in lo[:3]])
    p.box_hi = _d3(*[float(v) for v in hi[:3]])
    p.degree = int(d["p"])
    p.omega = float(d["omega"])
    p.kappa = float(d.get("kappa", 1.0))
    keep = []
    for name in ("mu", "eps"):
        v = d.get(name)
        if v is not None:
            arr = np.ascontiguousarray(np.asarray(v, dtype=np.float64).ravel())
            keep.append(arr)
            setattr(p, name, arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    p.inc_faces = int(d.get("inc_faces", 1))
    dirv = list(d.get("inc_dir", (1.0, 0.0, 0.0))) + [0.0] * 3
    pol = [complex(v) for v in list(d.get("inc_pol", (0.0, 1.0, 0.0))) + [0.0] * 3]
    p.inc_dir = _d3(*[float(v) for v in dirv[:3]])
    p.inc_pol_re = _d3(*[v.real for v in pol[:3]])
    p.inc_pol_im = _d3(*[v.imag for v in pol[:3]])
    sub = list(d.get("subdomains", (1, 1, 1))) + [1] * 3
    p.subdomains = _i3(*[int(v) for v in sub[:3]])
    ts = complex(d.get("transmission", 1.0))
    p.transmission = (ctypes.c_double * 2)(ts.real, ts.imag)
    return p, keep


class System:
    """An assembled problem (owns a thm_system handle)."""

    def __init__(self, handle, spec):
        self.handle = ctypes.c_void_p(handle)
        self.spec = spec
        self._info = None

    @property
    def info(self):
        if self._info is None:
            self._info = self.fresh_info()
        return self._info

    def fresh_info(self):
        i = ThmInfo()
        _check(_lib.thm_system_info(self.handle, ctypes.byref(i)))
        return {k: getattr(i, k) for k, _ in ThmInfo._fields_}

    @property
    def n(self):
        return self.info["n_dofs"]

    def close(self):
        if self.handle and self.handle.value:
            _lib.thm_system_destroy(self.handle)
            self.handle = ctypes.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def thm_assemble(spec, stream=None):
    p, keep = make_problem(spec)
    h = ctypes.c_void_p()
    _check(_lib.thm_assemble(ctypes.byref(p), _stream(stream), ctypes.byref(h)))
    del keep
    return System(h.value, spec)


def _cvec(n, E=None):
    torch = _torch()
    if E is None:
        return torch.zeros(n, dtype=torch.complex128, device="cuda")
    if E.dtype != torch.complex128 or not E.is_cuda or not E.is_contiguous() or E.numel() != n:
        raise ValueError("vectors must be contiguous complex128 CUDA tensors of length n_dofs")
    return E


def thm_gmres_solve(systems, opts=None, E=None, stream=None, allow_not_converged=False):
    """Solve each system; returns (list of complex128 tensors, list of stats dicts)."""
    if isinstance(systems, System):
        systems = [systems]
    opts = opts or default_opts()
    ns = len(systems)
    Es = [_cvec(s.n, None if E is None else E[i]) for i, s in enumerate(systems)]
    hs = (ctypes.c_void_p * ns)(*[s.handle.value for s in systems])
    es = (ctypes.c_void_p * ns)(*[e.data_ptr() for e in Es])
    st = (ThmStats * ns)()
    rc = _lib.thm_gmres_solve(ns, hs, ctypes.byref(opts), es, st, _stream(stream))
    _check(rc, allow_warning=allow_not_converged)
    return Es, [s.as_dict() for s in st]


def thm_ddm_solve(system, opts=None, E=None, stream=None, allow_not_converged=False):
    opts = opts or default_opts()
    Eo = _cvec(system.n, E)
    st = ThmStats()
    rc = _lib.thm_ddm_solve(system.handle, ctypes.byref(opts), ctypes.c_void_p(Eo.data_ptr()), ctypes.byref(st),
                            _stream(stream))
    _check(rc, allow_warning=allow_not_converged)
    return Eo, st.as_dict()


def thm_adjoint_grad(system, E, tgt_lo, tgt_hi, opts=None, stream=None):
    torch = _torch()
    opts = opts or default_opts()
    g = torch.empty(system.info["n_cells"], dtype=torch.float64, device="cuda")
    J = ctypes.c_double()
    lo = _d3(*[float(v) for v in (list(tgt_lo) + [0.0] * 3)[:3]])
    hi = _d3(*[float(v) for v in (list(tgt_hi) + [1.0] * 3)[:3]])
    _check(_lib.thm_adjoint_grad(system.handle, ctypes.c_void_p(_cvec(system.n, E).data_ptr()), lo, hi,
                                 ctypes.byref(opts), ctypes.c_void_p(g.data_ptr()), ctypes.byref(J),
                                 _stream(stream)))
    return g, J.value


def thm_system_release_workspaces(system):
    """Free the solve workspaces kept for the system (its matrices and factorisation stay)."""
    _check(_lib.thm_system_release_workspaces(system.handle))


def thm_system_set_mu(system, mu, stream=None):
    torch = _torch()
    mu = mu.detach().to(device="cuda", dtype=torch.float64).contiguous()
    _check(_lib.thm_system_set_mu(system.handle, ctypes.c_void_p(mu.data_ptr()), _stream(stream)))


def thm_apply_operator(system, x, transpose=False, precision=THM_FP64, stream=None):
    torch = _torch()
    y = torch.empty_like(_cvec(system.n, x))
    _check(_lib.thm_apply_operator(system.handle, int(bool(transpose)), int(precision),
                                   ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()), _stream(stream)))
    return y


def thm_apply_precond(system, x, precision=THM_FP64, stream=None):
    torch = _torch()
    y = torch.empty_like(_cvec(system.n, x))
    _check(_lib.thm_apply_precond(system.handle, int(precision), ctypes.c_void_p(x.data_ptr()),
                                  ctypes.c_void_p(y.data_ptr()), _stream(stream)))
    return y


def thm_apply_precond_noalloc(system, x, y, precision=THM_FP64, stream=None):
    """y = diag(K, K)^{-1} x into the caller's y, without any device allocation in the library
    (its work vectors live in a static device array); enqueued on the stream, not synchronised.
    The system's factor must exist (thm_apply_precond once first)."""
    _cvec(system.n, x)
    _cvec(system.n, y)
    _check(_lib.thm_apply_precond_noalloc(system.handle, int(precision), ctypes.c_void_p(x.data_ptr()),
                                          ctypes.c_void_p(y.data_ptr()), _stream(stream)))
    return y


def thm_apply_precond_full(system, x, transpose=False, precision=THM_FP64, stream=None):
    """y = (K + iC)^{-1} x, or (K - iC)^{-1} x with transpose (complete inverse, THM_PREC_FULL)."""
    torch = _torch()
    y = torch.empty_like(_cvec(system.n, x))
    _check(_lib.thm_apply_precond_full(system.handle, int(bool(transpose)), int(precision),
                                       ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                       _stream(stream)))
    return y


def thm_export_matrices(system):
    """Host copies of the assembled K and C (CSR, before the Dirichlet modification)."""
    i = system.info
    n, nnz, nnzc = i["n_dofs"], i["nnz"], i["nnz_c"]
    kr = np.zeros(n + 1, np.int32)
    kc = np.zeros(nnz, np.int32)
    kv = np.zeros(nnz, np.float64)
    cr = np.zeros(n + 1, np.int32)
    cc = np.zeros(max(nnzc, 1), np.int32)
    cv = np.zeros(max(nnzc, 1), np.float64)
    ptr = lambda a: ctypes.c_void_p(a.ctypes.data)
    _check(_lib.thm_export_matrices(system.handle, ptr(kr), ptr(kc), ptr(kv), ptr(cr), ptr(cc), ptr(cv)))
    return (kr, kc, kv), (cr, cc[:nnzc], cv[:nnzc])


def thm_export_rhs(system):
    n = system.n
    d = np.zeros(n, np.uint8)
    g = np.zeros(n, np.complex128)
    r = np.zeros(n, np.complex128)
    _check(_lib.thm_export_rhs(system.handle, ctypes.c_void_p(d.ctypes.data), ctypes.c_void_p(g.ctypes.data),
                               ctypes.c_void_p(r.ctypes.data)))
    return d, g, r


def thm_export_elements(system, c0, count, n_loc):
    out = np.zeros((count, n_loc, n_loc), np.float64)
    _check(_lib.thm_export_elements(system.handle, int(c0), int(count), ctypes.c_void_p(out.ctypes.data)))
    return out


def thm_time_spmv(system, precision=THM_FP64, reps=20, stream=None):
    ms = ctypes.c_double()
    by = ctypes.c_double()
    _check(_lib.thm_time_spmv(system.handle, int(precision), int(reps), ctypes.byref(ms), ctypes.byref(by),
                              _stream(stream)))
    return ms.value, by.value


def thm_time_spmv_batch(system, precision=THM_FP64, variant=-1, reps=20, stream=None):
    """(ms, algorithmic bytes) of one SpMV over the DDM's subdomain batch (after a DDM solve)."""
    ms = ctypes.c_double()
    by = ctypes.c_double()
    _check(_lib.thm_time_spmv_batch(system.handle, int(precision), int(variant), int(reps), ctypes.byref(ms),
                                    ctypes.byref(by), _stream(stream)))
    return ms.value, by.value


def thm_time_spmv_systems(systems, precision=THM_FP64, reps=20, stream=None):
    """(ms, algorithmic bytes) of one block SpMV over a batch of independent systems."""
    ns = len(systems)
    hs = (ctypes.c_void_p * ns)(*[s.handle.value for s in systems])
    ms = ctypes.c_double()
    by = ctypes.c_double()
    _check(_lib.thm_time_spmv_systems(ns, hs, int(precision), int(reps), ctypes.byref(ms), ctypes.byref(by),
                                      _stream(stream)))
    return ms.value, by.value


def thm_set_spmv_variant(system, precision, variant):
    """Pin the SpMV variant of the system's own context (-1: autotune again)."""
    _check(_lib.thm_set_spmv_variant(system.handle, int(precision), int(variant)))


def thm_time_precond(system, precision=THM_FP64, reps=20, stream=None):
    """(ms per application, algorithmic bytes per application, launches per application)."""
    ms = ctypes.c_double()
    by = ctypes.c_double()
    nl = ctypes.c_int32()
    _check(_lib.thm_time_precond(system.handle, int(precision), int(reps), ctypes.byref(ms), ctypes.byref(by),
                                 ctypes.byref(nl), _stream(stream)))
    return ms.value, by.value, nl.value


def _make_objective():
    torch = _torch()

    class ThmObjective(torch.autograd.Function):
        """J(mu) = int_T |E_h(mu)|^2 with the adjoint gradient in backward.

        forward(mu, system, tgt_lo, tgt_hi, opts) -> J (0-d float64 tensor)
        """

        @staticmethod
        def forward(ctx, mu, system, tgt_lo, tgt_hi, opts):
            thm_system_set_mu(system, mu)
            (E,), _ = thm_gmres_solve([system], opts)
            g, J = thm_adjoint_grad(system, E, tgt_lo, tgt_hi, opts)
            ctx.save_for_backward(g)
            return torch.tensor(J, dtype=torch.float64, device=mu.device)

        @staticmethod
        def backward(ctx, gJ):
            (g,) = ctx.saved_tensors
            return gJ * g, None, None, None, None

    return ThmObjective


class _Lazy:
    obj = None


def ThmObjective():
    """The torch.autograd.Function class (created on first use so that importing the
    binding does not import torch)."""
    if _Lazy.obj is None:
        _Lazy.obj = _make_objective()
    return _Lazy.obj
