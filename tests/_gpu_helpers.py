"""Shared helpers of the GPU parity tests: oracle reference quantities on the same inputs."""
import numpy as np
import scipy.sparse as sp

from oracle import system
from oracle.system import Problem


def problem(d):
    return Problem(**d)


def spec(dim, m, p, omega, **kw):
    d = dict(dim=dim, n=(m,) * dim + (1,) * (3 - dim), p=p, omega=float(omega), kappa=1.0, mu=None, inc_faces=1,
             inc_dir=(1.0, 0.0, 0.0), inc_pol=(0.0, 1.0, 0.0), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
             subdomains=(1, 1, 1))
    d.update(kw)
    return d


def csr(parts, n):
    rp, c, v = parts
    return sp.csr_matrix((v, c, rp), shape=(n, n))


def dirichletized(sys_o):
    """Oracle real block operator with Dirichlet rows/columns as identity (complex form)."""
    n = sys_o.n
    D = np.zeros(n, bool)
    D[sys_o.D] = True
    keep = sp.diags((~D).astype(float))
    S = keep @ sys_o.S @ keep + sp.diags(D.astype(float))
    return S.tocsr(), D


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


# Parity protocol for solves that stop on a residual: FP64 runs to rtol 1e-13 (or until the
# outer iteration stagnates) and must match the oracle to 1e-10; FP32 inner solves with FP64
# refinement run to 1e-11 and must match to 1e-8.
FP64_TIGHT = dict(rtol=1e-13, inner_rtol=1e-13)
MIXED_TIGHT = dict(rtol=1e-11, inner_rtol=1e-11)


def ddm_fp64(thm, S, **kw):
    """DDM solve under the FP64 protocol; returns (host field, stats)."""
    o = thm.default_opts(**dict(FP64_TIGHT, **kw))
    E, st = thm.thm_ddm_solve(S, o, allow_not_converged=True)
    return E.cpu().numpy(), st


def ddm_mixed(thm, S, **kw):
    o = thm.default_opts(**dict(MIXED_TIGHT, precision=thm.THM_FP32_IR, **kw))
    E, st = thm.thm_ddm_solve(S, o, allow_not_converged=True)
    return E.cpu().numpy(), st


# ---- oracle work in worker processes (CPU only; they never touch the GPU)
def _oracle_lu(d):
    return system.solve_lu(system.assemble(Problem(**d)))


def _oracle_residual(args):
    d, E = args
    return system.relative_residual(system.assemble(Problem(**d)), E)


def oracle_map(fn, items, workers=None):
    """fn over items in fresh worker processes (spawned, one BLAS thread each, at most 12)."""
    import multiprocessing as mp
    import os
    workers = workers or max(1, min(12, len(os.sched_getaffinity(0)), len(items)))
    keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in keep:
        os.environ[k] = "1"
    try:
        with mp.get_context("spawn").Pool(workers) as pool:
            return pool.map(fn, items, chunksize=1)
    finally:
        for k, v in keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def oracle_solutions(specs):
    return oracle_map(_oracle_lu, list(specs))


def oracle_residuals(specs, fields):
    return oracle_map(_oracle_residual, list(zip(specs, fields)))
