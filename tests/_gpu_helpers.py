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
