"""Objective J = int_T |E_h|^2 and its exact discrete gradient in the per-cell mu.

Derivation (from eqs. (2)-(4)): S_FF E_F = -S_FD g_D with S = K + iC and g_D
independent of mu.  For J = E^H M_T E (M_T the mass matrix of the target box T):
    dJ = 2 Re((M_T E)_F^H dE_F),   dE_F = -S_FF^{-1} dS_{F,:} E.
With the adjoint state lambda solving S_FF^H lambda = (M_T E)_F (S^H = conj(S) =
K - iC since K, C are real symmetric: the transposed real block operator
[[K, C], [-C, K]]) and dS/dmu_c = -mu_c^{-2} Ahat_c:
    dJ/dmu_c = 2 mu_c^{-2} Re(lambda_c^H Ahat_c E_c),
lambda extended by zero on the Dirichlet DoFs.  C does not depend on mu.

M_T integrates exactly over cell n T (Gauss q = p+2 per axis on the clipped box).
"""
from dataclasses import replace

import numpy as np
import scipy.sparse as sp

from . import fe, system


def target_mass(sys, tlo, thi):
    mesh = sys.mesh
    d, p = mesh.dim, mesh.p
    q = p + 2
    x1, w1 = fe.gauss01(q)
    T = mesh.table()
    rows, cols, vals = [], [], []
    for c in range(mesh.n_cells):
        o = mesh.cell_origin(c)
        ta, tb = [], []
        ok = True
        for a in range(d):
            lo = max(tlo[a], o[a])
            hi = min(thi[a], o[a] + mesh.h[a])
            if hi <= lo:
                ok = False
                break
            ta.append((lo - o[a]) / mesh.h[a])
            tb.append((hi - o[a]) / mesh.h[a])
        if not ok:
            continue
        axes_pts = [ta[a] + (tb[a] - ta[a]) * x1 for a in range(d)]
        axes_w = [(tb[a] - ta[a]) * w1 for a in range(d)]
        grids = np.meshgrid(*axes_pts, indexing="ij")
        pts = np.stack([g.ravel() for g in grids], axis=1)
        W = axes_w[0]
        for a in range(1, d):
            W = np.multiply.outer(W, axes_w[a])
        W = W.ravel()
        vals_ref, _ = fe.ref_eval(d, p, pts)
        pv = vals_ref / mesh.h[None, :, None]
        Mc = np.einsum("uaq,vaq,q->uv", pv, pv, W) * np.prod(mesh.h)
        nl = Mc.shape[0]
        rows.append(np.repeat(T[c], nl))
        cols.append(np.tile(T[c], nl))
        vals.append(Mc.ravel())
    N = mesh.n_dofs
    if not rows:
        return sp.csr_matrix((N, N))
    return sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                         shape=(N, N)).tocsr()


def objective(sys, E, MT):
    return float(np.real(np.vdot(E, MT @ E)))


def gradient(sys, E, MT):
    """Exact discrete dJ/dmu per cell by one adjoint (conjugate) solve."""
    F = sys.F
    rhs = (MT @ E)[F]
    lam = np.zeros(sys.n, dtype=np.complex128)
    lam[F] = system.lu_factor(sys, conj=True)(rhs)
    T = sys.T
    Ec = E[T]
    Lc = lam[T]
    bil = np.real(np.einsum("cu,uv,cv->c", Lc.conj(), sys.Ahat, Ec))
    return 2.0 * bil / sys.mu ** 2, lam


def fd_gradient(prob, cells, tlo, thi, rel=1e-5):
    """Central finite differences of J with fresh LU solves (h_c = rel * mu_c)."""
    mesh = prob.mesh()
    mu0 = prob.mu_cells(mesh.n_cells).copy()
    out = []
    MT = None
    for c in cells:
        h = rel * mu0[c]
        Js = []
        for sgn in (+1, -1):
            mu = mu0.copy()
            mu[c] += sgn * h
            s = system.assemble(replace(prob, mu=mu))
            if MT is None:
                MT = target_mass(s, tlo, thi)
            E = system.solve_lu(s)
            Js.append(objective(s, E, MT))
        out.append((Js[0] - Js[1]) / (2 * h))
    return np.array(out)
