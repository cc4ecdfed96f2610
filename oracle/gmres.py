"""Plain restarted GMRES with right preconditioning (oracle side).

Paper Sec. 3.2: GMRES, preconditioned by the block-diagonal operator of eq. (11),
diag(A - w^2 M, A - w^2 M)^{-1}; relative accuracy 1e-8 (Sec. 4.1).  Readings:
right preconditioning, restart m, x0 = 0, stop on ||b - A x|| / ||b|| <= rtol.
Modified Gram-Schmidt and complex Givens rotations; written for clarity.

Givens convention: G = [[c, s], [-conj(s), c]], c real >= 0, chosen so that
G [a; b] = [r; 0].
"""
import numpy as np


def _givens(a, b):
    den = np.sqrt(abs(a) ** 2 + abs(b) ** 2)
    if den == 0.0:
        return 1.0, 0.0, 0.0
    if a == 0:
        return 0.0, 1.0, b
    c = abs(a) / den
    s = (a / abs(a)) * np.conj(b) / den
    r = (a / abs(a)) * den
    return c, s, r


def gmres(apply_A, b, apply_Minv=None, rtol=1e-8, restart=50, max_iter=5000, x0=None):
    """Solve A x = b. Returns (x, iterations, relative residual history)."""
    b = np.asarray(b)
    dtype = np.complex128 if np.iscomplexobj(b) else np.float64
    n = b.size
    x = np.zeros(n, dtype=dtype) if x0 is None else np.array(x0, dtype=dtype)
    Minv = (lambda v: v) if apply_Minv is None else apply_Minv
    bnorm = np.linalg.norm(b)
    hist = []
    if bnorm == 0.0:
        return np.zeros(n, dtype=dtype), 0, [0.0]
    it = 0
    while True:
        r = b - apply_A(x)
        beta = np.linalg.norm(r)
        hist.append(beta / bnorm)
        if beta / bnorm <= rtol or it >= max_iter:
            break
        m = min(restart, max_iter - it)
        V = np.zeros((n, m + 1), dtype=dtype)
        H = np.zeros((m + 1, m), dtype=dtype)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=dtype)
        g = np.zeros(m + 1, dtype=dtype)
        g[0] = beta
        V[:, 0] = r / beta
        k = 0
        for j in range(m):
            w = apply_A(Minv(V[:, j]))
            for i in range(j + 1):
                H[i, j] = np.vdot(V[:, i], w)
                w = w - H[i, j] * V[:, i]
            hn = np.linalg.norm(w)
            H[j + 1, j] = hn
            if hn != 0.0:
                V[:, j + 1] = w / hn
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -np.conj(sn[i]) * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            cs[j], sn[j], H[j, j] = _givens(H[j, j], H[j + 1, j])
            H[j + 1, j] = 0.0
            g[j + 1] = -np.conj(sn[j]) * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            k = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) / bnorm <= rtol or hn == 0.0:
                break
        y = np.linalg.solve(np.triu(H[:k, :k]), g[:k])
        x = x + Minv(V[:, :k] @ y)
    return x, it, hist
