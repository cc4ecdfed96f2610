"""Pins of the oracle's reference basis and element matrices (Sec. 2, eq. (3))."""
import numpy as np
import pytest

from oracle import fe
from tests._golden import read_blocks


def test_appendix_b_2d_lowest_order():
    g = read_blocks("appendix_b_2d_p0.txt")
    for h, mu in ((1.0, 1.0), (1.0 / 16, 1.0), (0.37, 2.5)):
        M, A = fe.element_matrices(2, 0, [h, h])
        assert np.allclose(6 * M, g["M"], atol=1e-14, rtol=0)
        assert np.allclose(mu * h * h * (A / mu), g["A"], atol=1e-13, rtol=0)


def test_appendix_b_3d_lowest_order():
    g = read_blocks("appendix_b_3d_p0.txt")
    for h in (1.0, 0.25):
        M, A = fe.element_matrices(3, 0, [h, h, h])
        assert np.allclose(36 / h * M, g["M"], atol=1e-13, rtol=0)
        assert np.allclose(6 * h * A, g["A"], atol=1e-13, rtol=0)


@pytest.mark.parametrize("dim,p", [(2, 0), (2, 1), (2, 2), (2, 3), (3, 0), (3, 1), (3, 2)])
def test_element_symmetry_definiteness_and_rule_independence(dim, p):
    h = [0.3, 0.7, 0.45][:dim]
    M, A = fe.element_matrices(dim, p, h)
    assert M.shape == (fe.n_local(dim, p),) * 2
    assert np.abs(M - M.T).max() <= 1e-15 * np.abs(M).max()
    assert np.abs(A - A.T).max() <= 1e-14 * np.abs(A).max()
    assert np.linalg.eigvalsh(M).min() > 0
    assert np.linalg.eigvalsh(A).min() > -1e-10 * np.abs(A).max()
    M2, A2 = fe.element_matrices(dim, p, h, q=p + 5)
    assert np.abs(M - M2).max() <= 1e-14 * np.abs(M).max()
    assert np.abs(A - A2).max() <= 1e-13 * np.abs(A).max()


def test_normal_family_is_integrated_legendre():
    t = np.linspace(0, 1, 41)
    for p in range(5):
        v, d = fe.fam_l(p, t)
        L = fe.fam_L(p + 1, t)
        assert np.allclose(v[:, 0], [1, 0] + [0] * p, atol=1e-15)
        assert np.allclose(v[:, -1], [0, 1] + [0] * p, atol=1e-15)
        assert np.allclose(d[0], -L[0]) and np.allclose(d[1], L[0])
        for j in range(2, p + 2):
            assert np.allclose(d[j], L[j - 1], atol=1e-14)
            eps = 1e-6
            vp, _ = fe.fam_l(p, t + eps)
            vm, _ = fe.fam_l(p, t - eps)
            assert np.allclose((vp[j] - vm[j]) / (2 * eps), d[j], atol=1e-8)


@pytest.mark.parametrize("dim,p", [(2, 0), (2, 2), (3, 0), (3, 1)])
def test_constant_field_is_reproduced(dim, p):
    """A constant field (a, b[, c]) has DoFs a_axis*h on the L_0 edge functions only."""
    h = np.array([0.5, 0.25, 0.75][:dim])
    funcs = fe.local_functions(dim, p)
    coef = np.array([1.3, -0.7, 2.1][:dim])
    u = np.zeros(len(funcs))
    for k, f in enumerate(funcs):
        comp, i = f[0], f[1]
        rest = f[2:]
        if i == 0 and all(r in (0, 1) for r in rest):
            u[k] = coef[comp] * h[comp]
    # value check at random points: sum of covariant-Piola functions equals the constant
    pts = np.random.default_rng(0).random((7, dim))
    vals, curls = fe.ref_eval(dim, p, pts)
    field = np.einsum("u,uaq->qa", u, vals / h[None, :, None])
    assert np.allclose(field, coef[None, :], atol=1e-14)
    M, A = fe.element_matrices(dim, p, h)
    assert np.isclose(u @ M @ u, np.prod(h) * (coef ** 2).sum(), rtol=1e-14)
    assert np.abs(A @ u).max() < 1e-12


def test_local_gradient_has_zero_curl():
    """Discrete de Rham on one cell: gradients of Q_{p+1} functions are curl free.

    The gradient of l_a(xi) l_b(eta) is written in the Nedelec basis with
    coefficients in {0, +-1} (l_0' = -L_0, l_1' = L_0, l_j' = L_{j-1}); A_c G_c = 0.
    """
    for dim, pmax in ((2, 3), (3, 2)):
        for p in range(pmax + 1):
            funcs = fe.local_functions(dim, p)
            index = {f: k for k, f in enumerate(funcs)}
            cols = []
            for ab in np.ndindex(*(p + 2,) * dim):
                g = np.zeros(len(funcs))
                for comp in range(dim):
                    a = ab[comp]
                    i, s = (0, -1.0) if a == 0 else (0, 1.0) if a == 1 else (a - 1, 1.0)
                    others = tuple(ab[b] for b in range(dim) if b != comp)
                    g[index[(comp, i) + others]] += s
                cols.append(g)
            G = np.array(cols).T
            h = [0.4, 0.9, 0.6][:dim]
            M, A = fe.element_matrices(dim, p, h)
            assert np.abs(A @ G).max() < 1e-11 * np.abs(A).max()
            # the gradient field itself: check against a finite difference of psi
            pts = np.random.default_rng(1).random((5, dim))
            vals, _ = fe.ref_eval(dim, p, pts)
            hh = np.asarray(h)
            for k, ab in enumerate(np.ndindex(*(p + 2,) * dim)):
                field = np.einsum("u,uaq->qa", G[:, k], vals / hh[None, :, None])
                for comp in range(dim):
                    eps = 1e-6
                    def psi(x):
                        out = np.ones(x.shape[0])
                        for b in range(dim):
                            out *= fe.fam_l(p, x[:, b])[0][ab[b]]
                        return out
                    xp = pts.copy(); xp[:, comp] += eps
                    xm = pts.copy(); xm[:, comp] -= eps
                    fd = (psi(xp) - psi(xm)) / (2 * eps) / hh[comp]
                    assert np.allclose(field[:, comp], fd, atol=1e-7)
