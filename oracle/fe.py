"""Reference Nedelec (first kind, tensor product) basis and element matrices.

Paper, Sec. 2: the discrete space is the Nedelec space N_h^p with a hierarchical
basis built from the de Rham complex (Zaglmayr).  The printed space formula is the
tetrahedral one; on quads/hexes we use the tensor-product first-kind space
Q_{p,p+1} x Q_{p+1,p} (2D) and Q_{p,p+1,p+1} x ... (3D), degree p = 0 lowest order.

1D families on t in [0,1]:
  tangential  L_i(t) = P_i(2t-1),                 i = 0..p   (shifted Legendre)
  normal      l_0 = 1-t, l_1 = t,
              l_j(t) = int_0^t P_{j-1}(2s-1) ds,  j = 2..p+1 (integrated Legendre)
  with l_0' = -L_0, l_1' = L_0, l_j' = L_{j-1}.

Shape function of component a:  L_i(t_a) * prod over the other axes b of l_{j_b}(t_b).
Entity association: every normal index in {0,1} -> edge; exactly one >= 2 -> face
(3D); all >= 2 -> cell interior.

Local DoF order (reference cell [0,1]^d):
 2D: edges bottom (x-comp, eta-side 0), top (x-comp, eta-side 1), left (y-comp,
     xi-side 0), right (y-comp, xi-side 1), p+1 each ordered by i; then interior
     x-comp then y-comp, each ordered (j-2)*(p+1)+i.
 3D: 12 edges, component a in x,y,z, with the two normal axes (b<c) at sides
     (jb, kc) ordered 2*jb+kc, p+1 each ordered by i; then 6 faces ordered
     2*normal_axis+side, inside a face the two tangential components in
     increasing axis order, each ordered (bubble-2)*(p+1)+i; then interior
     components x,y,z each ordered ((jb-2)*p+(kc-2))*(p+1)+i.

Physical cells are axis-aligned boxes of size h = (h_x, h_y[, h_z]); the map is
affine with J = diag(h) and the covariant Piola map phi = J^{-T} phi_hat, so
component a is divided by h_a and curl phi = J curl_hat phi_hat / det J.

Element matrices (eq. (3)): M_uv = int phi_u . phi_v,  A_uv = mu^{-1} int curl phi_u . curl phi_v.
Quadrature: Gauss-Legendre with q = p+2 points per axis (exact for these
polynomial integrands on affine cells).
"""
import numpy as np
from numpy.polynomial import legendre as _npleg


def gauss01(q):
    """Gauss-Legendre nodes and weights on [0,1] (library primitive)."""
    x, w = _npleg.leggauss(q)
    return 0.5 * (x + 1.0), 0.5 * w


def legendre_all(n, u):
    """P_0..P_n at points u (three-term recurrence); shape (n+1, len(u))."""
    u = np.asarray(u, dtype=np.float64)
    P = np.zeros((max(n, 0) + 1,) + u.shape)
    P[0] = 1.0
    if n >= 1:
        P[1] = u
    for k in range(1, n):
        P[k + 1] = ((2 * k + 1) * u * P[k] - k * P[k - 1]) / (k + 1)
    return P


def fam_L(p, t):
    """Tangential family L_i(t) = P_i(2t-1), i=0..p; shape (p+1, len(t))."""
    return legendre_all(p, 2.0 * np.asarray(t) - 1.0)


def fam_l(p, t):
    """Normal family l_j(t), j = 0..p+1, and derivatives; shapes (p+2, len(t)).

    l_j for j >= 2 uses int_{-1}^{u} P_n = (P_{n+1}(u) - P_{n-1}(u)) / (2n+1), u = 2t-1,
    n = j-1, with the factor 1/2 from ds = du/2.
    """
    t = np.asarray(t, dtype=np.float64)
    u = 2.0 * t - 1.0
    P = legendre_all(p + 1, u)
    v = np.zeros((p + 2,) + t.shape)
    d = np.zeros((p + 2,) + t.shape)
    v[0] = 1.0 - t
    v[1] = t
    d[0] = -1.0
    d[1] = 1.0
    for j in range(2, p + 2):
        v[j] = (P[j] - P[j - 2]) / (2.0 * (2 * j - 1))
        d[j] = P[j - 1]
    return v, d


# ---------------------------------------------------------------- local enumeration

def local_functions(dim, p):
    """List of shape functions in local DoF order.

    2D entries: (comp, i, j)   meaning L_i(t_comp) * l_j(t_other)
    3D entries: (comp, i, jb, kc) meaning L_i(t_comp) l_jb(t_b) l_kc(t_c), (b<c) the
    two axes other than comp.
    """
    out = []
    if dim == 2:
        for comp, side in ((0, 0), (0, 1), (1, 0), (1, 1)):
            for i in range(p + 1):
                out.append((comp, i, side))
        for comp in (0, 1):
            for j in range(2, p + 2):
                for i in range(p + 1):
                    out.append((comp, i, j))
        return out
    # 3D edges
    for comp in range(3):
        for jb in (0, 1):
            for kc in (0, 1):
                for i in range(p + 1):
                    out.append((comp, i, jb, kc))
    # 3D faces
    for n in range(3):
        for side in (0, 1):
            tang = [a for a in range(3) if a != n]
            for comp in tang:
                other = [a for a in range(3) if a != comp]  # (b, c) sorted
                m = [a for a in tang if a != comp][0]       # axis carrying the bubble
                for bub in range(2, p + 2):
                    for i in range(p + 1):
                        idx = {n: side, m: bub}
                        out.append((comp, i, idx[other[0]], idx[other[1]]))
    # 3D interior
    for comp in range(3):
        for jb in range(2, p + 2):
            for kc in range(2, p + 2):
                for i in range(p + 1):
                    out.append((comp, i, jb, kc))
    return out


def n_local(dim, p):
    return 2 * (p + 1) * (p + 2) if dim == 2 else 3 * (p + 1) * (p + 2) ** 2


def n_interior(dim, p):
    return 2 * p * (p + 1) if dim == 2 else 3 * p * p * (p + 1)


# ---------------------------------------------------------------- reference tables

def ref_eval(dim, p, pts):
    """Reference basis values and reference curls at points.

    pts: (npts, dim) in [0,1]^dim.
    returns vals (n_loc, dim, npts), curls (n_loc, ncurl, npts) with ncurl = 1 (2D) or 3.
    """
    pts = np.atleast_2d(pts)
    funcs = local_functions(dim, p)
    nl = len(funcs)
    npts = pts.shape[0]
    Lv = [fam_L(p, pts[:, a]) for a in range(dim)]
    lv = [fam_l(p, pts[:, a]) for a in range(dim)]
    vals = np.zeros((nl, dim, npts))
    curls = np.zeros((nl, 1 if dim == 2 else 3, npts))
    for u, f in enumerate(funcs):
        if dim == 2:
            comp, i, j = f
            o = 1 - comp
            val = Lv[comp][i] * lv[o][0][j]
            vals[u, comp] = val
            # curl_hat = d_xi f_y - d_eta f_x
            dother = Lv[comp][i] * lv[o][1][j]  # derivative along the other axis
            curls[u, 0] = dother if comp == 1 else -dother
        else:
            comp, i, jb, kc = f
            b, c = [a for a in range(3) if a != comp]
            val = Lv[comp][i] * lv[b][0][jb] * lv[c][0][kc]
            vals[u, comp] = val
            db = Lv[comp][i] * lv[b][1][jb] * lv[c][0][kc]  # d/dt_b of the component
            dc = Lv[comp][i] * lv[b][0][jb] * lv[c][1][kc]  # d/dt_c
            # curl_hat_r = eps_{r s t} d_s f_t ; here only f_comp != 0
            # contribution of d_b f_comp to curl component r with eps_{r b comp}
            for s, dv in ((b, db), (c, dc)):
                r = 3 - s - comp
                eps = _levi(r, s, comp)
                curls[u, r] += eps * dv
    return vals, curls


def _levi(i, j, k):
    return (i - j) * (j - k) * (k - i) / 2


def tensor_quad(dim, q):
    x, w = gauss01(q)
    if dim == 2:
        X, Y = np.meshgrid(x, x, indexing="ij")
        W = np.outer(w, w)
        return np.stack([X.ravel(), Y.ravel()], axis=1), W.ravel()
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")
    W = np.einsum("i,j,k->ijk", w, w, w)
    return np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1), W.ravel()


def element_matrices(dim, p, h, q=None):
    """Mass M and unit-coefficient curl-curl A_hat for a box cell of size h (eq. (3)).

    The returned curl-curl matrix is for mu = 1; the cell's A is A_hat / mu_c.
    """
    h = np.asarray(h, dtype=np.float64)
    if q is None:
        q = p + 2
    pts, w = tensor_quad(dim, q)
    vals, curls = ref_eval(dim, p, pts)
    det = np.prod(h)
    # covariant Piola: component a scaled by 1/h_a
    pv = vals / h[None, :, None]
    M = np.einsum("uaq,vaq,q->uv", pv, pv, w) * det
    if dim == 2:
        pc = curls / det
    else:
        pc = curls * h[None, :, None] / det
    A = np.einsum("uaq,vaq,q->uv", pc, pc, w) * det
    return M, A


# ---------------------------------------------------------------- boundary traces

def face_functions(dim, p, axis, side):
    """Local DoFs whose tangential trace is nonzero on the reference side {t_axis = side}."""
    funcs = local_functions(dim, p)
    out = []
    for u, f in enumerate(funcs):
        comp = f[0]
        if comp == axis:
            continue  # purely normal component on this side: zero tangential trace
        if dim == 2:
            j = f[2]
            if j == side:
                out.append(u)
        else:
            b, c = [a for a in range(3) if a != comp]
            idx = {b: f[2], c: f[3]}
            if idx[axis] == side:
                out.append(u)
    return out


def side_points(dim, axis, side, q):
    """Quadrature on the reference side {t_axis = side}: points (npts, dim), weights."""
    x, w = gauss01(q)
    if dim == 2:
        pts = np.zeros((q, 2))
        pts[:, axis] = side
        pts[:, 1 - axis] = x
        return pts, w
    t1, t2 = [a for a in range(3) if a != axis]
    X, Y = np.meshgrid(x, x, indexing="ij")
    pts = np.zeros((q * q, 3))
    pts[:, axis] = side
    pts[:, t1] = X.ravel()
    pts[:, t2] = Y.ravel()
    return pts, np.outer(w, w).ravel()


def side_mass(dim, p, h, axis, side, q=None):
    """Tangential trace mass int_side gamma^T phi_u . gamma^T phi_v ds (all local DoFs).

    On an axis-aligned side the tangential trace is the vector of the components
    along the other axes; surface measure = prod of the tangential h.
    """
    h = np.asarray(h, dtype=np.float64)
    if q is None:
        q = p + 2
    pts, w = side_points(dim, axis, side, q)
    vals, _ = ref_eval(dim, p, pts)
    pv = vals / h[None, :, None]
    tang = [a for a in range(dim) if a != axis]
    ds = np.prod(h[tang])
    return np.einsum("uaq,vaq,q->uv", pv[:, tang], pv[:, tang], w) * ds


def side_load(dim, p, h, x0, axis, side, Einc, q=10):
    """Load s_u = int_side gamma^T(E^inc) . gamma^T(phi_u) ds for every local DoF.

    Einc(x) -> complex array (npts, dim) of the field at physical points x (npts, dim).
    """
    h = np.asarray(h, dtype=np.float64)
    pts, w = side_points(dim, axis, side, q)
    vals, _ = ref_eval(dim, p, pts)
    pv = vals / h[None, :, None]
    xphys = np.asarray(x0)[None, :] + pts * h[None, :]
    E = Einc(xphys)  # (npts, dim)
    tang = [a for a in range(dim) if a != axis]
    ds = np.prod(h[tang])
    return np.einsum("uaq,qa,q->u", pv[:, tang], E[:, tang], w) * ds
