"""Global discrete system of the time-harmonic Maxwell problem (oracle side).

Paper eq. (1): curl(mu^{-1} curl E) - w^2 E = 0 in Omega,
               mu^{-1} g^t(curl E) - i k w g^T(E) = 0 on Gamma^inf,
               g^T(E) = g^T(E^inc) on Gamma^inc.
Weak form (eq. (2)) and elementary integrals (eq. (3)) give the complex symmetric
matrix S = K + iC with
    K = A - w^2 M   (A: mu^{-1} curl-curl, M: mass; real symmetric, indefinite)
    C = k w M_inf   (tangential trace mass on Gamma^inf; real symmetric PSD).
Readings of the paper used here:
 * materials of refractive index n (the block benchmark of Sec. 4.1) enter as a relative
   permittivity eps = n^2 per cell in the mass term, curl(mu^{-1} curl E) - w^2 eps E = 0,
   so M is the eps-weighted mass (the paper's equations carry mu only; eps = 1 there);
 * the impedance coefficient is i k w without mu (the strong form's coefficient;
   integration by parts of eq. (1) gives exactly +i k w int g^T E . g^T phi);
 * B of eq. (4) is real (the i is factored out): S = K + iC <-> [[K, -C], [C, K]];
 * Gamma^inc is a strong Dirichlet boundary: the Dirichlet values g_D are the
   boundary L2 projection of g^T(E^inc) on the closure of Gamma^inc (the paper's
   load s_u is exactly the right-hand side of that projection); test functions
   vanish there and the data are lifted: S_FF E_F = -S_FD g_D;
 * E^inc(x) = pol * exp(-i w d.x) (time factor e^{i w t}, outgoing e^{-i w x}).
"""
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fe
from .mesh import BoxMesh


@dataclass
class Problem:
    dim: int
    n: tuple
    p: int
    omega: float
    kappa: float = 1.0
    mu: np.ndarray = None            # per cell, x fastest; None -> 1
    inc_faces: int = 1               # bit 2*axis+side -> Gamma^inc; other sides Gamma^inf
    inc_dir: tuple = (1.0, 0.0, 0.0)
    inc_pol: tuple = (0.0, 1.0, 0.0)  # complex allowed
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    subdomains: tuple = (1, 1, 1)
    eps: np.ndarray = None           # relative permittivity per cell (refractive index squared); None -> 1
    transmission: complex = 1.0      # DDM: transmission operator S = s 1 on interfaces (eq. (10): s = 1)

    def mesh(self):
        return BoxMesh(self.dim, self.n, self.lo, self.hi, self.p)

    def mu_cells(self, n_cells):
        if self.mu is None:
            return np.ones(n_cells)
        mu = np.asarray(self.mu, dtype=np.float64).ravel()
        assert mu.size == n_cells
        return mu

    def eps_cells(self, n_cells):
        if self.eps is None:
            return np.ones(n_cells)
        eps = np.asarray(self.eps, dtype=np.float64).ravel()
        assert eps.size == n_cells
        return eps

    def einc(self):
        d = np.asarray(self.inc_dir[: self.dim], dtype=np.float64)
        pol = np.asarray(self.inc_pol[: self.dim], dtype=np.complex128)
        w = self.omega

        def E(x):
            phase = np.exp(-1j * w * (x @ d))
            return phase[:, None] * pol[None, :]

        return E


def _coo(T, blocks):
    """COO triplets from per-cell dense blocks (n_cells, n_loc, n_loc)."""
    nl = T.shape[1]
    rows = np.repeat(T, nl, axis=1).ravel()
    cols = np.tile(T, (1, nl)).ravel()
    return rows, cols, blocks.ravel()


@dataclass
class System:
    prob: Problem
    mesh: BoxMesh
    T: np.ndarray          # cell -> DoF table
    mu: np.ndarray         # per cell
    Mhat: np.ndarray       # element mass (uniform box)
    Ahat: np.ndarray       # element unit-coefficient curl-curl
    K: sp.csr_matrix
    M: sp.csr_matrix       # eps-weighted mass
    A: sp.csr_matrix
    Minf: sp.csr_matrix
    C: sp.csr_matrix
    D: np.ndarray          # Dirichlet DoFs (sorted)
    gD: np.ndarray         # complex values on D
    F: np.ndarray          # free DoFs (sorted)
    extra: dict = field(default_factory=dict)

    @property
    def S(self):
        return (self.K + 1j * self.C).tocsr()

    @property
    def n(self):
        return self.mesh.n_dofs

    def full(self, EF):
        E = np.zeros(self.n, dtype=np.complex128)
        E[self.F] = EF
        E[self.D] = self.gD
        return E

    def rhs_free(self):
        """f_F = -S_FD g_D (eq. (4) right-hand side after lifting)."""
        S = self.S
        return -(S[self.F][:, self.D] @ self.gD)


def side_list(dim, inc_faces):
    inc, inf = [], []
    for axis in range(dim):
        for side in (0, 1):
            (inc if (inc_faces >> (2 * axis + side)) & 1 else inf).append((axis, side))
    return inc, inf


def side_matrix(mesh, axis, side, weight=1.0):
    """Assembled tangential trace mass on one box side (N x N, sparse)."""
    T = mesh.table()
    cells = mesh.side_cells(axis, side)
    Ms = fe.side_mass(mesh.dim, mesh.p, mesh.h, axis, side) * weight
    blocks = np.broadcast_to(Ms, (len(cells),) + Ms.shape)
    r, c, v = _coo(T[cells], np.ascontiguousarray(blocks))
    return sp.coo_matrix((v, (r, c)), shape=(mesh.n_dofs, mesh.n_dofs)).tocsr()


def dirichlet_data(prob, mesh, inc_sides):
    """Boundary L2 projection of g^T(E^inc) on the closure of Gamma^inc."""
    N = mesh.n_dofs
    if not inc_sides:
        return np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.complex128)
    T = mesh.table()
    Minc = sp.csr_matrix((N, N))
    s = np.zeros(N, dtype=np.complex128)
    E = prob.einc()
    for axis, side in inc_sides:
        Minc = Minc + side_matrix(mesh, axis, side)
        loc = np.arange(mesh.n_loc)
        for c in mesh.side_cells(axis, side):
            x0 = mesh.cell_origin(c)
            s_loc = fe.side_load(mesh.dim, mesh.p, mesh.h, x0, axis, side, E)
            np.add.at(s, T[c, loc], s_loc)
    D = np.unique(np.concatenate([mesh.side_dofs(a, sd) for a, sd in inc_sides]))
    MDD = Minc[D][:, D].tocsc()
    gD = spla.spsolve(MDD, s[D]) if len(D) > 1 else s[D] / MDD.toarray().ravel()
    return D, np.atleast_1d(np.asarray(gD, dtype=np.complex128))


def assemble(prob, extra_inf_sides=()):
    """Assemble K, M, A, C and the Dirichlet data of eq. (4).

    extra_inf_sides: additional sides (axis, side) carrying an impedance mass
    (used by the domain decomposition for interface sides).
    """
    mesh = prob.mesh()
    T = mesh.table()
    N = mesh.n_dofs
    mu = prob.mu_cells(mesh.n_cells)
    Mh, Ah = fe.element_matrices(mesh.dim, mesh.p, mesh.h)
    nc = mesh.n_cells
    # mass weighted by the cell's relative permittivity (K = A - w^2 M_eps; eps = 1 is eq. (3))
    Mb = Mh[None, :, :] * prob.eps_cells(nc)[:, None, None]
    Ab = Ah[None, :, :] / mu[:, None, None]
    r, c, v = _coo(T, np.ascontiguousarray(Mb))
    M = sp.coo_matrix((v, (r, c)), shape=(N, N)).tocsr()
    r, c, v = _coo(T, Ab)
    A = sp.coo_matrix((v, (r, c)), shape=(N, N)).tocsr()
    K = (A - prob.omega ** 2 * M).tocsr()
    inc, inf = side_list(mesh.dim, prob.inc_faces)
    Minf = sp.csr_matrix((N, N))
    for axis, side in inf:
        Minf = Minf + side_matrix(mesh, axis, side)
    C = (prob.kappa * prob.omega) * Minf
    for axis, side in extra_inf_sides:
        C = C + (prob.kappa * prob.omega) * side_matrix(mesh, axis, side)
    D, gD = dirichlet_data(prob, mesh, inc)
    F = np.setdiff1d(np.arange(N), D)
    return System(prob, mesh, T, mu, Mh, Ah, K.tocsr(), M, A, Minf.tocsr(), C.tocsr(), D, gD, F)


def nested_dissection(mesh, dofs):
    """Fill-reducing order of `dofs` for the sparse LU (an ordering only: the solve is the same
    linear system).  The box of cells is cut in halves along its longest axis at a mesh plane;
    the DoFs on entities inside that plane separate the two halves (no cell holds DoFs of both),
    so they are ordered after the two halves, each ordered the same way recursively."""
    X = mesh.dof_positions2()[dofs]
    out = []

    def rec(idx, lo, hi):
        span = (hi - lo) // 2
        a = int(np.argmax(span))
        if span[a] <= 1 or len(idx) < 64:
            out.append(idx)
            return
        cut = lo[a] + 2 * (span[a] // 2)
        c = X[idx, a]
        hi1, lo2 = hi.copy(), lo.copy()
        hi1[a] = lo2[a] = cut
        rec(idx[c < cut], lo, hi1)
        rec(idx[c > cut], lo2, hi)
        out.append(idx[c == cut])

    rec(np.arange(len(dofs)), np.zeros(mesh.dim, np.int64), 2 * np.asarray(mesh.n, np.int64))
    perm = np.concatenate(out)
    assert len(perm) == len(dofs)
    return perm


def lu_factor(sys, conj=False, refine=3):
    """SuperLU factorisation of S_FF (or conj(S_FF)) with the unknowns in nested-dissection
    order (threshold partial pivoting, threshold 0.1).  Returns solve(rhs_F) -> x_F: the LU
    solution followed by up to `refine` steps of iterative refinement with the same factors
    (x += LU^{-1}(b - S_FF x), while the residual keeps falling), so that ill-conditioned systems
    (near-resonant cavities of the uneven batch) are still solved to rounding level rather than
    to the accuracy of a threshold-pivoted LU."""
    perm = nested_dissection(sys.mesh, sys.F)
    SFF = sys.S[sys.F][:, sys.F]
    if conj:
        SFF = SFF.conj()
    SFF = SFF.tocsr()
    lu = spla.splu(SFF[perm][:, perm].tocsc(), permc_spec="NATURAL", diag_pivot_thresh=0.1,
                   options=dict(SymmetricMode=True))

    def lu_solve(b):
        y = lu.solve(b[perm])
        x = np.empty_like(y)
        x[perm] = y
        return x

    def solve(b):
        b = np.asarray(b, dtype=np.complex128)
        x = lu_solve(b)
        r = b - SFF @ x
        rn = np.linalg.norm(r)
        for _ in range(refine):
            x1 = x + lu_solve(r)
            r1 = b - SFF @ x1
            rn1 = np.linalg.norm(r1)
            if not rn1 < rn:
                break
            x, r, rn = x1, r1, rn1
        return x

    return solve


def solve_lu(sys):
    """E = [S_FF^{-1}(-S_FD g_D); g_D] by sparse LU (SuperLU)."""
    return sys.full(lu_factor(sys)(sys.rhs_free()))


def solve_dense(sys):
    """Same solution by a dense complex solve (brute force, tiny meshes only)."""
    S = sys.S.toarray()
    F, D = sys.F, sys.D
    EF = np.linalg.solve(S[np.ix_(F, F)], -S[np.ix_(F, D)] @ sys.gD)
    return sys.full(EF)


def block_real(sys):
    """Real 2x2 block system of eq. (4) on the free DoFs: [[K,-C],[C,K]] [Er;Ei] = [fr;fi]."""
    K = sys.K[sys.F][:, sys.F]
    C = sys.C[sys.F][:, sys.F]
    Ab = sp.bmat([[K, -C], [C, K]]).tocsr()
    f = sys.rhs_free()
    return Ab, np.concatenate([f.real, f.imag])


def relative_residual(sys, E):
    """||f_F - S_FF E_F|| / ||f_F|| for a full-length complex E (Dirichlet entries ignored)."""
    S = sys.S
    f = sys.rhs_free()
    r = f - S[sys.F][:, sys.F] @ E[sys.F]
    return np.linalg.norm(r) / np.linalg.norm(f)


def field_l2(sys, E, exact=None, q=None):
    """L2(Omega) norm of E_h - exact and of curl(E_h - exact), by Gauss quadrature.

    exact: callable x -> (E (npts,dim) complex, curlE (npts,ncurl) complex) or None.
    """
    mesh = sys.mesh
    d, p = mesh.dim, mesh.p
    if q is None:
        q = p + 4
    pts, w = fe.tensor_quad(d, q)
    vals, curls = fe.ref_eval(d, p, pts)
    h = mesh.h
    det = np.prod(h)
    pv = vals / h[None, :, None]
    pc = curls / det if d == 2 else curls * h[None, :, None] / det
    T = mesh.table()
    Ec = E[T]                                   # (nc, nl)
    Eh = np.einsum("cu,uaq->cqa", Ec, pv)       # (nc, nq, d)
    Ch = np.einsum("cu,uaq->cqa", Ec, pc)
    if exact is not None:
        origins = np.array([mesh.cell_origin(c) for c in range(mesh.n_cells)])
        X = origins[:, None, :] + pts[None, :, :] * h[None, None, :]
        Ex, Cx = exact(X.reshape(-1, d))
        Eh = Eh - Ex.reshape(Eh.shape)
        Ch = Ch - Cx.reshape(Ch.shape)
    e0 = np.sqrt(np.sum(np.abs(Eh) ** 2 * w[None, :, None]) * det)
    e1 = np.sqrt(np.sum(np.abs(Ch) ** 2 * w[None, :, None]) * det)
    return e0, e1
