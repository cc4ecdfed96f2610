"""Impedance-transmission domain decomposition (oracle side).

Paper Sec. 3.1, eqs. (5)-(10).  Omega is split into a box grid of
non-overlapping subdomains Omega_i (eq. (5)); ids are 0-based, lexicographic with
x fastest.  Each subdomain solves eq. (7) with the transmission operator S = s 1,
a complex multiple of the identity (the paper's choice, eq. (10), is s = 1; the
problem's `transmission` field gives s).  Readings used here (the printed indices
of eqs. (6)-(8) are not consistent with each other):
 * subdomain i uses the data g_{j->i} coming from its neighbour j; its discrete
   matrix is S_i = K_i + i k w (M_inf,i + s sum_j M_Sigma_ij) (the transmission
   coefficient is k w, as on Gamma^inf, without mu); for complex s the term
   i k w s M_Sigma has the real part -k w Im(s) M_Sigma, which joins K_i;
 * data are dual vectors on the DoFs of the closure of Sigma_ij that are not
   Dirichlet: G_{j->i}[v] = int_Sigma g_{j->i} . g^T phi_v; they enter the
   right-hand side of subdomain i as -G_{j->i};
 * update (eq. (8)): G_{i->j} = -G_{j->i} - 2 i k w s M_Sigma_ij E_i; for any s != 0
   the fixed point is still the global solution (G_ij + G_ji = -2 i k w s M_Sigma E_i
   = -2 i k w s M_Sigma E_j forces continuity, and the summed subdomain rows lose their
   interface terms);
 * the initial solves use G = 0 (homogeneous impedance on interfaces);
 * eq. (9): G^{k+1} = A0 G^k + b with A0 the linear part and b the update from
   the incident data alone; solved by Jacobi (the paper's iteration) or by
   GMRES on (I - A0) G = b (the paper's alternative);
 * Dirichlet values in a subdomain are the global projection's values;
 * the glued field takes each shared DoF from the lowest subdomain id.
"""
from dataclasses import dataclass, replace

import numpy as np

from . import system
from .gmres import gmres as _gmres


@dataclass
class Interface:
    a: int            # lower subdomain id
    b: int            # upper subdomain id (a + step along axis)
    axis: int
    gdofs: np.ndarray          # global DoFs (sorted) carrying data
    la: np.ndarray             # their local indices in a
    lb: np.ndarray             # their local indices in b
    Ma: object                 # M_Sigma rows (interface DoFs) x local columns of a
    Mb: object


class DDM:
    def __init__(self, prob):
        self.prob = prob
        d = prob.dim
        S = tuple(int(s) for s in prob.subdomains[:d])
        n = prob.n[:d]
        for a in range(d):
            assert n[a] % S[a] == 0, "cells must divide evenly into subdomains"
        self.S = S
        self.glob = system.assemble(prob)
        gm = self.glob.mesh
        gT = gm.table()
        gD = dict(zip(self.glob.D.tolist(), self.glob.gD.tolist()))
        self.gDset = set(self.glob.D.tolist())
        nloc = [n[a] // S[a] for a in range(d)]
        self.subs = []
        nsub = int(np.prod(S))
        self.s = complex(prob.transmission)
        assert self.s != 0
        kw = prob.kappa * prob.omega
        mu_g = prob.mu_cells(gm.n_cells).reshape(tuple(reversed(n)))
        eps_g = prob.eps_cells(gm.n_cells).reshape(tuple(reversed(n)))
        for s in range(nsub):
            pos = self.sub_pos(s)
            lo = [gm.lo[a] + pos[a] * nloc[a] * gm.h[a] for a in range(d)]
            hi = [lo[a] + nloc[a] * gm.h[a] for a in range(d)]
            inc = 0
            for a in range(d):
                if pos[a] == 0 and (prob.inc_faces >> (2 * a)) & 1:
                    inc |= 1 << (2 * a)
                if pos[a] == S[a] - 1 and (prob.inc_faces >> (2 * a + 1)) & 1:
                    inc |= 1 << (2 * a + 1)
            sl = tuple(slice(pos[a] * nloc[a], (pos[a] + 1) * nloc[a]) for a in reversed(range(d)))
            mu_l = mu_g[sl].ravel()
            lp = replace(prob, n=tuple(nloc) + (1,) * (3 - d), lo=tuple(lo) + (0.0,) * (3 - d),
                         hi=tuple(hi) + (1.0,) * (3 - d), inc_faces=inc, mu=mu_l,
                         eps=eps_g[sl].ravel(), subdomains=(1, 1, 1))
            ls = system.assemble(lp)
            if self.s != 1:
                # interface sides carry k w s M_Sigma instead of the k w M_Sigma of an impedance side
                Mi = None
                for a in range(d):
                    for side, inner in ((0, pos[a] > 0), (1, pos[a] < S[a] - 1)):
                        if inner:
                            m_ = system.side_matrix(ls.mesh, a, side)
                            Mi = m_ if Mi is None else Mi + m_
                if Mi is not None:
                    ls.K = (ls.K - kw * self.s.imag * Mi).tocsr()
                    ls.C = (ls.C + kw * (self.s.real - 1.0) * Mi).tocsr()
            # local -> global DoF map through the shared local cell ordering
            lm = ls.mesh
            l2g = np.full(lm.n_dofs, -1, dtype=np.int64)
            lT = lm.table()
            for c in range(lm.n_cells):
                ci = lm.cell_index(c)
                gi = [ci[a] + pos[a] * nloc[a] for a in range(d)]
                if d == 2:
                    gc = gi[1] * n[0] + gi[0]
                else:
                    gc = (gi[2] * n[1] + gi[1]) * n[0] + gi[0]
                l2g[lT[c]] = gT[gc]
            assert (l2g >= 0).all()
            ls.gD = np.array([gD[g] for g in l2g[ls.D]], dtype=np.complex128)
            ls.extra["l2g"] = l2g
            ls.extra["lu"] = system.lu_factor(ls)
            self.subs.append(ls)
        self.ifaces = []
        for s in range(nsub):
            pos = self.sub_pos(s)
            for a in range(d):
                if pos[a] + 1 < S[a]:
                    pt = list(pos)
                    pt[a] += 1
                    t = self.sub_id(pt)
                    self.ifaces.append(self._make_iface(s, t, a))
        self.kw = prob.kappa * prob.omega

    def sub_pos(self, s):
        S = self.S
        if len(S) == 2:
            return (s % S[0], s // S[0])
        return (s % S[0], (s // S[0]) % S[1], s // (S[0] * S[1]))

    def sub_id(self, pos):
        S = self.S
        if len(S) == 2:
            return pos[1] * S[0] + pos[0]
        return (pos[2] * S[1] + pos[1]) * S[0] + pos[0]

    def _make_iface(self, s, t, axis):
        A, B = self.subs[s], self.subs[t]
        ga = A.extra["l2g"][A.mesh.side_dofs(axis, 1)]
        gb = B.extra["l2g"][B.mesh.side_dofs(axis, 0)]
        g = np.array(sorted(set(ga.tolist()) - self.gDset), dtype=np.int64)
        assert set(g.tolist()) <= set(gb.tolist())
        inv_a = {v: i for i, v in enumerate(A.extra["l2g"].tolist())}
        inv_b = {v: i for i, v in enumerate(B.extra["l2g"].tolist())}
        la = np.array([inv_a[v] for v in g], dtype=np.int64)
        lb = np.array([inv_b[v] for v in g], dtype=np.int64)
        Ma = system.side_matrix(A.mesh, axis, 1)[la]
        Mb = system.side_matrix(B.mesh, axis, 0)[lb]
        return Interface(s, t, axis, g, la, lb, Ma, Mb)

    # ---------------------------------------------------------------- data layout
    def zero_data(self):
        """Directed data: list over interfaces of (G_{a->b}, G_{b->a})."""
        return [(np.zeros(len(f.gdofs), np.complex128), np.zeros(len(f.gdofs), np.complex128))
                for f in self.ifaces]

    def pack(self, G):
        return np.concatenate([np.concatenate(x) for x in G]) if G else np.zeros(0, np.complex128)

    def unpack(self, v):
        out, o = [], 0
        for f in self.ifaces:
            m = len(f.gdofs)
            out.append((v[o:o + m].copy(), v[o + m:o + 2 * m].copy()))
            o += 2 * m
        return out

    # ---------------------------------------------------------------- one sweep
    def solve_subdomains(self, G, incident=True):
        """E_i for all subdomains given the incoming data (eq. (7))."""
        Es = []
        for s, ls in enumerate(self.subs):
            rhs = np.zeros(ls.mesh.n_dofs, dtype=np.complex128)
            for f, (gab, gba) in zip(self.ifaces, G):
                if f.a == s:
                    rhs[f.la] -= gba      # data from b into a
                elif f.b == s:
                    rhs[f.lb] -= gab
            rF = rhs[ls.F]
            if incident and len(ls.D):
                rF = rF + ls.rhs_free()
            EF = ls.extra["lu"](rF)
            E = np.zeros(ls.mesh.n_dofs, dtype=np.complex128)
            E[ls.F] = EF
            if incident:
                E[ls.D] = ls.gD
            Es.append(E)
        return Es

    def update(self, G, Es):
        """Eq. (8) with S = s 1 in dual form."""
        out = []
        c = 2j * self.kw * self.s
        for f, (gab, gba) in zip(self.ifaces, G):
            nab = -gba - c * (f.Ma @ Es[f.a])
            nba = -gab - c * (f.Mb @ Es[f.b])
            out.append((nab, nba))
        return out

    def glue(self, Es):
        E = np.zeros(self.glob.n, dtype=np.complex128)
        for s in reversed(range(len(self.subs))):
            E[self.subs[s].extra["l2g"]] = Es[s]
        return E

    # ---------------------------------------------------------------- outer solvers
    def jacobi(self, iters):
        """G^0 = 0, then `iters` sweeps; returns the glued E after each sweep."""
        G = self.zero_data()
        out = []
        for _ in range(iters):
            Es = self.solve_subdomains(G, incident=True)
            out.append(self.glue(Es))
            G = self.update(G, Es)
        return out, G

    def interface_rhs(self):
        G0 = self.zero_data()
        return self.pack(self.update(G0, self.solve_subdomains(G0, incident=True)))

    def apply_I_minus_A0(self, v):
        G = self.unpack(v)
        AG = self.update(G, self.solve_subdomains(G, incident=False))
        return v - self.pack(AG)

    def solve_gmres(self, rtol=1e-10, restart=100, max_iter=2000):
        b = self.interface_rhs()
        g, it, hist = _gmres(self.apply_I_minus_A0, b, rtol=rtol, restart=restart, max_iter=max_iter)
        G = self.unpack(g)
        E = self.glue(self.solve_subdomains(G, incident=True))
        return E, it, hist
