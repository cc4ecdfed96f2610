"""Pins of the oracle's GMRES, domain decomposition and adjoint.

* GMRES (Sec. 3.2): with the exact block preconditioner diag(K, K)^{-1} of
  eq. (11), P^{-1} A - I has rank <= 2 rank(C), so unrestarted GMRES terminates
  within 2 rank(C) + 1 steps; its result equals the LU solution.
* DDM (eqs. (5)-(10)): the fixed point of the interface iteration is the global
  discrete solution (dual-vector argument: G_ij + G_ji = -2 i k w M_Sigma E_i =
  -2 i k w M_Sigma E_j forces continuity, and the summed subdomain rows are the
  assembled global rows); a 1x1 partition is the single-domain solve; Jacobi
  sweeps on the waveguide contract.
* adjoint: central finite differences of J (fresh LU per evaluation).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads
from oracle import adjoint, closed_form, ddm, gmres, system
from oracle.system import Problem


def _precond(s):
    K = s.K[s.F][:, s.F].tocsc()
    lu = spla.splu(K)
    return lambda v: lu.solve(np.ascontiguousarray(v.real)) + 1j * lu.solve(np.ascontiguousarray(v.imag))


def test_gmres_exact_block_preconditioner_terminates_and_matches_lu():
    pr = Problem(**workloads.c1())
    s = system.assemble(pr)
    S = s.S[s.F][:, s.F]
    f = s.rhs_free()
    rankC = np.linalg.matrix_rank(s.C[s.F][:, s.F].toarray())
    x, it, hist = gmres.gmres(lambda v: S @ v, f, _precond(s), rtol=1e-13, restart=1000, max_iter=1000)
    assert it <= 2 * rankC + 1
    E = system.solve_lu(s)
    assert np.linalg.norm(x - E[s.F]) <= 1e-10 * np.linalg.norm(E[s.F])


def test_gmres_restarted_plain_real_system():
    rng = np.random.default_rng(0)
    A = np.eye(60) * 4 + rng.standard_normal((60, 60)) * 0.3
    b = rng.standard_normal(60)
    x, it, _ = gmres.gmres(lambda v: A @ v, b, rtol=1e-12, restart=7, max_iter=500)
    assert np.linalg.norm(A @ x - b) <= 1e-11 * np.linalg.norm(b)


@pytest.mark.parametrize("dim,m,p,S", [(2, 8, 0, (2, 2, 1)), (2, 8, 1, (2, 1, 1)), (2, 12, 1, (3, 2, 1)),
                                       (3, 4, 0, (2, 2, 2)), (3, 4, 1, (2, 1, 1))])
def test_ddm_fixed_point_is_global_solution(dim, m, p, S):
    th = 0.3
    pr = Problem(dim=dim, n=(m,) * dim + (1,) * (3 - dim), p=p, omega=6.0,
                 mu=np.random.default_rng(1).uniform(1, 2, m ** dim),
                 inc_dir=(np.cos(th), np.sin(th), 0.0), inc_pol=(-np.sin(th), np.cos(th), 0.0),
                 subdomains=S)
    D = ddm.DDM(pr)
    E, it, _ = D.solve_gmres(rtol=1e-12)
    Eg = system.solve_lu(D.glob)
    assert np.linalg.norm(E - Eg) <= 1e-9 * np.linalg.norm(Eg)


@pytest.mark.parametrize("dim,m,p,S,ts", [(2, 8, 1, (2, 2, 1), 0.6 + 0.8j), (2, 8, 0, (2, 1, 1), 2.0),
                                          (3, 4, 1, (2, 1, 1), 1.5 - 0.5j)])
def test_ddm_fixed_point_with_scaled_transmission(dim, m, p, S, ts):
    """S = s 1 on the interfaces (eq. (7)-(8) with a complex scalar s instead of the paper's 1):
    the interface iteration changes -- its first Jacobi iterate differs from the s = 1 one --
    but its fixed point is the same global discrete solution."""
    th = 0.3
    base = dict(dim=dim, n=(m,) * dim + (1,) * (3 - dim), p=p, omega=6.0,
                mu=np.random.default_rng(2).uniform(1, 2, m ** dim),
                inc_dir=(np.cos(th), np.sin(th), 0.0), inc_pol=(-np.sin(th), np.cos(th), 0.0), subdomains=S)
    D = ddm.DDM(Problem(**base, transmission=ts))
    E, it, _ = D.solve_gmres(rtol=1e-12)
    Eg = system.solve_lu(D.glob)
    assert np.linalg.norm(E - Eg) <= 1e-9 * np.linalg.norm(Eg)
    D1 = ddm.DDM(Problem(**base))
    J1, _ = D1.jacobi(2)
    Js, _ = D.jacobi(2)
    assert np.linalg.norm(J1[1] - Js[1]) > 1e-3 * np.linalg.norm(Eg)


def test_ddm_single_subdomain_is_single_domain_solve():
    pr = Problem(**workloads.c1())
    D = ddm.DDM(pr)
    Es, _ = D.jacobi(1)
    Eg = system.solve_lu(D.glob)
    assert np.linalg.norm(Es[0] - Eg) <= 1e-12 * np.linalg.norm(Eg)


def test_ddm_jacobi_contracts_on_waveguide_split():
    pr = Problem(dim=2, n=(16, 8, 1), p=1, omega=10.0, inc_faces=closed_form.WAVEGUIDE_INC_2D,
                 subdomains=(2, 1, 1))
    D = ddm.DDM(pr)
    Es, _ = D.jacobi(6)
    Eg = system.solve_lu(D.glob)
    err = [np.linalg.norm(e - Eg) / np.linalg.norm(Eg) for e in Es]
    assert all(b < a for a, b in zip(err, err[1:]))
    assert err[-1] < 1e-3 * err[0]


def test_adjoint_gradient_matches_central_differences():
    pr = Problem(**workloads.c5(16))
    s = system.assemble(pr)
    E = system.solve_lu(s)
    lo, hi = workloads.C5_TARGET
    MT = adjoint.target_mass(s, lo, hi)
    g, _ = adjoint.gradient(s, E, MT)
    cells = workloads.fd_cells(s.mesh.n_cells, 12)
    fd = adjoint.fd_gradient(pr, cells, lo, hi)
    rel = np.abs(g[cells] - fd) / np.maximum(np.abs(fd), 1e-3 * np.abs(fd).max())
    assert rel.max() <= 1e-6


def test_target_mass_is_exact_area():
    """M_T on the constant field (1, 0): E^T M_T E = |T n Omega| (clipped cells)."""
    pr = Problem(dim=2, n=(10, 10, 1), p=1, omega=1.0)
    s = system.assemble(pr)
    E = np.zeros(s.n)
    mesh = s.mesh
    for i in range(10):
        for j in range(11):
            E[mesh.edge_dofs(0, mesh.edge_id(0, i, j))[0]] = 0.1
    MT = adjoint.target_mass(s, (0.23, 0.41), (0.67, 0.88))
    assert abs(E @ MT @ E - 0.44 * 0.47) < 1e-14
