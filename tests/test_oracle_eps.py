"""Pins of the oracle's relative permittivity eps (refractive index squared, the block
benchmark of Sec. 4.1), which enters only the mass term: curl(mu^{-1} curl E) - w^2 eps E = 0.

* Scaling invariance (exact): with a constant eps = n^2, the discrete system at
  (w, k, d) is K = A - w^2 n^2 M, C = k w M_inf, and the incident phase is w d.x. The
  eps = 1 system at (w n, k / n, d / n) has the same three quantities, so both give the
  same discrete solution. eps applied to A or to C instead, or squared or dropped, breaks
  the identity.
* eps = 1 given explicitly equals no eps (bitwise).
* DDM with a piecewise eps (the block benchmark's centre square): the interface fixed
  point equals the global LU solution, which checks that eps is cut per subdomain with the
  cells.
"""
import numpy as np
import pytest
from dataclasses import replace

import workloads
from oracle import ddm, system
from oracle.system import Problem


def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("dim,m,p", [(2, 6, 1), (2, 4, 2), (3, 3, 1)])
def test_constant_eps_is_a_scaling_of_omega_and_kappa(dim, m, p):
    n = 1.5
    th = 0.4
    d = (np.cos(th), np.sin(th), 0.2 if dim == 3 else 0.0)
    base = Problem(dim=dim, n=(m,) * dim + (1,) * (3 - dim), p=p, omega=4.0, kappa=1.3,
                   mu=np.random.default_rng(2).uniform(1, 2, m ** dim), inc_dir=d,
                   inc_pol=(-np.sin(th), np.cos(th), 0.1j if dim == 3 else 0.0))
    with_eps = replace(base, eps=np.full(m ** dim, n * n))
    scaled = replace(base, omega=base.omega * n, kappa=base.kappa / n, inc_dir=tuple(x / n for x in d))
    E1 = system.solve_lu(system.assemble(with_eps))
    E2 = system.solve_lu(system.assemble(scaled))
    # equal in exact arithmetic; w^2 n^2 and (w n)^2 (and k w, (k/n)(w n)) differ by
    # rounding, amplified by cond(S) (2e-12 measured in 3D)
    assert _rel(E1, E2) <= 1e-10
    # and it is a different problem from eps = 1 at the same w
    E0 = system.solve_lu(system.assemble(base))
    assert _rel(E1, E0) > 1e-2


def test_unit_eps_equals_no_eps():
    pr = Problem(**workloads.c1())
    s0 = system.assemble(pr)
    s1 = system.assemble(replace(pr, eps=np.ones(256)))
    assert (s0.K != s1.K).nnz == 0


@pytest.mark.parametrize("S", [(2, 2, 1), (4, 1, 1)])
def test_ddm_with_piecewise_eps_is_global_solution(S):
    d = workloads.block(m=8, omega=7.0)
    pr = Problem(**dict(d, subdomains=S))
    D = ddm.DDM(pr)
    E, it, _ = D.solve_gmres(rtol=1e-12)
    Eg = system.solve_lu(D.glob)
    assert _rel(E, Eg) <= 1e-9
    # the centre square changes the solution
    Ea = system.solve_lu(system.assemble(replace(pr, eps=None)))
    assert _rel(Eg, Ea) > 1e-2
